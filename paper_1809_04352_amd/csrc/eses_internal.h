// Internal device-side layout of the ESES hot path (gfx950).
//
// Atoms are re-ordered by a uniform cell list (cell edge s_max, so SAS
// neighbours lie in the 5x5x5 stencil) and renumbered; every per-atom,
// per-circle and per-vertex array below uses these internal ids, which keeps
// the candidates of one cell contiguous in memory.  Circles and concave probe
// positions are owned by their lowest internal atom id, so the features of a
// cell are a contiguous range too.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace eses {

// Atom flags.
constexpr uint32_t AF_EXPOSED_VERTEX = 1u;   // an admissible three-sphere point lies on S_i
constexpr uint32_t AF_EXPOSED_CIRCLE = 2u;   // a crossing-free circle on S_i is admissible
constexpr uint32_t AF_CONTAINED = 4u;        // S_i lies strictly inside another SAS ball
constexpr uint32_t AF_FACE = 8u;             // S_i may hold an admissible point

// Circle flags.
constexpr uint32_t CF_CROSSED = 1u;          // another sphere cuts the circle at two points
constexpr uint32_t CF_EXPOSED_VERTEX = 2u;   // an admissible three-sphere point lies on it
constexpr uint32_t CF_EXPOSED_FREE = 4u;     // crossing-free and admissible
constexpr uint32_t CF_EXPOSED = CF_EXPOSED_VERTEX | CF_EXPOSED_FREE;

// Lists are built with a small positive slack on every distance threshold, so
// a candidate that rounding would put just outside a reach is still listed;
// listing too much never changes a result, only the decisions below do.
constexpr double LIST_SLACK = 1e-7;

// Pointers into device memory.  In device code they carry the global address
// space, so that loads through them are global loads, which the compiler may
// reorder with LDS accesses and which do not wait on the LDS counter, rather
// than generic (flat) ones, which may alias LDS.  Host code sees plain
// pointers (the layout is the same).
#if defined(__HIP_DEVICE_COMPILE__)
#define GMEM __attribute__((address_space(1)))
#else
#define GMEM
#endif

// A device address stored into such a field from host code: dev(p).
template <typename T>
struct DevAddr {
    T *p;
    template <typename U>
    operator U *() const { return (U *)p; }
};
template <typename T>
inline DevAddr<T> dev(T *p) { return DevAddr<T>{p}; }

// Device view of one molecule.  Plain pointers and scalars, passed by value.
struct Mol {
    int n;              // atoms
    double rho, h;
    double lo[3];
    int dims[3];
    long long npts;
    // cell list over the atom box
    double cell;         // cell edge (s_max plus the list slack, or more for sparse input)
    double smax;
    double clo[3];
    int nc[3];
    int ncell;
    // tiles
    int tile;
    int force_recheck;   // FP32 path: every phase-1 decision treated as uncertain
    int edge_fallback;   // every crossing edge through the wavefront root kernel
    int tdims[3];
    int ntiles;
    int kz0;             // z index of plane 0 in the molecule's whole grid: 0, or the
                         // first plane of a slab view (out-of-core form)

    GMEM int *diag;           // [4] diagnostics: [0] fill-pass overflows, [1] FP32 points
                         // re-tested in FP64, [2] shared centres, [3] crossing
                         // edges whose walk found no owning surface
    double cmag;         // max |coordinate| of any centre, plus s_max: the scale of
                         // the rounding error of positions derived from centres
    // points whose FP64 decision could not be certified (re-decided exactly
    // on the host): grid indices, their count (may exceed the capacity)
    GMEM long long *unc_idx;
    GMEM int *unc_n;
    int unc_cap;

    GMEM const double *in_c;  // caller centres [n][3]
    GMEM const double *in_r;  // caller radii [n]

    GMEM double4 *atom;       // internal order: x, y, z, r
    GMEM int *orig;           // internal id -> caller id
    GMEM int *cell_start;     // [ncell + 1]

    GMEM int *nbr_off;        // [n + 1]
    GMEM int *nbr;            // internal ids, ascending per atom
    GMEM int *nbr_cov;        // the same lists, largest cap cut from S_i first
    GMEM int *circ_any;       // [n] circles on S_i (either owner)
    GMEM uint32_t *aflag;     // [n]

    int ncirc;
    GMEM int *circ_off;       // [n + 1] circles owned by atom i (partner > i)
    GMEM int *circ_i;         // [ncirc] owner
    GMEM int *circ_j;         // [ncirc] partner, ascending per owner
    GMEM double4 *circ_oR;    // [ncirc] centre o, radius R
    GMEM double4 *circ_n;     // [ncirc] unit axis n (owner -> partner); w: a bound on the
                         // rounding error of o's components and of R
    GMEM uint32_t *cflag;     // [ncirc]

    int nvert;
    GMEM int *vert_off;       // [ncirc + 1]
    GMEM double4 *vert_p;     // [nvert] position; w: a bound on its rounding error
    GMEM int4 *vert_ijks;     // [nvert] internal i < j < k, sign (+1/-1, internal order)
    GMEM int *vert_off_atom;  // [n + 1]

    int nface;
    GMEM int *face_off_atom;  // [n + 1]
    GMEM int *face_atom;      // [nface]
    GMEM int *face_cut_off;   // [nface + 1]
    GMEM double4 *face_cut;   // (c_k - c_i, tau_ik), tau = (s_i^2 + d^2 - s_k^2) / (2 s_i)

    int nec;
    GMEM int *ec_off_atom;    // [n + 1]
    GMEM int *ec_circ;        // [nec] circle id
    GMEM int *ec_cut_off;     // [nec + 1]
    GMEM double4 *ec_cut;     // (u_perp, T_k), u_perp = in-plane part of c_k - o,
                         // T_k = (R^2 + |o - c_k|^2 - s_k^2) / (2 R)

    // per-tile candidate lists (CSR over tiles)
    GMEM int *tA_off, *tA;    // atoms whose SAS ball reaches the tile box
    GMEM int *tF_off, *tF;    // exposed faces within s_i + rho
    GMEM int *tC_off, *tC;    // exposed circles within rho
    GMEM int *tV_off, *tV;    // exposed vertices within rho
};

// Grid point coordinate fl(lo + fl(i h)): two correctly rounded operations,
// never contracted into a fused multiply-add.
__device__ inline double grid_coord(double lo, double h, long long i) {
    return __dadd_rn(lo, __dmul_rn((double)i, h));
}

// Coordinate of grid index i along axis a of molecule view m (a slab view
// starts at plane kz0 of the whole grid, so its points keep their coordinates).
__device__ inline double mol_coord(const Mol &m, int a, long long i) {
    return grid_coord(m.lo[a], m.h, a == 2 ? i + m.kz0 : i);
}

}  // namespace eses
