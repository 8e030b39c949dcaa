// Internal device-side layout of the ESES hot path (gfx950).
//
// Atoms are re-ordered by a uniform cell list (cell edge 2 * s_max, so SAS
// neighbours lie in the 3x3x3 stencil) and renumbered; every per-atom,
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

// Device view of one molecule.  Plain pointers and scalars, passed by value.
struct Mol {
    int n;              // atoms
    double rho, h;
    double lo[3];
    int dims[3];
    long long npts;
    // cell list over the atom box
    double cell;         // cell edge (2 * s_max)
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

    int *diag;           // [4] diagnostics: [0] fill-pass overflows, [1] FP32 points
                         // re-tested in FP64, [2] shared centres, [3] crossing
                         // edges whose walk found no owning surface
    double cmag;         // max |coordinate| of any centre, plus s_max: the scale of
                         // the rounding error of positions derived from centres
    // points whose FP64 decision could not be certified (re-decided exactly
    // on the host): grid indices, their count (may exceed the capacity)
    long long *unc_idx;
    int *unc_n;
    int unc_cap;

    const double *in_c;  // caller centres [n][3]
    const double *in_r;  // caller radii [n]

    double4 *atom;       // internal order: x, y, z, r
    int *orig;           // internal id -> caller id
    int *cell_start;     // [ncell + 1]

    int *nbr_off;        // [n + 1]
    int *nbr;            // internal ids, ascending per atom
    int *nbr_cov;        // the same lists, largest cap cut from S_i first
    int *circ_any;       // [n] circles on S_i (either owner)
    uint32_t *aflag;     // [n]

    int ncirc;
    int *circ_off;       // [n + 1] circles owned by atom i (partner > i)
    int *circ_i;         // [ncirc] owner
    int *circ_j;         // [ncirc] partner, ascending per owner
    double4 *circ_oR;    // [ncirc] centre o, radius R
    double4 *circ_n;     // [ncirc] unit axis n (owner -> partner); w: a bound on the
                         // rounding error of o's components and of R
    uint32_t *cflag;     // [ncirc]

    int nvert;
    int *vert_off;       // [ncirc + 1]
    double4 *vert_p;     // [nvert] position; w: a bound on its rounding error
    int4 *vert_ijks;     // [nvert] internal i < j < k, sign (+1/-1, internal order)
    int *vert_off_atom;  // [n + 1]

    int nface;
    int *face_off_atom;  // [n + 1]
    int *face_atom;      // [nface]
    int *face_cut_off;   // [nface + 1]
    double4 *face_cut;   // (c_k - c_i, tau_ik), tau = (s_i^2 + d^2 - s_k^2) / (2 s_i)

    int nec;
    int *ec_off_atom;    // [n + 1]
    int *ec_circ;        // [nec] circle id
    int *ec_cut_off;     // [nec + 1]
    double4 *ec_cut;     // (u_perp, T_k), u_perp = in-plane part of c_k - o,
                         // T_k = (R^2 + |o - c_k|^2 - s_k^2) / (2 R)

    // per-tile candidate lists (CSR over tiles)
    int *tA_off, *tA;    // atoms whose SAS ball reaches the tile box
    int *tF_off, *tF;    // exposed faces within s_i + rho
    int *tC_off, *tC;    // exposed circles within rho
    int *tV_off, *tV;    // exposed vertices within rho
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
