// Device helpers shared by the ESES kernels: wavefront prefix/ballot
// primitives, box distances, the pair-circle construction, and the FP64
// inside/outside test of one point against a tile's candidate lists.
#pragma once

#include "eses_internal.h"

namespace eses {

constexpr int WAVE = 64;

__device__ inline int lane_id() { return __lane_id(); }

// Number of set lanes below this lane in a 64-bit ballot mask.
__device__ inline int mask_prefix(unsigned long long m) {
    return __popcll(m & ((1ull << lane_id()) - 1ull));
}

// Visibility of LDS writes of a wavefront to its other lanes.
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Inclusive prefix sum across a wavefront.
template <typename T>
__device__ inline T wave_incl_scan(T v) {
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        T t = __shfl_up(v, d, WAVE);
        if (lane >= d) v += t;
    }
    return v;
}

// Exclusive prefix sum across a block of BLOCK threads (multiple of 64);
// returns the prefix and writes the block total.  Uses `lds` of BLOCK/64 slots.
template <typename T, int BLOCK>
__device__ inline T block_excl_scan(T v, T *lds, T *total) {
    constexpr int NW = BLOCK / WAVE;
    const int w = threadIdx.x / WAVE;
    const int lane = lane_id();
    T inc = wave_incl_scan(v);
    if (lane == WAVE - 1) lds[w] = inc;
    __syncthreads();
    if (w == 0) {
        T s = lane < NW ? lds[lane] : T(0);
        T si = wave_incl_scan(s);
        if (lane < NW) lds[lane] = si - s;
        if (lane == NW - 1) lds[NW] = si;
    }
    __syncthreads();
    T res = lds[w] + inc - v;
    *total = lds[NW];
    __syncthreads();
    return res;
}

__device__ inline double sq(double a) { return a * a; }

// Squared distance from point p to the axis-aligned box [lo, hi].
__device__ inline double box_dist2(const double lo[3], const double hi[3], double px, double py,
                                   double pz) {
    double dx = fmax(0.0, fmax(lo[0] - px, px - hi[0]));
    double dy = fmax(0.0, fmax(lo[1] - py, py - hi[1]));
    double dz = fmax(0.0, fmax(lo[2] - pz, pz - hi[2]));
    return dx * dx + dy * dy + dz * dz;
}

// Circle where SAS spheres of atoms a (owner) and b meet.  Exists iff
// |s_a - s_b| < d < s_a + s_b; centre o = c_a + t n with
// t = (s_a^2 - s_b^2 + d^2) / (2 d), n the unit vector c_a -> c_b, radius
// R = sqrt(s_a^2 - t^2).  Both build passes call this, so their decisions agree.
__device__ inline bool pair_circle(double4 a, double4 b, double rho, double4 &oR, double4 &nn) {
    double vx = b.x - a.x, vy = b.y - a.y, vz = b.z - a.z;
    double d2 = vx * vx + vy * vy + vz * vz;
    double d = sqrt(d2);
    double sa = a.w + rho, sb = b.w + rho;
    if (!(d < sa + sb) || !(d > fabs(sa - sb))) return false;
    double t = (sa * sa - sb * sb + d2) / (2.0 * d);
    double R2 = sa * sa - t * t;
    if (!(R2 > 0.0)) return false;
    double inv = 1.0 / d;
    nn = make_double4(vx * inv, vy * inv, vz * inv, 0.0);
    oR = make_double4(a.x + t * nn.x, a.y + t * nn.y, a.z + t * nn.z, sqrt(R2));
    return true;
}

// A unit vector perpendicular to n (used only when a point sits on a circle's
// axis, where every circle point is equally near).
__device__ inline void perp_unit(double nx, double ny, double nz, double &ux, double &uy,
                                 double &uz) {
    double ax = fabs(nx), ay = fabs(ny), az = fabs(nz);
    double ex = 0, ey = 0, ez = 0;
    if (ax <= ay && ax <= az) ex = 1;
    else if (ay <= az) ey = 1;
    else ez = 1;
    double dn = ex * nx + ey * ny + ez * nz;
    ux = ex - dn * nx;
    uy = ey - dn * ny;
    uz = ez - dn * nz;
    double l = sqrt(ux * ux + uy * uy + uz * uz);
    ux /= l;
    uy /= l;
    uz /= l;
}

// Work counters of one classification (for the statistics pass only).
enum WorkCounter {
    WC_ATOM = 0,     // point-atom tests (van der Waals / SAS ball)
    WC_VERTEX,       // point-probe tests
    WC_FACE,         // face reach tests
    WC_FACE_CUT,     // face admissibility half-space tests
    WC_CIRCLE,       // circle reach tests
    WC_CIRCLE_CUT,   // circle admissibility half-space tests
    WC_CASE_SHELL,   // points decided by case 3
    WC_COUNT
};

// Inside/outside of point x (eq. 2) in FP64 against the candidate lists of
// `tile` (which cover every atom and exposed feature that can decide any
// point of the tile box).  Three cases:
//   1. x in a closed van der Waals ball                  -> inside;
//   2. x outside every open SAS ball (x is itself in A)  -> outside;
//   3. otherwise outside iff an admissible candidate -- an exposed
//      three-sphere point, the radial projection onto an exposed face, or the
//      nearest point of an exposed circle -- lies closer than rho.
// Face admissibility against neighbour k reduces to
//   (x - c_i) . (c_k - c_i) <= |x - c_i| tau_ik,
// circle admissibility to  w_perp . u_k <= |w_perp| T_k  (w = x - o).
// With CNT the tests performed are tallied in cnt[WC_COUNT].
template <bool CNT>
__device__ inline int label_fp64_t(const Mol &m, int tile, double x, double y, double z,
                                   unsigned long long *cnt) {
    const double rho = m.rho;
    const double rho2 = rho * rho;
    bool inU = false;
    for (int q = m.tA_off[tile], e = m.tA_off[tile + 1]; q < e; ++q) {
        double4 a = m.atom[m.tA[q]];
        double dx = x - a.x, dy = y - a.y, dz = z - a.z;
        double d2 = dx * dx + dy * dy + dz * dz;
        if (CNT) ++cnt[WC_ATOM];
        if (d2 <= a.w * a.w) return 1;
        double s = a.w + rho;
        inU |= d2 < s * s;
    }
    if (!inU) return 0;
    if (CNT) ++cnt[WC_CASE_SHELL];
    for (int q = m.tV_off[tile], e = m.tV_off[tile + 1]; q < e; ++q) {
        double4 p = m.vert_p[m.tV[q]];
        double dx = x - p.x, dy = y - p.y, dz = z - p.z;
        if (CNT) ++cnt[WC_VERTEX];
        if (dx * dx + dy * dy + dz * dz < rho2) return 0;
    }
    for (int q = m.tF_off[tile], e = m.tF_off[tile + 1]; q < e; ++q) {
        int f = m.tF[q];
        double4 a = m.atom[m.face_atom[f]];
        double dx = x - a.x, dy = y - a.y, dz = z - a.z;
        double d2 = dx * dx + dy * dy + dz * dz;
        double sr = a.w + 2.0 * rho;
        if (CNT) ++cnt[WC_FACE];
        if (!(d2 < sr * sr)) continue;
        double d = sqrt(d2);
        bool ok = true;
        for (int c = m.face_cut_off[f], ce = m.face_cut_off[f + 1]; c < ce; ++c) {
            double4 v = m.face_cut[c];
            if (CNT) ++cnt[WC_FACE_CUT];
            if (dx * v.x + dy * v.y + dz * v.z > d * v.w) {
                ok = false;
                break;
            }
        }
        if (ok) return 0;
    }
    for (int q = m.tC_off[tile], e = m.tC_off[tile + 1]; q < e; ++q) {
        int ec = m.tC[q];
        int ci = m.ec_circ[ec];
        double4 oR = m.circ_oR[ci];
        double4 n = m.circ_n[ci];
        double wx = x - oR.x, wy = y - oR.y, wz = z - oR.z;
        double t = wx * n.x + wy * n.y + wz * n.z;
        double ww = wx * wx + wy * wy + wz * wz;
        double b = sqrt(fmax(ww - t * t, 0.0));
        double R = oR.w;
        if (CNT) ++cnt[WC_CIRCLE];
        if (!(ww + R * R - rho2 < 2.0 * b * R)) continue;
        double px = wx, py = wy, pz = wz, pb = b;
        if (!(b > 0.0)) {
            perp_unit(n.x, n.y, n.z, px, py, pz);
            pb = 1.0;
        }
        bool ok = true;
        for (int c = m.ec_cut_off[ec], ce = m.ec_cut_off[ec + 1]; c < ce; ++c) {
            double4 u = m.ec_cut[c];
            if (CNT) ++cnt[WC_CIRCLE_CUT];
            if (px * u.x + py * u.y + pz * u.z > pb * u.w) {
                ok = false;
                break;
            }
        }
        if (ok) return 0;
    }
    return 1;
}

__device__ inline int label_fp64(const Mol &m, int tile, double x, double y, double z) {
    return label_fp64_t<false>(m, tile, x, y, z, nullptr);
}

// Case 3 only (x inside some SAS ball and in no van der Waals ball): outside
// iff an admissible candidate lies closer than rho.
__device__ inline int shell_label_fp64(const Mol &m, int tile, double x, double y, double z) {
    const double rho = m.rho;
    const double rho2 = rho * rho;
    for (int q = m.tV_off[tile], e = m.tV_off[tile + 1]; q < e; ++q) {
        double4 p = m.vert_p[m.tV[q]];
        double dx = x - p.x, dy = y - p.y, dz = z - p.z;
        if (dx * dx + dy * dy + dz * dz < rho2) return 0;
    }
    for (int q = m.tF_off[tile], e = m.tF_off[tile + 1]; q < e; ++q) {
        int f = m.tF[q];
        double4 a = m.atom[m.face_atom[f]];
        double dx = x - a.x, dy = y - a.y, dz = z - a.z;
        double d2 = dx * dx + dy * dy + dz * dz;
        double sr = a.w + 2.0 * rho;
        if (!(d2 < sr * sr)) continue;
        double d = sqrt(d2);
        bool ok = true;
        for (int c = m.face_cut_off[f], ce = m.face_cut_off[f + 1]; c < ce; ++c) {
            double4 v = m.face_cut[c];
            if (dx * v.x + dy * v.y + dz * v.z > d * v.w) {
                ok = false;
                break;
            }
        }
        if (ok) return 0;
    }
    for (int q = m.tC_off[tile], e = m.tC_off[tile + 1]; q < e; ++q) {
        int ec = m.tC[q];
        int ci = m.ec_circ[ec];
        double4 oR = m.circ_oR[ci];
        double4 n = m.circ_n[ci];
        double wx = x - oR.x, wy = y - oR.y, wz = z - oR.z;
        double t = wx * n.x + wy * n.y + wz * n.z;
        double ww = wx * wx + wy * wy + wz * wz;
        double b = sqrt(fmax(ww - t * t, 0.0));
        double R = oR.w;
        if (!(ww + R * R - rho2 < 2.0 * b * R)) continue;
        double px = wx, py = wy, pz = wz, pb = b;
        if (!(b > 0.0)) {
            perp_unit(n.x, n.y, n.z, px, py, pz);
            pb = 1.0;
        }
        bool ok = true;
        for (int c = m.ec_cut_off[ec], ce = m.ec_cut_off[ec + 1]; c < ce; ++c) {
            double4 u = m.ec_cut[c];
            if (px * u.x + py * u.y + pz * u.z > pb * u.w) {
                ok = false;
                break;
            }
        }
        if (ok) return 0;
    }
    return 1;
}

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  Map block b to tile (b % 8) * per + b / 8 so each XCD walks a
// contiguous run of tiles and neighbouring tiles share its L2.  `nblocks`
// is a multiple of 8; blocks past `ntiles` return -1.
constexpr int NXCD = 8;

__device__ inline int xcd_tile(int b, int nblocks, int ntiles) {
    int per = nblocks / NXCD;
    int t = (b % NXCD) * per + b / NXCD;
    return t < ntiles ? t : -1;
}

// Grid indices (i, j, k) of point index idx (x fastest): 32-bit divisions
// while idx fits, which is every grid below 2^31 points.
__device__ inline void grid_ijk(long long idx, int nx, int ny, int &i, int &j, int &k) {
    if (idx < (1LL << 31)) {
        const unsigned u = (unsigned)idx, q = u / (unsigned)nx;
        i = (int)(u - q * (unsigned)nx);
        j = (int)(q % (unsigned)ny);
        k = (int)(q / (unsigned)ny);
    } else {
        const long long q = idx / nx;
        i = (int)(idx - q * nx);
        j = (int)(q % ny);
        k = (int)(q / ny);
    }
}

// A molecule's view from a device array at a workgroup-uniform index, copied
// word by word into uniform registers: read through the pointer, every field
// would be a vector load (the kernels' stores might alias it) and hold VGPRs.
__device__ inline Mol uniform_mol(const Mol *mols, int q) {
    static_assert(sizeof(Mol) % 4 == 0, "Mol is copied in 32-bit words");
    Mol r;
    const int *src = (const int *)(mols + q);
    int *dst = (int *)&r;
#pragma unroll
    for (int i = 0; i < (int)(sizeof(Mol) / 4); ++i) dst[i] = __builtin_amdgcn_readfirstlane(src[i]);
    return r;
}

__device__ inline void fill_i32(int *p, long long n, int v) {
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n;
         q += (long long)gridDim.x * blockDim.x)
        p[q] = v;
}

}  // namespace eses
