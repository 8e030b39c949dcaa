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

constexpr double U64 = 1.1102230246251565e-16;  // 2^-53, unit roundoff of FP64

// Circle where SAS spheres of atoms a (owner) and b meet.  Exists iff
// |s_a - s_b| < d < s_a + s_b; centre o = c_a + t n with
// t = (s_a^2 - s_b^2 + d^2) / (2 d), n the unit vector c_a -> c_b, radius
// R = sqrt(s_a^2 - t^2).  Both build passes call this, so their decisions agree.
// nn.w receives a bound on the rounding error of each component of o and of R
// (first order, safety 4): d is within 4u d, t within
// dt = 2u (s_a^2 + s_b^2 + 3 d^2) / d + 5u |t|, R^2 within
// 3u s_a^2 + 2 |t| dt + u t^2 (so R within that over 2R, plus u R), n within 6u
// per component, and o = c_a + t n within 2u (|c_a| + |t| + s_a) + dt + 6u |t|.
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
    const double R = sqrt(R2);
    const double at = fabs(t);
    const double dt = 2.0 * U64 * (sa * sa + sb * sb + 3.0 * d2) / d + 5.0 * U64 * at;
    const double dR = (3.0 * U64 * sa * sa + 2.0 * at * dt + U64 * t * t) / (2.0 * R) + U64 * R;
    const double cm = fmax(fabs(a.x), fmax(fabs(a.y), fabs(a.z)));
    const double eps = 4.0 * (2.0 * U64 * (cm + at + sa) + dt + 6.0 * U64 * at + dR);
    nn = make_double4(vx * inv, vy * inv, vz * inv, eps);
    oR = make_double4(a.x + t * nn.x, a.y + t * nn.y, a.z + t * nn.z, R);
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

// ------------------------------------------------ certified FP64 tests
// Every comparison of the label is made in FP64 together with a bound on its
// rounding error; three-valued results: certainly true, certainly false, or
// undecided (the margin lies within the bound).  A label that depends on an
// undecided comparison is re-decided exactly on the host.  The bounds are first
// order with a safety factor of at least 4; CERT_BAND = 2^-40, relative to the
// squared length scale of a test, is at least 2^11 times the few-ulp rounding
// of its sums of squares.
constexpr double CERT_BAND = 9.094947017729282e-13;
enum { TV_NO = 0, TV_YES = 1, TV_UNSURE = 2 };

// "m < 0" (or "m <= 0": they differ only at m = 0, undecided either way) for a
// margin computed within err.
__device__ inline int tv_neg(double m, double err) {
    return m < -err ? TV_YES : (m > err ? TV_NO : TV_UNSURE);
}

// Bounds of one molecule and tile.
struct CertK {
    double gf;       // face cut: |error of c.(x - c_i) - |x - c_i| tau| <= gf |x - c_i|
    double fw_band;  // face reach: |x - c_i|^2 against (r_i + 2 rho)^2
    double inv_rho;
    double smax;
};

// tile edge span: points of a tile lie within sqrt(3) T h of each other, and a
// listed atom or face within s_max (+ rho) + sqrt(3) T h of any of them.
// Face cut (v = c_k - c_i within u|v|, tau = (s_i^2 + |v|^2 - s_k^2) / 2 s_i
// within 24u s_max^2 / rho, |v| <= 2 s_max, |tau| <= 3 s_max^2 / rho, the dot
// product within 4u d |v|, d = |x - c_i| within 4u d): the margin's error is at
// most u d (10 s_max + 42 s_max^2 / rho); gf carries a factor 2^13 over it.
__device__ inline CertK cert_consts(const Mol &m) {
    CertK k;
    const double span = 2.0 * m.tile * m.h;
    const double smax = m.smax, rho = m.rho;
    k.gf = CERT_BAND * (10.0 * smax + 42.0 * smax * smax / rho);
    k.fw_band = CERT_BAND * sq(smax + rho + span);
    k.inv_rho = 1.0 / rho;
    k.smax = smax;
    return k;
}

// Concave probe p (w: its rounding-error bound e): x strictly within rho.
// |x - p|^2 is within 2 |x - p| e (+ rounding), and 2 |x - p| <= |x - p|^2 / rho + rho.
__device__ inline int tv_probe(double x, double y, double z, double4 p, double rho2, double rho,
                               double inv_rho) {
    const double dx = x - p.x, dy = y - p.y, dz = z - p.z;
    const double d2 = dx * dx + dy * dy + dz * dz;
    const double err = 2.0 * p.w * (d2 * inv_rho + rho) + CERT_BAND * (d2 + rho2);
    return tv_neg(d2 - rho2, err);
}

// Half-space cuts of a face: admissible iff dot(x - c_i, v) <= d tau for all.
__device__ inline int tv_face_cuts(const double4 *cuts, int b, int e, double dx, double dy,
                                   double dz, double d, double gf) {
    const double err = d * gf;
    bool unsure = false;
    for (int c = b; c < e; ++c) {
        const double4 v = cuts[c];
        const double mg = dx * v.x + dy * v.y + dz * v.z - d * v.w;
        if (mg > err) return TV_NO;
        if (mg >= -err) unsure = true;
    }
    return unsure ? TV_UNSURE : TV_YES;
}

// Square root for the FP32-based classification: the FP32 root s of x
// (within 2^-21.5 relative, the conversion of x included) refined by one
// Newton step y = s + (x - s^2) h, h = 1 / 2s from the FP32 reciprocal
// (within 2^-22).  s^2 is exact in FP64, the step leaves alpha^2 / 2 of the
// FP32 error alpha and the approximate h adds |alpha| 2^-22: y is within
// 2^-42 of sqrt(x), relative (below 1e-30, where the FP32 root underflows,
// the FP64 root is taken).
constexpr double FAST_SQRT_REL = 2.2737367544323206e-13;  // 2^-42

__device__ inline double sqrt_fast(double x) {
    if (!(x >= 1e-30)) return sqrt(fmax(x, 0.0));
    const float s = __builtin_amdgcn_sqrtf((float)x);
    const double sd = (double)s;
    return sd + (x - sd * sd) * (0.5 * (double)__builtin_amdgcn_rcpf(s));
}

// Square root with a relative error bound: exact rounding (FP64) or within
// FAST_SQRT_REL (FAST).
template <bool FAST>
__device__ inline double sqrt_sel(double x) {
    if (FAST) return sqrt_fast(x);
    return sqrt(x);
}

// Per-circle constants of the cut test: the circle's bound e; with
// U = R + s_max (|o - c_k| <= R + s_k for a listed cut), Tmax = (R^2 + U^2 +
// s_max^2) / 2R >= |T_k|, the cut vector within du = e + 8u U and T_k within
// dT = (8u (R^2 + U^2 + s_max^2) + 2 R e + 2 U e) / 2R + Tmax e / R:
// ac = 4 (2 du + dT), bc = 8 U, tmax.
__device__ inline double4 circle_cut_consts(double R, double e, double smax) {
    const double U = R + smax;
    const double tmax = (R * R + U * U + smax * smax) / (2.0 * R);
    const double du = e + 8.0 * U64 * U;
    const double dT = (8.0 * U64 * (R * R + U * U + smax * smax) + 2.0 * R * e + 2.0 * U * e) /
                          (2.0 * R) +
                      tmax * e / R;
    return make_double4(e, 4.0 * (2.0 * du + dT), 8.0 * U, tmax);
}

// Circle candidate: the nearest circle point q to x strictly within rho and
// admissible.  oR: centre and radius, n: unit axis, cq: circle_cut_consts.
// w = x - o within e + u|w|; t = w.n and b = sqrt(|w|^2 - t^2); |w|^2 - t^2
// within db2 = 8u |w|^2 + 4 (b + |t|) e, so b within min(sqrt(db2), db2 / 2b);
// |x - q|^2 = |w|^2 + R^2 - 2 b R within 8 (|w| + R)(e + 8u |w|) + 2 R db;
// the in-plane vector within dwp = 2 e + 16u (b + |t|).  Each cut
// w_perp . u_k <= b T_k is within b ac + bc dwp + tmax db.  Near the axis
// (b <= 4 dwp) the nearest point's direction is not determined.
// FAST: b from sqrt_fast, its extra error FAST_SQRT_REL b added to db, and db
// itself from FP32 operations rounded up by a factor 1 + 2^-18.
template <class CutAt, bool FAST = false>
__device__ inline int tv_circle(double x, double y, double z, double4 oR, double4 n, double4 cq,
                                double rho2, int ncut, CutAt cut_at) {
    const double wx = x - oR.x, wy = y - oR.y, wz = z - oR.z;
    const double t = wx * n.x + wy * n.y + wz * n.z;
    const double ww = wx * wx + wy * wy + wz * wz;
    const double b = sqrt_sel<FAST>(fmax(ww - t * t, 0.0));
    const double R = oR.w, e = cq.x;
    const double at = fabs(t), wl = b + at;
    const double db2 = 8.0 * U64 * ww + 4.0 * wl * e;
    double db;
    if (FAST) {
        const float f2 = (float)db2, fb = (float)b;
        const float r = __builtin_amdgcn_sqrtf(f2);
        const float q = b > 0.0 ? fminf(r, f2 * 0.5f * __builtin_amdgcn_rcpf(fb)) : r;
        db = (double)q * (1.0 + 3.814697265625e-06) + FAST_SQRT_REL * b;
    } else {
        db = b > 0.0 ? fmin(sqrt(db2), db2 / (2.0 * b)) : sqrt(db2);
    }
    const double mg = ww + R * R - rho2 - 2.0 * b * R;
    const double err = 8.0 * (wl + R) * (e + 8.0 * U64 * wl) + 2.0 * R * db +
                       CERT_BAND * (ww + R * R + rho2 + 2.0 * b * R);
    const int within = tv_neg(mg, err);
    if (within == TV_NO) return TV_NO;
    const double dwp = 2.0 * e + 16.0 * U64 * wl;
    if (!(b > 4.0 * dwp)) return ncut > 0 ? TV_UNSURE : within;
    const double px = wx - t * n.x, py = wy - t * n.y, pz = wz - t * n.z;
    const double cerr = b * cq.y + cq.z * dwp + cq.w * db;
    bool unsure = within == TV_UNSURE;
    for (int c = 0; c < ncut; ++c) {
        const double4 u = cut_at(c);
        const double cm = px * u.x + py * u.y + pz * u.z - b * u.w;
        if (cm > cerr) return TV_NO;
        if (cm >= -cerr) unsure = true;
    }
    return unsure ? TV_UNSURE : TV_YES;
}

// Certified inside/outside of x against the global candidate lists of `tile`
// (the three cases of label_fp64_t): 1, 0, or 2 when undecided.
__device__ inline int label_cert(const Mol &m, int tile, double x, double y, double z) {
    const CertK K = cert_consts(m);
    const double rho = m.rho, rho2 = rho * rho;
    const double ab = CERT_BAND * sq(m.smax + 2.0 * m.tile * m.h);
    bool u_yes = false, u_uns = false, v_uns = false;
    for (int q = m.tA_off[tile], e = m.tA_off[tile + 1]; q < e; ++q) {
        double4 a = m.atom[m.tA[q]];
        double dx = x - a.x, dy = y - a.y, dz = z - a.z;
        double d2 = dx * dx + dy * dy + dz * dz;
        const int v = tv_neg(d2 - a.w * a.w, ab);
        if (v == TV_YES) return 1;
        v_uns |= v == TV_UNSURE;
        double s = a.w + rho;
        const int u = tv_neg(d2 - s * s, ab);
        u_yes |= u == TV_YES;
        u_uns |= u == TV_UNSURE;
    }
    if (v_uns) return 2;
    if (!u_yes) return u_uns ? 2 : 0;
    bool unsure = false;
    for (int q = m.tV_off[tile], e = m.tV_off[tile + 1]; q < e; ++q) {
        const int t = tv_probe(x, y, z, m.vert_p[m.tV[q]], rho2, rho, K.inv_rho);
        if (t == TV_YES) return 0;
        unsure |= t == TV_UNSURE;
    }
    for (int q = m.tF_off[tile], e = m.tF_off[tile + 1]; q < e; ++q) {
        int f = m.tF[q];
        double4 a = m.atom[m.face_atom[f]];
        double dx = x - a.x, dy = y - a.y, dz = z - a.z;
        double d2 = dx * dx + dy * dy + dz * dz;
        const int w = tv_neg(d2 - sq(a.w + 2.0 * rho), K.fw_band);
        if (w == TV_NO) continue;
        const int c = tv_face_cuts(m.face_cut, m.face_cut_off[f], m.face_cut_off[f + 1], dx, dy,
                                   dz, sqrt(d2), K.gf);
        if (c == TV_NO) continue;
        if (w == TV_YES && c == TV_YES) return 0;
        unsure = true;
    }
    for (int q = m.tC_off[tile], e = m.tC_off[tile + 1]; q < e; ++q) {
        int ec = m.tC[q];
        int ci = m.ec_circ[ec];
        double4 oR = m.circ_oR[ci];
        double4 n = m.circ_n[ci];
        const double4 cq = circle_cut_consts(oR.w, n.w, K.smax);
        const int cb = m.ec_cut_off[ec];
        const int t = tv_circle(x, y, z, oR, n, cq, rho2, m.ec_cut_off[ec + 1] - cb,
                                [&](int c) { return m.ec_cut[cb + c]; });
        if (t == TV_YES) return 0;
        unsure |= t == TV_UNSURE;
    }
    return unsure ? 2 : 1;
}

// A point whose label could not be certified: queued (grid index) for the
// exact re-decision on the host; its byte is overwritten there.
__device__ inline void push_uncertain(const Mol &m, long long gi) {
    const int slot = atomicAdd(m.unc_n, 1);
    if (slot < m.unc_cap) m.unc_idx[slot] = gi;
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
