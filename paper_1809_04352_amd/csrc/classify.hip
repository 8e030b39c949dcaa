// Stage 2: inside/outside label of every grid point (eq. 2).
//
// One workgroup per tile of TILE^3 points.  Each lane owns one point; the
// tile's candidate lists (shared by all its points) are read through the
// cache, and the label is written as one byte per point (x fastest).
#include "eses_device.h"
#include "launch.h"

namespace eses {

constexpr int CLS_BLOCK = 512;

// One workgroup per tile.
//  Phase 1 stages the tile's atom list in LDS (chunks of CLS_ATOMS), with a
//  sub-list per 4^3 sub-tile of the atoms that can reach it, and decides
//  cases 1 and 2 for every point; the undecided points (inside an SAS ball,
//  in no van der Waals ball) are compacted into an LDS queue.
//  Staging copies the tile's probe, face and circle lists into LDS together
//  with the cuts that can matter inside the tile: a cut (v, tau) of a face
//  can only reject a direction u from c_i with u . v > tau, so a cut whose
//  half-space holds the whole cone of directions from c_i towards the tile is
//  dropped (likewise for circle cuts, with in-plane directions from o).
//  Phase 2 runs the candidate tests over the queue with every lane busy.
// Lists or cut pools larger than the LDS capacities fall back to global
// memory (uncut), so results never depend on the capacities.
constexpr int CLS_THREADS = 256;
constexpr int CLS_WAVES = CLS_THREADS / WAVE;
constexpr int CLS_ATOMS = 256;
constexpr int CLS_MAXPTS = 512;  // points per tile (8^3)
constexpr int CAP_V = 48, CAP_F = 48, CAP_C = 48, CAP_CUT = 320;
// Six waves per SIMD (80 VGPRs, a few spilled; 26 KB of LDS per workgroup, so
// that six workgroups fit the 160 KB of a CU):
// the kernel waits mostly on dependent loads, and on the batch the extra
// resident workgroups outweigh the spills (28.6 vs 33.3 ms at four waves;
// seven and eight waves, with more spills and smaller cut pools, 29.9 and
// 30.1 ms).
constexpr int CLS_WAVES_PER_EU = 6;

// 8^3 tiles: the staged atoms whose SAS ball (plus a margin far above any
// rounding) reaches each 4^3 sub-tile; the other atoms are certainly outside
// the SAS ball of every point there, so their tests are skipped.
struct ClsSubLists {
    unsigned char at[8][CLS_ATOMS];
    int n[8];
};

struct ClsPhase1 {
    double4 a[CLS_ATOMS];  // FP64: x, y, z, r^2
    double s2[CLS_ATOMS];  // FP64: (r + rho)^2
    double bd[CLS_ATOMS];  // FP64: error bound of both comparisons
    ClsSubLists sub;
};

struct ClsPhase1f {
    float4 a[CLS_ATOMS];   // FP32: atom offset from the tile origin
    float4 t[CLS_ATOMS];   // FP32 thresholds: vdW (lo, hi), SAS (lo, hi)
    ClsSubLists sub;
};

struct ClsPhase2 {
    double4 v[CAP_V];      // probe positions
    double4 f[CAP_F];      // face atom x, y, z, (r + 2 rho)^2
    int2 fr[CAP_F];        // cut range in `cut` (start, count), or (-1, face id): global cuts
    double4 co[CAP_C];     // circle o, R
    double4 cn[CAP_C];     // circle n, rounding-error bound of o and R
    double4 cq[CAP_C];     // constants of the certified cut test (circle_cut_consts)
    int2 cr[CAP_C];        // cut range, or (-1, exposed-circle id)
    double4 cut[CAP_CUT];
    // staging of the cuts: per surface (faces, then circles) the first
    // global cut, the prefix of the uncut counts (pair -> surface), the
    // number of cuts kept and their region in `cut`
    // each surface's cone over the tile, rounded to FP32 (axis, sin; cos, or
    // -1 for a cone of every direction); the cut test allows for the rounding
    float4 cna[CAP_F + CAP_C];
    float cnc[CAP_F + CAP_C];
    int ccb[CAP_F + CAP_C];
    int coff[CAP_F + CAP_C + 1];
    int ccur[CAP_F + CAP_C];
    int koff[CAP_F + CAP_C];
    int dead[CAP_F + CAP_C];  // one cut rejects the surface's candidate over the whole tile
    int scan[CLS_WAVES + 1];
};

struct ClsShared {
    union {
        ClsPhase1 p1;
        ClsPhase1f p1f;
        ClsPhase2 p2;
    };
    int queue[CLS_MAXPTS];   // points for the candidate tests (case 3)
    int rqueue[CLS_MAXPTS];  // FP32 points whose phase-1 decision was not certified
    int qn, rqn, pool;
};

// Certified FP32 phase-1 thresholds.  With offsets X, C of the point and the
// atom from the tile origin (|components| <= lam), the FP32 difference
// delta differs from the exact x - c by at most E = 4.01 u lam per component
// (two conversions and one subtraction, u = 2^-24), so the exact squared
// distance is within c0 = 3 E (4 lam + E) of sum(delta^2), and the FP32 sum of
// squares S is within gamma_3 <= 4u (relative) of sum(delta^2), with or
// without fused multiply-adds.  Hence, for an exact threshold t,
//   S < lo = (t (1 - 2^-52) - c0) (1 - 4u)  =>  |x - c|^2 < t   (certain),
//   S > hi = (t (1 + 2^-52) + c0) (1 + 4u)  =>  |x - c|^2 > t   (certain),
// with lo rounded down and hi rounded up to FP32.
constexpr double U32 = 5.9604644775390625e-08;  // 2^-24

__device__ inline float thr_lo(double t, double c0) {
    return __double2float_rd((t * (1.0 - 2.220446049250313e-16) - c0) * (1.0 - 4.0 * U32));
}

__device__ inline float thr_hi(double t, double c0) {
    return __double2float_ru((t * (1.0 + 2.220446049250313e-16) + c0) * (1.0 + 4.0 * U32));
}

// Directional cone of the tile from an apex: axis `a` (unit), sin and cos of
// the half-angle; `all` when the apex is inside the tile's ball.
struct Cone {
    double ax, ay, az, st, ct;
    bool all;
};

__device__ inline Cone make_cone(double vx, double vy, double vz, double rb) {
    Cone c;
    double L = sqrt(vx * vx + vy * vy + vz * vz);
    c.all = !(L > rb * (1.0 + 1e-12) + 1e-12);
    if (c.all) {
        c.ax = c.ay = c.az = c.st = 0.0;
        c.ct = 1.0;
        return c;
    }
    c.ax = vx / L;
    c.ay = vy / L;
    c.az = vz / L;
    c.st = rb / L;
    c.ct = sqrt(fmax(0.0, 1.0 - c.st * c.st));
    return c;
}

// Whether cut (v, tau) can reject some direction u of the cone (u . v >
// tau): the maximum of u . v over the cone, |v| cos(max(0, phi - theta)),
// against tau with a small slack.  The cone's parameters are rounded to FP32
// (each within 2^-23 relative of its FP64 value).  The axis a' is rescaled
// by one Newton step for 1 / |a'| (|a'|^2 is within 4e-7 of 1, so the step
// is exact to 1e-13): cp is then the cosine of the angle phi' between v and
// a direction within 2e-7 rad of the exact axis, to 1e-13, so that
// phi' is within 4e-7 rad of phi even where cp is near +-1, and the maximum
// moves by less than 1e-6 |v|; the slack covers it, so no cut that matters is
// dropped (an extra kept cut only costs a test).
__device__ inline double cone_cos(float4 a, double4 v, double vn) {
    const double ax = a.x, ay = a.y, az = a.z;
    return (ax * v.x + ay * v.y + az * v.z) / vn * (1.5 - 0.5 * (ax * ax + ay * ay + az * az));
}

__device__ inline bool cut_matters_f(float4 a, float ct, double4 cut) {
    if (ct < 0.0f) return true;
    const double vn = sqrt(cut.x * cut.x + cut.y * cut.y + cut.z * cut.z);
    if (!(vn > 0.0)) return 0.0 > cut.w - 1e-9;
    const double cp = cone_cos(a, cut, vn);
    double best;
    if (cp >= (double)ct) {
        best = vn;
    } else {
        const double sp = sqrt(fmax(0.0, 1.0 - cp * cp));
        best = vn * (cp * (double)ct + sp * (double)a.w);
    }
    return best > cut.w - 1e-9 - 1e-6 * vn;
}

// Whether cut (v, tau) rejects every direction u of the cone: the minimum of
// u . v over the cone, |v| cos(phi + theta), above tau by the same slack
// (when the cone does not reach -v).  The surface's candidate is then
// inadmissible at every point of the tile, and its tests are skipped.
__device__ inline bool cut_rejects_cone_f(float4 a, float ct, double4 cut) {
    if (ct < 0.0f) return false;
    const double vn = sqrt(cut.x * cut.x + cut.y * cut.y + cut.z * cut.z);
    if (!(vn > 0.0)) return false;
    const double cp = cone_cos(a, cut, vn);
    if (cp <= -(double)ct) return false;
    const double sp = sqrt(fmax(0.0, 1.0 - cp * cp));
    return vn * (cp * (double)ct - sp * (double)a.w) >
           cut.w + 1e-9 * (vn + fabs(cut.w)) + 1e-6 * vn;
}

__device__ inline bool cuts_pass(const double4 *cuts, int b, int e, double dx, double dy,
                                 double dz, double d) {
    for (int c = b; c < e; ++c) {
        double4 v = cuts[c];
        if (dx * v.x + dy * v.y + dz * v.z > d * v.w) return false;
    }
    return true;
}

// Case 3 of one queued point against the staged lists (global beyond them),
// every comparison certified: 0 (an admissible candidate certainly within
// rho), 1 (certainly none), 2 (undecided in FP64).  FAST (the FP32-based
// mode): the square roots come from FP32 roots refined by a Newton step
// (sqrt_fast, within 2^-42 relative).  For a face that adds at most
// 2^-42 d |tau| <= 3 2^-42 d s_max^2 / rho to the cut margins' error, about
// 1/50 of the gf bound; tv_circle widens its own bounds.
template <bool FAST>
__device__ inline int shell_cert_staged(const Mol &m, const ClsShared &sh, const CertK &K,
                                        int tile, int nV, int nF, int nC, double x, double y,
                                        double z) {
    const double rho = m.rho;
    const double rho2 = rho * rho;
    bool unsure = false;
    for (int q = 0; q < nV; ++q) {
        const int t = tv_probe(x, y, z, sh.p2.v[q], rho2, rho, K.inv_rho);
        if (t == TV_YES) return 0;
        unsure |= t == TV_UNSURE;
    }
    for (int q = m.tV_off[tile] + nV, e = m.tV_off[tile + 1]; q < e; ++q) {
        const int t = tv_probe(x, y, z, m.vert_p[m.tV[q]], rho2, rho, K.inv_rho);
        if (t == TV_YES) return 0;
        unsure |= t == TV_UNSURE;
    }
    for (int q = 0; q < nF; ++q) {
        const int2 r = sh.p2.fr[q];
        if (r.x == -2) continue;  // candidate inadmissible over the whole tile
        double4 a = sh.p2.f[q];
        double dx = x - a.x, dy = y - a.y, dz = z - a.z;
        double d2 = dx * dx + dy * dy + dz * dz;
        const int w = tv_neg(d2 - a.w, K.fw_band);
        if (w == TV_NO) continue;
        const double d = sqrt_sel<FAST>(d2);
        const int c = r.x >= 0 ? tv_face_cuts(sh.p2.cut, r.x, r.x + r.y, dx, dy, dz, d, K.gf)
                               : tv_face_cuts(m.face_cut, m.face_cut_off[r.y],
                                              m.face_cut_off[r.y + 1], dx, dy, dz, d, K.gf);
        if (c == TV_NO) continue;
        if (w == TV_YES && c == TV_YES) return 0;
        unsure = true;
    }
    for (int q = m.tF_off[tile] + nF, e = m.tF_off[tile + 1]; q < e; ++q) {
        int f = m.tF[q];
        double4 a = m.atom[m.face_atom[f]];
        double dx = x - a.x, dy = y - a.y, dz = z - a.z;
        double d2 = dx * dx + dy * dy + dz * dz;
        const int w = tv_neg(d2 - sq(a.w + 2.0 * rho), K.fw_band);
        if (w == TV_NO) continue;
        const int c = tv_face_cuts(m.face_cut, m.face_cut_off[f], m.face_cut_off[f + 1], dx, dy,
                                   dz, sqrt_sel<FAST>(d2), K.gf);
        if (c == TV_NO) continue;
        if (w == TV_YES && c == TV_YES) return 0;
        unsure = true;
    }
    for (int q = 0; q < nC + (m.tC_off[tile + 1] - m.tC_off[tile] - nC); ++q) {
        double4 oR, n, cq;
        int2 r;
        if (q < nC) {
            r = sh.p2.cr[q];
            if (r.x == -2) continue;  // candidate inadmissible over the whole tile
            oR = sh.p2.co[q];
            n = sh.p2.cn[q];
            cq = sh.p2.cq[q];
        } else {
            int ec = m.tC[m.tC_off[tile] + q];
            int ci = m.ec_circ[ec];
            oR = m.circ_oR[ci];
            n = m.circ_n[ci];
            cq = circle_cut_consts(oR.w, n.w, K.smax);
            r = make_int2(-1, ec);
        }
        int t;
        if (r.x >= 0) {
            auto at = [&](int c) { return sh.p2.cut[r.x + c]; };
            t = tv_circle<decltype(at), FAST>(x, y, z, oR, n, cq, rho2, r.y, at);
        } else {
            const int cb = m.ec_cut_off[r.y];
            auto at = [&](int c) { return m.ec_cut[cb + c]; };
            t = tv_circle<decltype(at), FAST>(x, y, z, oR, n, cq, rho2,
                                              m.ec_cut_off[r.y + 1] - cb, at);
        }
        if (t == TV_YES) return 0;
        unsure |= t == TV_UNSURE;
    }
    return unsure ? 2 : 1;
}

// Grid point p of tile t3 (T^3 points).  An 8^3 tile takes its points by 4^3
// sub-tiles, 64 consecutive p each, so that a wavefront holds one sub-tile;
// other tiles go row by row.
__device__ inline void tile_point(int p, int T, const int *t3, int &i, int &j, int &k) {
    if (T == 8) {
        const int sb = p >> 6, l = p & 63;
        i = t3[0] * 8 + ((sb & 1) << 2) + (l & 3);
        j = t3[1] * 8 + (((sb >> 1) & 1) << 2) + ((l >> 2) & 3);
        k = t3[2] * 8 + ((sb >> 2) << 2) + (l >> 4);
    } else {
        i = t3[0] * T + p % T;
        j = t3[1] * T + (p / T) % T;
        k = t3[2] * T + p / (T * T);
    }
}

// F32: phase 1 (cases 1 and 2, every point against the tile's atoms) in FP32
// with the certified thresholds above; points it cannot certify are
// re-labelled in FP64 (counted in diag[1]).  Case 3 runs in FP64 either way,
// with the square roots of its tests from FP32 roots and one Newton step.
template <bool F32>
__device__ void classify_tile(const Mol &m, int tile, uint8_t *labels, ClsShared &sh) {
    const int T = m.tile;
    const int P = T * T * T;
    const int t3[3] = {tile % m.tdims[0], (tile / m.tdims[0]) % m.tdims[1],
                       tile / (m.tdims[0] * m.tdims[1])};
    constexpr int PPT = CLS_MAXPTS / CLS_THREADS;  // points per thread
    double px[PPT], py[PPT], pz[PPT];
    float fx[PPT], fy[PPT], fz[PPT];
    bool valid[PPT], inv[PPT], inu[PPT], vmay[PPT], umay[PPT];
    double org[3];
    for (int a = 0; a < 3; ++a) org[a] = mol_coord(m, a, t3[a] * T);
    for (int r = 0; r < PPT; ++r) {
        int p = threadIdx.x + r * CLS_THREADS;
        int i, j, k;
        tile_point(p, T, t3, i, j, k);
        valid[r] = p < P && i < m.dims[0] && j < m.dims[1] && k < m.dims[2];
        px[r] = mol_coord(m, 0, i);
        py[r] = mol_coord(m, 1, j);
        pz[r] = mol_coord(m, 2, k);
        fx[r] = (float)(px[r] - org[0]);
        fy[r] = (float)(py[r] - org[1]);
        fz[r] = (float)(pz[r] - org[2]);
        inv[r] = false;
        inu[r] = false;
        vmay[r] = false;
        umay[r] = false;
    }
    if (threadIdx.x == 0) {
        sh.qn = 0;
        sh.rqn = 0;
        sh.pool = 0;
    }
    const int a0 = m.tA_off[tile], a1 = m.tA_off[tile + 1];
    const double rho = m.rho;
    // bound of the offsets' components: tile points and atoms within s_max of it
    const double lam = (T - 1) * m.h + m.smax + 1e-3;
    // FP64 phase 1: |x - c|^2, r^2 and s^2 within a few ulps; a listed atom's
    // centre lies within s + span of every point of the tile
    const double span = 2.0 * T * m.h;
    const double bandA = CERT_BAND;
    const double E = 4.01 * U32 * lam;
    const double cb = 3.0 * E * (4.0 * lam + E) + 1e-30;
    const bool subt = T == 8;
    ClsSubLists &SL = F32 ? sh.p1f.sub : sh.p1.sub;
    for (int base = a0; base < a1; base += CLS_ATOMS) {
        int cnt = min(CLS_ATOMS, a1 - base);
        __syncthreads();
        if (subt) {
            if (threadIdx.x < 8) SL.n[threadIdx.x] = 0;
            __syncthreads();
        }
        for (int q = threadIdx.x; q < cnt; q += CLS_THREADS) {
            double4 a = m.atom[m.tA[base + q]];
            if (subt) {
                // squared distance from the centre to each half of the tile
                // per axis (points 0-3 and 4-7); an atom joins the sub-tiles
                // its SAS ball, grown by 1e-3, reaches
                double dh[3][2];
                const double cc[3] = {a.x, a.y, a.z};
                for (int ax = 0; ax < 3; ++ax)
                    for (int hb = 0; hb < 2; ++hb) {
                        const double lo = mol_coord(m, ax, t3[ax] * 8 + 4 * hb),
                                     hi = mol_coord(m, ax, t3[ax] * 8 + 4 * hb + 3);
                        const double dd = cc[ax] < lo ? lo - cc[ax] : cc[ax] > hi ? cc[ax] - hi : 0.0;
                        dh[ax][hb] = dd * dd;
                    }
                const double reach = sq(a.w + rho + 1e-3);
                for (int sb = 0; sb < 8; ++sb) {
                    const double d2 = dh[0][sb & 1] + dh[1][(sb >> 1) & 1] + dh[2][sb >> 2];
                    if (d2 < reach) SL.at[sb][atomicAdd(&SL.n[sb], 1)] = (unsigned char)q;
                }
            }
            if (F32) {
                sh.p1f.a[q] = make_float4((float)(a.x - org[0]), (float)(a.y - org[1]),
                                          (float)(a.z - org[2]), 0.0f);
                double s = a.w + rho;
                sh.p1f.t[q] = make_float4(thr_lo(a.w * a.w, cb), thr_hi(a.w * a.w, cb),
                                          thr_lo(s * s, cb), thr_hi(s * s, cb));
            } else {
                sh.p1.a[q] = make_double4(a.x, a.y, a.z, a.w * a.w);
                sh.p1.s2[q] = sq(a.w + rho);
                sh.p1.bd[q] = bandA * sq(a.w + rho + span);
            }
        }
        __syncthreads();
        for (int r = 0; r < PPT; ++r) {
            if (!valid[r] || inv[r]) continue;
            // the atoms that can reach the point's sub-tile (every staged atom
            // for other tiles): the order of the tests does not matter
            const int sb = subt ? (int)(threadIdx.x >> 6) + 4 * r : 0;
            const int nl = subt ? SL.n[sb] : cnt;
            if (F32) {
                bool v = false, vm = vmay[r], u = inu[r], um = umay[r];
                for (int qq = 0; qq < nl; ++qq) {
                    const int q = subt ? (int)SL.at[sb][qq] : qq;
                    float4 a = sh.p1f.a[q];
                    float4 t = sh.p1f.t[q];
                    float dx = fx[r] - a.x, dy = fy[r] - a.y, dz = fz[r] - a.z;
                    float d2 = dx * dx + dy * dy + dz * dz;
                    v |= d2 < t.x;
                    vm |= d2 <= t.y;
                    u |= d2 < t.z;
                    um |= d2 <= t.w;
                }
                inv[r] = v;
                vmay[r] = vm;
                inu[r] = u;
                umay[r] = um;
            } else {
                // certified: certainly in (margin below -bound), maybe in
                // (margin at most +bound)
                bool v = false, vm = vmay[r], u = inu[r], um = umay[r];
                for (int qq = 0; qq < nl; ++qq) {
                    const int q = subt ? (int)SL.at[sb][qq] : qq;
                    double4 a = sh.p1.a[q];
                    double dx = px[r] - a.x, dy = py[r] - a.y, dz = pz[r] - a.z;
                    double d2 = dx * dx + dy * dy + dz * dz;
                    const double bd = sh.p1.bd[q];
                    const double mv = d2 - a.w, ms = d2 - sh.p1.s2[q];
                    v |= mv < -bd;
                    vm |= mv <= bd;
                    u |= ms < -bd;
                    um |= ms <= bd;
                }
                inv[r] = v;
                vmay[r] = vm;
                inu[r] = u;
                umay[r] = um;
            }
        }
    }
    __syncthreads();
    for (int r = 0; r < PPT; ++r) {
        if (!valid[r]) continue;
        int p = threadIdx.x + r * CLS_THREADS;
        int i, j, k;
        tile_point(p, T, t3, i, j, k);
        long long gi = (long long)i + (long long)m.dims[0] * ((long long)j + (long long)m.dims[1] * k);
        // certain: in a vdW ball; outside every SAS ball; or shell (in an SAS
        // ball, certainly in no vdW ball).  Otherwise FP32 decisions are
        // re-tested in FP64 and FP64 ones re-decided exactly on the host.
        if (F32 && m.force_recheck) {
            sh.rqueue[atomicAdd(&sh.rqn, 1)] = p;
        } else if (inv[r]) {
            labels[gi] = 1;
        } else if (!umay[r]) {
            labels[gi] = 0;
        } else if (inu[r] && !vmay[r]) {
            sh.queue[atomicAdd(&sh.qn, 1)] = p;
        } else if (F32) {
            sh.rqueue[atomicAdd(&sh.rqn, 1)] = p;
        } else {
            labels[gi] = 0;
            push_uncertain(m, gi);
        }
    }
    __syncthreads();
    if (F32) {
        const int nr = sh.rqn;
        for (int q = threadIdx.x; q < nr; q += CLS_THREADS) {
            int p = sh.rqueue[q];
            int i, j, k;
            tile_point(p, T, t3, i, j, k);
            const long long gi =
                (long long)i + (long long)m.dims[0] * ((long long)j + (long long)m.dims[1] * k);
            const int lab = label_cert(m, tile, mol_coord(m, 0, i),
                                       mol_coord(m, 1, j), mol_coord(m, 2, k));
            labels[gi] = (uint8_t)(lab == 1);
            if (lab == 2) push_uncertain(m, gi);
        }
        if (threadIdx.x == 0 && nr > 0) atomicAdd(&m.diag[1], nr);
    }
    const int nq = sh.qn;
    if (nq == 0) return;  // uniform: no point needs the candidate tests
    const CertK K = cert_consts(m);

    // staging of the candidate lists (phase-1 LDS is dead from here on)
    const int v0 = m.tV_off[tile], f0 = m.tF_off[tile], c0 = m.tC_off[tile];
    const int nV = min(CAP_V, m.tV_off[tile + 1] - v0);
    const int nF = min(CAP_F, m.tF_off[tile + 1] - f0);
    const int nC = min(CAP_C, m.tC_off[tile + 1] - c0);
    for (int q = threadIdx.x; q < nV; q += CLS_THREADS) sh.p2.v[q] = m.vert_p[m.tV[v0 + q]];
    for (int q = threadIdx.x; q < nF; q += CLS_THREADS) {
        double4 a = m.atom[m.face_atom[m.tF[f0 + q]]];
        sh.p2.f[q] = make_double4(a.x, a.y, a.z, sq(a.w + 2.0 * rho));
    }
    for (int q = threadIdx.x; q < nC; q += CLS_THREADS) {
        int ci = m.ec_circ[m.tC[c0 + q]];
        double4 oR = m.circ_oR[ci];
        double4 n = m.circ_n[ci];
        sh.p2.co[q] = oR;
        sh.p2.cn[q] = n;
        sh.p2.cq[q] = circle_cut_consts(oR.w, n.w, m.smax);
    }
    // the cone loop below reads circles staged by other threads
    __syncthreads();
    // the tile's own points span T - 1 spacings per axis
    double bc[3], rb;
    {
        double half = 0.5 * (T - 1) * m.h;
        for (int a = 0; a < 3; ++a)
            bc[a] = m.lo[a] + (double)(t3[a] * T + (a == 2 ? m.kz0 : 0)) * m.h + half;
        rb = sqrt(3.0) * half * (1.0 + 1e-12) + 1e-12;
    }
    // cuts of the staged faces and circles that can matter inside the tile,
    // tested with every thread on a (surface, cut) pair: one pass counts the
    // kept cuts per surface, the next copies them into the surface's region
    // of the pool; a surface whose kept cuts overflow the pool keeps all of
    // its cuts in global memory
    const int nS = nF + nC;
    int ncut = 0;
    if ((int)threadIdx.x < nS) {
        const int q = threadIdx.x;
        int id, cb, ce;
        if (q < nF) {
            id = m.tF[f0 + q];
            cb = m.face_cut_off[id];
            ce = m.face_cut_off[id + 1];
        } else {
            id = m.tC[c0 + q - nF];
            cb = m.ec_cut_off[id];
            ce = m.ec_cut_off[id + 1];
        }
        sh.p2.ccb[q] = cb;
        sh.p2.ccur[q] = 0;
        sh.p2.dead[q] = 0;
        ncut = ce - cb;
    }
    // each surface's cone over the tile, once
    for (int q = threadIdx.x; q < nS; q += CLS_THREADS) {
        double vx, vy, vz;
        if (q < nF) {
            const double4 a = sh.p2.f[q];
            vx = bc[0] - a.x;
            vy = bc[1] - a.y;
            vz = bc[2] - a.z;
        } else {
            const double4 oR = sh.p2.co[q - nF], n = sh.p2.cn[q - nF];
            const double wx = bc[0] - oR.x, wy = bc[1] - oR.y, wz = bc[2] - oR.z;
            const double t = wx * n.x + wy * n.y + wz * n.z;
            vx = wx - t * n.x;
            vy = wy - t * n.y;
            vz = wz - t * n.z;
        }
        const Cone cone = make_cone(vx, vy, vz, rb);
        sh.p2.cna[q] = make_float4((float)cone.ax, (float)cone.ay, (float)cone.az, (float)cone.st);
        sh.p2.cnc[q] = cone.all ? -1.0f : (float)cone.ct;
    }
    int total;
    const int coff = block_excl_scan<int, CLS_THREADS>(ncut, sh.p2.scan, &total);
    if ((int)threadIdx.x < nS) sh.p2.coff[threadIdx.x] = coff;
    if (threadIdx.x == 0) sh.p2.coff[nS] = total;
    __syncthreads();
    for (int pass = 0; pass < 2; ++pass) {
        for (int p = threadIdx.x; p < total; p += CLS_THREADS) {
            int lo = 0, hi = nS;
            while (lo < hi) {
                int mid = (lo + hi) >> 1;
                if (sh.p2.coff[mid + 1] <= p) lo = mid + 1;
                else hi = mid;
            }
            const int q = lo;
            if (pass == 1 && sh.p2.koff[q] < 0) continue;  // not staged
            const int c = sh.p2.ccb[q] + (p - sh.p2.coff[q]);
            const double4 v = q < nF ? m.face_cut[c] : m.ec_cut[c];
            if (pass == 0 && cut_rejects_cone_f(sh.p2.cna[q], sh.p2.cnc[q], v)) sh.p2.dead[q] = 1;
            if (!cut_matters_f(sh.p2.cna[q], sh.p2.cnc[q], v)) continue;
            const int k = atomicAdd(&sh.p2.ccur[q], 1);
            if (pass == 1) sh.p2.cut[sh.p2.koff[q] + k] = v;
        }
        if (pass == 1) break;
        // kept counts -> regions of the pool
        __syncthreads();
        int kept = 0;
        if ((int)threadIdx.x < nS && !sh.p2.dead[threadIdx.x]) kept = sh.p2.ccur[threadIdx.x];
        int ktot;
        const int koff = block_excl_scan<int, CLS_THREADS>(kept, sh.p2.scan, &ktot);
        if ((int)threadIdx.x < nS) {
            const int q = threadIdx.x;
            const bool dead = sh.p2.dead[q] != 0;
            const bool fits = !dead && koff + kept <= CAP_CUT;
            sh.p2.koff[q] = fits ? koff : -1;
            sh.p2.ccur[q] = 0;
            // (-2, 0): dead in this tile, skipped by the shell tests
            const int2 r = dead ? make_int2(-2, 0)
                         : fits ? make_int2(koff, kept)
                                : make_int2(-1, q < nF ? m.tF[f0 + q] : m.tC[c0 + q - nF]);
            if (q < nF) sh.p2.fr[q] = r;
            else sh.p2.cr[q - nF] = r;
        }
        __syncthreads();
    }
    __syncthreads();
    for (int q = threadIdx.x; q < nq; q += CLS_THREADS) {
        int p = sh.queue[q];
        int i, j, k;
        tile_point(p, T, t3, i, j, k);
        const int lab = shell_cert_staged<F32>(m, sh, K, tile, nV, nF, nC, mol_coord(m, 0, i),
                                          mol_coord(m, 1, j), mol_coord(m, 2, k));
        const long long gi =
            (long long)i + (long long)m.dims[0] * ((long long)j + (long long)m.dims[1] * k);
        labels[gi] = (uint8_t)(lab == 1);
        if (lab == 2) push_uncertain(m, gi);
    }
}

template <bool F32>
__global__ void __launch_bounds__(CLS_THREADS) __attribute__((amdgpu_waves_per_eu(CLS_WAVES_PER_EU)))
    k_classify(Mol m, uint8_t *labels, int nblocks) {
    __shared__ ClsShared sh;
    const int tile = xcd_tile(blockIdx.x, nblocks, m.ntiles);
    if (tile < 0) return;  // uniform across the workgroup
    classify_tile<F32>(m, tile, labels, sh);
}

// Persistent form for a batch of molecules: each workgroup pulls (molecule,
// tile) units from an atomic queue until the queue is empty (every wave
// reaches that exit).  Units are ordered heaviest first (tiles with
// candidate features, then tiles with atoms, then empty tiles).
template <bool F32>
__global__ void __launch_bounds__(CLS_THREADS) __attribute__((amdgpu_waves_per_eu(CLS_WAVES_PER_EU)))
    k_classify_batch(const Mol *mols,
                                                               uint8_t *const *labels,
                                                               const int2 *units, int nunits,
                                                               int *head) {
    __shared__ ClsShared sh;
    __shared__ int cur;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) cur = atomicAdd(head, 1);
        __syncthreads();
        // the unit and the molecule's view are uniform: keep them in SGPRs
        const int u = __builtin_amdgcn_readfirstlane(cur);
        if (u >= nunits) break;  // uniform across the workgroup
        const int2 w = units[u];
        const int mol = __builtin_amdgcn_readfirstlane(w.x);
        const int tile = __builtin_amdgcn_readfirstlane(w.y);
        classify_tile<F32>(uniform_mol(mols, mol), tile, labels[mol], sh);
    }
}

// Work units of a batch, heaviest first, so that the persistent workgroups
// end together (longest-processing-time order).  Each (molecule, tile) unit
// gets a class, counted then scattered class by class:
//   order 0: three classes, tiles with probe, face or circle candidates, then
//            tiles with atoms only, then empty tiles;
//   order 1: the tile's estimated cost, nA + 4 (nF + nC) + nV from its list
//            sizes (phase 1 tests every atom for every point; faces and
//            circles bring the shell tests and their cut planes), in
//            half-octave buckets, heaviest class first, empty tiles last.
__device__ inline int unit_class(const Mol *mols, const int *tile_base, int nmols, long long g,
                                 int order, int &mol, int &t) {
    int lo = 0, hi = nmols - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (tile_base[mid] <= g) lo = mid;
        else hi = mid - 1;
    }
    const Mol &m = mols[lo];
    mol = lo;
    t = (int)(g - tile_base[lo]);
    const int nA = m.tA_off[t + 1] - m.tA_off[t];
    const int nF = m.tF_off[t + 1] - m.tF_off[t], nC = m.tC_off[t + 1] - m.tC_off[t],
              nV = m.tV_off[t + 1] - m.tV_off[t];
    if (order == 0) return nF + nC + nV > 0 ? 0 : (nA > 0 ? 1 : 2);
    const unsigned cost = (unsigned)(nA + 4 * (nF + nC) + nV);
    if (cost == 0) return UNIT_CLASSES - 1;
    const int lg = 31 - __clz(cost);  // floor(log2(cost))
    const int half = lg > 0 ? (int)((cost >> (lg - 1)) & 1u) : 0;
    const int bucket = min(2 * lg + half, UNIT_CLASSES - 2);
    return UNIT_CLASSES - 2 - bucket;
}

// Units per class: counted in LDS, one global add per class and block.
__global__ void __launch_bounds__(256) k_unit_count(const Mol *mols, const int *tile_base,
                                                    int nmols, long long total, int order,
                                                    int *cls_count) {
    __shared__ int cls[UNIT_CLASSES];
    if (threadIdx.x < UNIT_CLASSES) cls[threadIdx.x] = 0;
    __syncthreads();
    long long g = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (g < total) {
        int mol, t;
        atomicAdd(&cls[unit_class(mols, tile_base, nmols, g, order, mol, t)], 1);
    }
    __syncthreads();
    if (threadIdx.x < UNIT_CLASSES && cls[threadIdx.x] > 0)
        atomicAdd(&cls_count[threadIdx.x], cls[threadIdx.x]);
}

// The unit list, class by class: a block ranks its units per class in LDS
// and reserves each class's run with one global add.
__global__ void __launch_bounds__(256) k_unit_scatter(const Mol *mols, const int *tile_base,
                                                      int nmols, long long total, int order,
                                                      int *cls_fill, int2 *units) {
    __shared__ int cls[UNIT_CLASSES], base[UNIT_CLASSES];
    if (threadIdx.x < UNIT_CLASSES) cls[threadIdx.x] = 0;
    __syncthreads();
    long long g = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    int c = -1, r = 0, mol = 0, t = 0;
    if (g < total) {
        c = unit_class(mols, tile_base, nmols, g, order, mol, t);
        r = atomicAdd(&cls[c], 1);
    }
    __syncthreads();
    if (threadIdx.x < UNIT_CLASSES && cls[threadIdx.x] > 0)
        base[threadIdx.x] = atomicAdd(&cls_fill[threadIdx.x], cls[threadIdx.x]);
    __syncthreads();
    if (c >= 0) units[base[c] + r] = make_int2(mol, t);
}

// cls_fill[c] = first slot of class c (an exclusive scan of the counts).
__global__ void k_unit_bases(const int *cls_count, int *cls_fill) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        int acc = 0;
        for (int c = 0; c < UNIT_CLASSES; ++c) {
            cls_fill[c] = acc;
            acc += cls_count[c];
        }
    }
}

// Statistics pass: the same decision with its tests tallied (not timed).
__global__ void __launch_bounds__(CLS_BLOCK) k_classify_work(Mol m, unsigned long long *work) {
    const int T = m.tile;
    const int per = T * T * T;
    const int tiles_per_block = CLS_BLOCK / per;
    int tile = blockIdx.x * tiles_per_block + threadIdx.x / per;
    unsigned long long cnt[WC_COUNT] = {0, 0, 0, 0, 0, 0, 0};
    if (tile < m.ntiles) {
        int local = threadIdx.x % per;
        int t3[3] = {tile % m.tdims[0], (tile / m.tdims[0]) % m.tdims[1],
                     tile / (m.tdims[0] * m.tdims[1])};
        int i = t3[0] * T + local % T;
        int j = t3[1] * T + (local / T) % T;
        int k = t3[2] * T + local / (T * T);
        if (i < m.dims[0] && j < m.dims[1] && k < m.dims[2])
            label_fp64_t<true>(m, tile, mol_coord(m, 0, i), mol_coord(m, 1, j),
                               mol_coord(m, 2, k), cnt);
    }
    for (int c = 0; c < WC_COUNT; ++c) {
        unsigned long long v = cnt[c];
        for (int d = WAVE / 2; d > 0; d >>= 1) v += __shfl_down(v, d, WAVE);
        if (lane_id() == 0 && v) atomicAdd(&work[c], v);
    }
}

hipError_t launch_classify_work(const Mol &m, unsigned long long *work, hipStream_t st) {
    const int per = m.tile * m.tile * m.tile;
    const int tpb = CLS_BLOCK / per;
    unsigned nb = (unsigned)((m.ntiles + tpb - 1) / tpb);
    hipLaunchKernelGGL(k_classify_work, dim3(nb < 1 ? 1 : nb), dim3(CLS_BLOCK), 0, st, m, work);
    return hipGetLastError();
}

__global__ void __launch_bounds__(256) k_count_inside(const uint8_t *L, long long n,
                                                      unsigned long long *out) {
    unsigned long long c = 0;
    for (long long q = blockIdx.x * 256LL + threadIdx.x; q < n; q += (long long)gridDim.x * 256)
        c += L[q];
    for (int d = WAVE / 2; d > 0; d >>= 1) c += __shfl_down(c, d, WAVE);
    if (lane_id() == 0 && c) atomicAdd(out, c);
}

hipError_t launch_count_inside(const uint8_t *labels, long long n, unsigned long long *out,
                               hipStream_t st) {
    long long nb = (n + 255) / 256;
    if (nb > 2048) nb = 2048;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_count_inside, dim3((unsigned)nb), dim3(256), 0, st, labels, n, out);
    return hipGetLastError();
}

hipError_t launch_units(const Mol *mols_dev, const int *tile_base_dev, int nmols, long long total,
                        int order, int *cls_count, int *cls_fill, int2 *units, hipStream_t st) {
    unsigned nb = (unsigned)((total + 255) / 256);
    hipError_t e = fill_i32(cls_count, UNIT_CLASSES, 0, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_unit_count, dim3(nb), dim3(256), 0, st, mols_dev, tile_base_dev, nmols,
                       total, order, cls_count);
    hipLaunchKernelGGL(k_unit_bases, dim3(1), dim3(64), 0, st, cls_count, cls_fill);
    hipLaunchKernelGGL(k_unit_scatter, dim3(nb), dim3(256), 0, st, mols_dev, tile_base_dev, nmols,
                       total, order, cls_fill, units);
    return hipGetLastError();
}

// Uncertain-point queues of a batch: counters zeroed (a kernel, so that the
// recorded graph holds no memset) and gathered for one read-back.
__global__ void k_unc_zero(const Mol *mols, int nmols) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < nmols) *mols[q].unc_n = 0;
}

__global__ void k_unc_gather(const Mol *mols, int nmols, int *out) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < nmols) out[q] = *mols[q].unc_n;
}

// Diagnostic word k of every molecule of a batch, gathered for one read-back.
__global__ void k_diag_gather(const Mol *mols, int nmols, int k, int *out) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < nmols) out[q] = mols[q].diag[k];
}

hipError_t launch_diag_gather(const Mol *mols_dev, int nmols, int k, int *out, hipStream_t st) {
    hipLaunchKernelGGL(k_diag_gather, dim3((nmols + 255) / 256), dim3(256), 0, st, mols_dev, nmols,
                       k, out);
    return hipGetLastError();
}

// Exactly re-decided labels written back: labels[idx[q]] = val[q].
__global__ void k_scatter_labels(const long long *idx, const uint8_t *val, int n,
                                 uint8_t *labels) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) labels[idx[q]] = val[q];
}

hipError_t launch_unc_zero(const Mol *mols_dev, int nmols, hipStream_t st) {
    hipLaunchKernelGGL(k_unc_zero, dim3((nmols + 255) / 256), dim3(256), 0, st, mols_dev, nmols);
    return hipGetLastError();
}

hipError_t launch_unc_gather(const Mol *mols_dev, int nmols, int *out, hipStream_t st) {
    hipLaunchKernelGGL(k_unc_gather, dim3((nmols + 255) / 256), dim3(256), 0, st, mols_dev, nmols,
                       out);
    return hipGetLastError();
}

hipError_t launch_scatter_labels(const long long *idx, const uint8_t *val, int n, uint8_t *labels,
                                 hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter_labels, dim3((n + 255) / 256), dim3(256), 0, st, idx, val, n,
                       labels);
    return hipGetLastError();
}

int classify_batch_blocks_per_cu(bool fp32) {
    int nb = 0;
    if (fp32)
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_classify_batch<true>, CLS_THREADS, 0);
    else
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_classify_batch<false>, CLS_THREADS, 0);
    return nb > 0 ? nb : 1;
}

hipError_t launch_classify_batch(const Mol *mols_dev, int nmols, uint8_t *const *labels_dev,
                                 const int2 *units, int nunits, int *head, int nblocks, bool fp32,
                                 hipStream_t st) {
    hipError_t e = fill_i32(head, 1, 0, st);
    if (e == hipSuccess) e = launch_unc_zero(mols_dev, nmols, st);
    if (e != hipSuccess) return e;
    if (fp32)
        hipLaunchKernelGGL(k_classify_batch<true>, dim3(nblocks), dim3(CLS_THREADS), 0, st,
                           mols_dev, labels_dev, units, nunits, head);
    else
        hipLaunchKernelGGL(k_classify_batch<false>, dim3(nblocks), dim3(CLS_THREADS), 0, st,
                           mols_dev, labels_dev, units, nunits, head);
    return hipGetLastError();
}

hipError_t launch_classify(const Mol &m, bool fp32, uint8_t *labels, hipStream_t st) {
    int nb = (m.ntiles + NXCD - 1) / NXCD * NXCD;
    if (fp32)
        hipLaunchKernelGGL(k_classify<true>, dim3(nb), dim3(CLS_THREADS), 0, st, m, labels, nb);
    else
        hipLaunchKernelGGL(k_classify<false>, dim3(nb), dim3(CLS_THREADS), 0, st, m, labels, nb);
    return hipGetLastError();
}

}  // namespace eses
