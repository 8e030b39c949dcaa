// Stage 3: intersections of the SES with grid edges (eq. 3-4).
//
// (a) Crossing edges: a streaming pass over the label array finds every axis
//     edge whose end labels differ; a block-level prefix sum plus a scan of
//     block counts gives each edge its slot, so keys come out ascending.
// (b) Roots: along s + u h e_axis, the roots in [0, 1] of every surface that
//     can carry the boundary of M there -- van der Waals spheres (convex),
//     tori of radius rho around exposed circles (saddle), probe spheres
//     around exposed concave probe positions (concave) -- are found, sorted,
//     and the intervals walked from s.  u* is the start of the first
//     interval whose label differs from Inside[s]; lambda = 1 - u*.  Edges
//     are processed in chunks of one tile (a workgroup per chunk, the tile's
//     surfaces staged in LDS).
#include <algorithm>
#include <atomic>

#include "eses_device.h"
#include "launch.h"

namespace eses {

constexpr int EDGE_BLOCK = 256;

// Work counters of the statistics pass of the root kernel.
enum EdgeCounter {
    EC_EDGES = 0,
    EC_REACH_SPHERE,   // reach tests of van der Waals and probe spheres
    EC_REACH_TORUS,    // reach tests of tori
    EC_QUAD,           // sphere quadratics solved
    EC_QUARTIC,        // torus quartics set up
    EC_HORNER_FLOPS,   // flops of polynomial evaluations in the quartic solver
    EC_CUT,            // admissibility half-space tests of roots
    EC_LABEL,          // interval labels evaluated
    EC_L_ATOM,         // the label evaluations' tests (as in classification)
    EC_L_VERTEX,
    EC_L_FACE,
    EC_L_FACE_CUT,
    EC_L_CIRCLE,
    EC_L_CIRCLE_CUT,
    EC_L_SHELL,        // (label_fp64_t's case-3 tally; not reported)
    EC_CONE,           // cut planes tested against an edge's direction cone
    EC_COUNT
};
// label_fp64_t tallies into cnt + EC_L_ATOM with the classification's layout
static_assert(EC_L_CIRCLE_CUT - EC_L_ATOM == WC_CIRCLE_CUT - WC_ATOM &&
                  EC_L_SHELL - EC_L_ATOM == WC_CASE_SHELL - WC_ATOM &&
                  EC_L_FACE_CUT - EC_L_ATOM == WC_FACE_CUT - WC_ATOM,
              "edge label counters must mirror the classification counters");

__device__ inline int edge_flags(const uint8_t *L, long long idx, int i, int j, int k, int nx,
                                 int ny, int nz) {
    uint8_t a = L[idx];
    int f = 0;
    if (i + 1 < nx && L[idx + 1] != a) f |= 1;
    if (j + 1 < ny && L[idx + nx] != a) f |= 2;
    if (k + 1 < nz && L[idx + (long long)nx * ny] != a) f |= 4;
    return f;
}

// Each thread takes EDGE_PPT consecutive points (in index order), each block
// EDGE_BLOCK x EDGE_PPT of them, so that the per-block scan is amortised;
// counts and keys come out in point order.
constexpr int EDGE_PPT = 8;

__device__ inline void point_ijk(long long idx, int nx, int ny, int &i, int &j, int &k) {
    i = (int)(idx % nx);
    const long long r = idx / nx;
    j = (int)(r % ny);
    k = (int)(r / ny);
}

// Next point after (i, j, k) in index order.
__device__ inline void point_next(int nx, int ny, int &i, int &j, int &k) {
    if (++i == nx) {
        i = 0;
        if (++j == ny) {
            j = 0;
            ++k;
        }
    }
}

// The eight labels L[a .. a + 8) as the bytes of a word (a any index; reads
// the two aligned words around it, so L must be 8-byte aligned and
// a - a % 8 + 16 <= the grid size).
__device__ inline unsigned long long label_word(const uint8_t *L, long long a) {
    const long long b = a & ~7LL;
    const int s = (int)(a - b) * 8;
    const unsigned long long lo = *(const unsigned long long *)(L + b);
    if (s == 0) return lo;
    const unsigned long long hi = *(const unsigned long long *)(L + b + 8);
    return (lo >> s) | (hi << (64 - s));
}

// Crossing-edge flags (bit a: the edge along axis a) of the EDGE_PPT points
// from idx0 (a multiple of EDGE_PPT) at (i, j, k), into fl[].  Away from the
// end of the grid and with L 8-byte aligned, the points' labels and those of
// their +x, +y and +z neighbours are read as words and compared bytewise.
__device__ inline void edge_flags8(const uint8_t *L, long long idx0, int i, int j, int k, int nx,
                                   int ny, int nz, long long npts, bool words, int *fl) {
    const long long nxy = (long long)nx * ny;
    if (words && idx0 + nxy + 16 <= npts) {
        // here every point has k + 1 < nz
        const unsigned long long a = label_word(L, idx0);
        const unsigned long long X = a ^ ((a >> 8) | ((unsigned long long)L[idx0 + 8] << 56));
        const unsigned long long Y = a ^ label_word(L, idx0 + nx);
        const unsigned long long Z = a ^ label_word(L, idx0 + nxy);
#pragma unroll
        for (int q = 0; q < EDGE_PPT; ++q) {
            const int sh = 8 * q;
            int f = ((Z >> sh) & 0xFF) ? 4 : 0;
            if (i + 1 < nx && ((X >> sh) & 0xFF)) f |= 1;
            if (j + 1 < ny && ((Y >> sh) & 0xFF)) f |= 2;
            fl[q] = f;
            point_next(nx, ny, i, j, k);
        }
        return;
    }
#pragma unroll
    for (int q = 0; q < EDGE_PPT; ++q) {
        fl[q] = idx0 + q < npts ? edge_flags(L, idx0 + q, i, j, k, nx, ny, nz) : 0;
        point_next(nx, ny, i, j, k);
    }
}

// Crossing edges of detection block blk (EDGE_BLOCK x EDGE_PPT points from
// blk's first) counted into bcount[blk].
__device__ __attribute__((always_inline)) inline void edge_count_block(const uint8_t *L, int nx, int ny, int nz, long long npts,
                                        long long blk, int *bcount, int *lds) {
    const long long idx0 = (blk * EDGE_BLOCK + threadIdx.x) * EDGE_PPT;
    const bool words = ((uintptr_t)L & 7) == 0;
    int c = 0;
    if (idx0 < npts) {
        int i, j, k, fl[EDGE_PPT];
        point_ijk(idx0, nx, ny, i, j, k);
        edge_flags8(L, idx0, i, j, k, nx, ny, nz, npts, words, fl);
#pragma unroll
        for (int q = 0; q < EDGE_PPT; ++q) c += __popc(fl[q]);
    }
    int tot;
    block_excl_scan<int, EDGE_BLOCK>(c, lds, &tot);
    if (threadIdx.x == 0) bcount[blk] = tot;
}

__global__ void __launch_bounds__(EDGE_BLOCK) k_edge_count(const uint8_t *L, int nx, int ny,
                                                           int nz, long long npts, int *bcount) {
    __shared__ int lds[EDGE_BLOCK / WAVE + 1];
    edge_count_block(L, nx, ny, nz, npts, blockIdx.x, bcount, lds);
}

// Keys of detection block blk's crossing edges, from slot wblk on (those
// below cap).  Also tallies the written edges per owning tile (tcount, zeroed
// before) and
// keeps each edge's rank among its tile's edges (rank[w]), so that grouping by
// tile needs no further atomics.  A thread takes one tally per run of its
// points in one tile; the runs of a tile's rows then meet its counter in lane
// order, which keeps the ranks close to key order (chunks of nearby edges).
__device__ __attribute__((always_inline)) inline void edge_write_block(const uint8_t *L, int nx, int ny, int nz,
                                        long long npts, long long blk, long long wblk,
                                        long long cap, long long *keys, int *tcount, int *rank,
                                        int T, int tdx, int tdy, int *lds) {
    const long long idx0 = (blk * EDGE_BLOCK + threadIdx.x) * EDGE_PPT;
    const bool words = ((uintptr_t)L & 7) == 0;
    int fl[EDGE_PPT], tl[EDGE_PPT];
    int c = 0;
    for (int q = 0; q < EDGE_PPT; ++q) fl[q] = tl[q] = 0;
    if (idx0 < npts) {
        int i, j, k;
        point_ijk(idx0, nx, ny, i, j, k);
        edge_flags8(L, idx0, i, j, k, nx, ny, nz, npts, words, fl);
#pragma unroll
        for (int q = 0; q < EDGE_PPT; ++q) {
            if (fl[q]) tl[q] = i / T + tdx * (j / T + tdy * (k / T));
            c += __popc(fl[q]);
            point_next(nx, ny, i, j, k);
        }
    }
    int tot;
    long long w = wblk + block_excl_scan<int, EDGE_BLOCK>(c, lds, &tot);
    // the written edges of a run of points in one tile are consecutive in w
    int trun = -1, nrun = 0;
    long long wrun = 0;
#pragma unroll
    for (int q = 0; q < EDGE_PPT; ++q) {
        int nwr = 0;
        const long long w0 = w;
        for (int a = 0; a < 3; ++a)
            if (fl[q] & (1 << a)) {
                if (w < cap) {
                    keys[w] = 3 * (idx0 + q) + a;
                    ++nwr;
                }
                ++w;
            }
        if (nwr) {
            if (tl[q] != trun) {
                if (nrun) {
                    const int r0 = atomicAdd(&tcount[trun], nrun);
                    for (int e = 0; e < nrun; ++e) rank[wrun + e] = r0 + e;
                }
                trun = tl[q];
                wrun = w0;
                nrun = 0;
            }
            nrun += nwr;
        }
    }
    if (nrun) {
        const int r0 = atomicAdd(&tcount[trun], nrun);
        for (int e = 0; e < nrun; ++e) rank[wrun + e] = r0 + e;
    }
}

__global__ void __launch_bounds__(EDGE_BLOCK) k_edge_write(const uint8_t *L, int nx, int ny,
                                                           int nz, long long npts,
                                                           const long long *boff, long long cap,
                                                           long long *keys, int *tcount,
                                                           int *rank, int T, int tdx, int tdy) {
    __shared__ int lds[EDGE_BLOCK / WAVE + 1];
    edge_write_block(L, nx, ny, nz, npts, blockIdx.x, boff[blockIdx.x], cap, keys, tcount, rank,
                     T, tdx, tdy, lds);
}

// ------------------------------------------------------------ root finding

// The polynomial c of degree DEG (ascending coefficients) at u.  The degree
// is a template argument so that the coefficients stay in registers.
template <int DEG>
__device__ inline double horner(const double (&c)[DEG + 1], double u) {
    double v = c[DEG];
#pragma unroll
    for (int q = DEG - 1; q >= 0; --q) v = v * u + c[q];
    return v;
}

// Root of the polynomial c (degree DEG) in [lo, hi] where its values at the
// ends (flo, fhi) have opposite signs: from the secant point of the ends,
// Newton steps kept inside a shrinking bracket, bisection when a step leaves
// it.
template <bool CNT, int DEG>
__device__ double bracket_root(const double (&c)[DEG + 1], double lo, double hi, double flo,
                               double fhi, unsigned long long *cnt) {
    double d[DEG];
#pragma unroll
    for (int q = 1; q <= DEG; ++q) d[q - 1] = q * c[q];
    double x = lo + (hi - lo) * (flo / (flo - fhi));
    if (!(x > lo && x < hi)) x = 0.5 * (lo + hi);
    for (int it = 0; it < 128; ++it) {
        if (CNT) cnt[EC_HORNER_FLOPS] += 4 * DEG + 4;  // f, f' and the step
        double f = horner<DEG>(c, x);
        if (f == 0.0) return x;
        if ((f < 0.0) == (flo < 0.0)) lo = x;
        else hi = x;
        double df = horner<DEG - 1>(d, x);
        double xn = x - f / df;
        if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
        if (fabs(xn - x) <= 1e-17 || hi - lo <= 2e-16) return xn;
        x = xn;
    }
    return x;
}

// Real roots in [0, 1] of a u^2 + b u + c (a > 0), numerically stable form.
// A root within END_SLACK outside an end counts as a root at that end: a
// surface through an end point (exactly, where its label is a tie decided
// exactly) then still owns the crossing there; a breakpoint at an end that
// the surface misses only splits off an empty interval.
constexpr double END_SLACK = 1e-9;

__device__ inline double clamp01(double u) { return fmin(1.0, fmax(0.0, u)); }

__device__ inline int quad01(double a, double b, double c, double &ra, double &rb) {
    double disc = b * b - 4.0 * a * c;
    if (disc < 0.0) return 0;
    double sd = sqrt(disc);
    double q = -0.5 * (b + copysign(sd, b));
    double r1 = q / a;
    double r2 = q != 0.0 ? c / q : r1;
    const bool in1 = r1 >= -END_SLACK && r1 <= 1.0 + END_SLACK;
    const bool in2 = r2 >= -END_SLACK && r2 <= 1.0 + END_SLACK;
    r1 = clamp01(r1);
    r2 = clamp01(r2);
    const bool two = in2 && !(in1 && r2 == r1);
    // the roots in order of (r1, r2), the kept ones first
    ra = in1 ? r1 : r2;
    rb = r2;
    return (in1 ? 1 : 0) + (two ? 1 : 0);
}

// Real roots in [0, 1] of the quartic g (ascending coefficients), passed to
// emit in increasing order: the roots of g'' split [0, 1] into intervals
// where g' is monotone, the root of g' found in each splits it further into
// intervals where g is monotone, and each sign change of g on those is
// refined by bracket_root.  Both stages run in one loop, without lists, so
// that each refinement is a single call site.
template <bool CNT, class Emit>
__device__ void quartic01(const double (&g)[5], Emit emit, unsigned long long *cnt) {
    // interior roots of g'' (sorted), 1.0 standing in for a missing one
    double x1 = 1.0, x2 = 1.0;
    {
        double a = 12.0 * g[4], b = 6.0 * g[3], c = 2.0 * g[2];
        double r0 = 2.0, r1 = 2.0;
        if (a != 0.0) {
            double disc = b * b - 4.0 * a * c;
            if (disc > 0.0) {
                double sd = sqrt(disc);
                double q = -0.5 * (b + copysign(sd, b));
                r0 = q / a;
                if (q != 0.0) r1 = c / q;
            }
        } else if (b != 0.0) {
            r0 = -c / b;
        }
        bool in0 = r0 > 0.0 && r0 < 1.0, in1 = r1 > 0.0 && r1 < 1.0;
        if (in0 && in1) {
            x1 = fmin(r0, r1);
            x2 = fmax(r0, r1);
        } else if (in0) {
            x1 = r0;
        } else if (in1) {
            x1 = r1;
        }
    }
    const double d1[4] = {g[1], 2.0 * g[2], 3.0 * g[3], 4.0 * g[4]};
    // An interior critical point where g vanishes to within rounding is a
    // root of even multiplicity: a line through the self-intersection of a
    // spindle torus on its axis, where the quartic is a perfect square.
    const double tol =
        1e-12 * (fabs(g[0]) + fabs(g[1]) + fabs(g[2]) + fabs(g[3]) + fabs(g[4]));
    double ca = 0.0;                 // last critical point of g (or 0)
    double fca = horner<4>(g, 0.0);  // g there
    // g vanishing at an end to within rounding: a root at that end (the
    // segment starts or ends on the torus)
    if (fabs(fca) <= tol) emit(0.0);
#pragma unroll 1
    for (int q = 0; q < 4; ++q) {
        // next critical point of g from the g' interval q; q == 3: the end 1
        double cp = 1.0;
        bool have = true, interior = q < 3;
        if (interior) {
            double a = q == 0 ? 0.0 : q == 1 ? x1 : x2;
            double b = q == 0 ? x1 : q == 1 ? x2 : 1.0;
            have = false;
            if (b > a) {
                double fa = horner<3>(d1, a), fb = horner<3>(d1, b);
                if (CNT) cnt[EC_HORNER_FLOPS] += 12;
                if (fa == 0.0 && a > 0.0) {
                    cp = a;
                    have = true;
                } else if (fa != 0.0 && fb != 0.0 && ((fa < 0.0) != (fb < 0.0))) {
                    cp = bracket_root<CNT, 3>(d1, a, b, fa, fb, cnt);
                    have = true;
                }
            }
        }
        if (!have || !(cp > ca)) continue;
        double fb = horner<4>(g, cp);
        if (CNT) cnt[EC_HORNER_FLOPS] += 16;
        if (fb == 0.0) emit(cp);
        else if (fca != 0.0 && ((fca < 0.0) != (fb < 0.0)))
            emit(bracket_root<CNT, 4>(g, ca, cp, fca, fb, cnt));
        if (fb != 0.0 && fabs(fb) <= tol) emit(cp);
        ca = cp;
        fca = fb;
    }
}

// ------------------------------------------------ admissibility of roots

// Every cut of cuts[b, e) passes for the direction p (scaled by s):
// p . v <= s v.w.  UNROLL: four cuts are fetched before they are tested, so
// that their loads overlap.  cc: the counter of the tests (statistics pass).
template <bool CNT, bool UNROLL = false>
__device__ inline bool cuts_pass(const double4 *cuts, int b, int e, double px, double py,
                                 double pz, double s, unsigned long long *cc) {
    int c = b;
    for (; UNROLL && c + 4 <= e; c += 4) {
        double4 v0 = cuts[c], v1 = cuts[c + 1], v2 = cuts[c + 2], v3 = cuts[c + 3];
        if (CNT) *cc += 4;
        bool out = (px * v0.x + py * v0.y + pz * v0.z > s * v0.w) |
                   (px * v1.x + py * v1.y + pz * v1.z > s * v1.w) |
                   (px * v2.x + py * v2.y + pz * v2.z > s * v2.w) |
                   (px * v3.x + py * v3.y + pz * v3.z > s * v3.w);
        if (out) return false;
    }
    for (; c < e; ++c) {
        double4 v = cuts[c];
        if (CNT) ++*cc;
        if (px * v.x + py * v.y + pz * v.z > s * v.w) return false;
    }
    return true;
}

// A point y of the sphere S_i seen from x along c_i -> x is admissible iff
// (x - c_i) . v_k <= |x - c_i| tau_k for every cut of the face;
// pass(px, py, pz, s) runs the face's cut tests.
template <class Pass>
__device__ inline bool face_admissible(Pass pass, double dx, double dy, double dz) {
    double d = sqrt(dx * dx + dy * dy + dz * dz);
    return pass(dx, dy, dz, d);
}

// The circle point nearest to x (w = x - o) is admissible iff
// w_perp . u_k <= |w_perp| T_k for every cut of the circle.
template <class Pass>
__device__ inline bool circle_admissible(Pass pass, double4 n, double wx, double wy, double wz) {
    double t = wx * n.x + wy * n.y + wz * n.z;
    double px = wx - t * n.x, py = wy - t * n.y, pz = wz - t * n.z;
    double pb = sqrt(px * px + py * py + pz * pz);
    if (!(pb > 0.0)) {
        perp_unit(n.x, n.y, n.z, px, py, pz);
        pb = 1.0;
    }
    return pass(px, py, pz, pb);
}

__device__ inline void sort3(int &a, int &b, int &c) {
    int t;
    if (a > b) { t = a; a = b; b = t; }
    if (b > c) { t = b; b = c; c = t; }
    if (a > b) { t = a; a = b; b = t; }
}


// Surface parameters as staged: spheres (van der Waals face, probe) as
// centre + radius; tori as circle centre + radius R and circle normal n.
struct SurfParams {
    double4 c;
    double4 n;
};

__device__ inline SurfParams surf_params(const Mol &m, int key) {
    const int type = key >> 28, id = key & ((1 << 28) - 1);
    SurfParams p;
    p.n = make_double4(0.0, 0.0, 0.0, 0.0);
    if (type == 1) {
        p.c = m.atom[m.face_atom[id]];
    } else if (type == 3) {
        double4 v = m.vert_p[id];
        p.c = make_double4(v.x, v.y, v.z, m.rho);
    } else {
        int ci = m.ec_circ[id];
        p.c = m.circ_oR[ci];
        p.n = m.circ_n[ci];
    }
    return p;
}

// Whether the surface can cross the edge: the distance from the edge's
// midpoint to the surface is at most `half` (distance to a set is
// 1-Lipschitz, so a crossing on the edge puts the midpoint within h/2).
__device__ inline bool surf_reaches(int type, const SurfParams &p, double rho, const double *mid,
                                    double half) {
    if (type != 2) {
        double r = p.c.w;
        double dm2 = sq(mid[0] - p.c.x) + sq(mid[1] - p.c.y) + sq(mid[2] - p.c.z);
        return !(dm2 > sq(r + half) || (r > half && dm2 < sq(r - half)));
    }
    double dm0 = mid[0] - p.c.x, dm1 = mid[1] - p.c.y, dm2 = mid[2] - p.c.z;
    double tm = dm0 * p.n.x + dm1 * p.n.y + dm2 * p.n.z;
    double bm = sqrt(fmax(0.0, dm0 * dm0 + dm1 * dm1 + dm2 * dm2 - tm * tm));
    double dc2 = tm * tm + sq(bm - p.c.w);  // squared distance of the midpoint from the circle
    return !(dc2 > sq(rho + half) || (rho > half && dc2 < sq(rho - half)));
}

// As surf_reaches, and in *rel whether the surface's candidate test of
// eq. (2) can hold at some point of the edge: a probe within rho, a face's
// projection within rho (|x - c| < r + 2 rho), a circle within rho.
__device__ inline bool surf_reaches_rel(int type, const SurfParams &p, double rho,
                                        const double *mid, double half, bool *rel) {
    if (type != 2) {
        double r = p.c.w;
        double dm2 = sq(mid[0] - p.c.x) + sq(mid[1] - p.c.y) + sq(mid[2] - p.c.z);
        *rel = dm2 < sq((type == 1 ? r + 2.0 * rho : rho) + half);
        return !(dm2 > sq(r + half) || (r > half && dm2 < sq(r - half)));
    }
    double dm0 = mid[0] - p.c.x, dm1 = mid[1] - p.c.y, dm2 = mid[2] - p.c.z;
    double tm = dm0 * p.n.x + dm1 * p.n.y + dm2 * p.n.z;
    double bm = sqrt(fmax(0.0, dm0 * dm0 + dm1 * dm1 + dm2 * dm2 - tm * tm));
    double dc2 = tm * tm + sq(bm - p.c.w);
    *rel = dc2 < sq(rho + half);
    return !(dc2 > sq(rho + half) || (rho > half && dc2 < sq(rho - half)));
}

// A staged sphere (van der Waals face or probe) keeps in n the squared
// bounds of surf_reaches_rel for edges of half-length `half`: the outer
// radius, the inner one (-1 when there is none) and the candidate's reach.
__device__ inline SurfParams sphere_reach_bounds(SurfParams p, int type, double rho,
                                                 double half) {
    if (type == 2) return p;
    const double r = p.c.w;
    p.n = make_double4(sq(r + half), r > half ? sq(r - half) : -1.0,
                       sq((type == 1 ? r + 2.0 * rho : rho) + half), 0.0);
    return p;
}

// surf_reaches_rel on a staged surface (spheres with their bounds in n).
__device__ inline bool staged_reaches_rel(int type, const SurfParams &p, double rho,
                                          const double *mid, double half, bool *rel) {
    if (type == 2) return surf_reaches_rel(type, p, rho, mid, half, rel);
    const double dm2 = sq(mid[0] - p.c.x) + sq(mid[1] - p.c.y) + sq(mid[2] - p.c.z);
    *rel = dm2 < p.n.z;
    return !(dm2 > p.n.x || dm2 < p.n.y);
}

// Roots in [0, 1] of one surface along the edge x(u) = xs + u h e, each
// passed to sink(u): spheres |x(u) - c|^2 = r^2 (a quadratic), tori
// (|w|^2 + R^2 - rho^2)^2 = 4 R^2 |w_perp|^2 of the circle's points at
// distance rho (a quartic; both branches, the far one is dropped later).
template <bool CNT, class Sink>
__device__ void surface_roots(int type, const SurfParams &p, double h, double rho,
                              const double *e, const double *xs, Sink sink,
                              unsigned long long *cnt) {
    const double w0[3] = {xs[0] - p.c.x, xs[1] - p.c.y, xs[2] - p.c.z};
    const double ww = w0[0] * w0[0] + w0[1] * w0[1] + w0[2] * w0[2];
    const double we = w0[0] * e[0] + w0[1] * e[1] + w0[2] * e[2];
    if (type != 2) {
        if (CNT) ++cnt[EC_QUAD];
        double r = p.c.w;
        double ra, rb;
        int n = quad01(h * h, 2.0 * h * we, ww - r * r, ra, rb);
        if (n > 0) sink(ra);
        if (n > 1) sink(rb);
        return;
    }
    const double4 nn = p.n;
    const double R = p.c.w;
    const double t0 = w0[0] * nn.x + w0[1] * nn.y + w0[2] * nn.z;
    const double ne = nn.x * e[0] + nn.y * e[1] + nn.z * e[2];
    const double RR = R * R;
    const double a0 = ww + RR - rho * rho, a1 = 2.0 * h * we, a2 = h * h;
    const double b0 = ww - t0 * t0, b1 = 2.0 * h * (we - t0 * ne), b2 = h * h * (1.0 - ne * ne);
    const double g[5] = {a0 * a0 - 4.0 * RR * b0, 2.0 * a0 * a1 - 4.0 * RR * b1,
                         a1 * a1 + 2.0 * a0 * a2 - 4.0 * RR * b2, 2.0 * a1 * a2, a2 * a2};
    if (CNT) ++cnt[EC_QUARTIC];
    quartic01<CNT>(g, sink, cnt);
}

// Whether a root is kept: only if the point of A that would put it on the
// boundary is admissible, the radial projection onto the exposed face (van
// der Waals roots) or the nearest point of the exposed circle on the near
// branch of the torus (torus roots).  Every label change lies on such a
// point, so dropping the others is exact.  Probe roots are always kept.
template <class Pass>
__device__ bool root_admissible(const Mol &m, int key, const SurfParams &p, Pass pass, double u,
                                const double *e, const double *xs) {
    const int type = key >> 28;
    if (type == 3) return true;
    const double s = u * m.h;
    const double x0 = xs[0] - p.c.x + s * e[0], x1 = xs[1] - p.c.y + s * e[1],
                 x2 = xs[2] - p.c.z + s * e[2];
    if (type == 1) return face_admissible(pass, x0, x1, x2);
    const double4 nn = p.n;
    const double R = p.c.w, rho = m.rho;
    double tt = x0 * nn.x + x1 * nn.y + x2 * nn.z;
    double bb = sqrt(fmax(0.0, x0 * x0 + x1 * x1 + x2 * x2 - tt * tt));
    double near = fabs(sq(bb - R) + tt * tt - rho * rho);
    double far = fabs(sq(bb + R) + tt * tt - rho * rho);
    return near <= far && circle_admissible(pass, nn, x0, x1, x2);
}

// The cut planes of surface `key` in global memory: [*cb, *ce) of the
// returned array (none for probes).
__device__ inline const double4 *global_cuts(const Mol &m, int key, int *cb, int *ce) {
    const int type = key >> 28, id = key & ((1 << 28) - 1);
    const int *fo = m.face_cut_off, *eo = m.ec_cut_off;
    const double4 *fc = m.face_cut, *ec = m.ec_cut;
    if (type == 1 || type == 2) {
        const int *o = type == 1 ? fo : eo;
        *cb = o[id];
        *ce = o[id + 1];
        return type == 1 ? fc : ec;
    }
    *cb = *ce = 0;
    return fc;
}

// Position and end labels of crossing edge `key` (3 * point index + axis).
struct EdgeGeom {
    double xs[3];
    double e[3];
    int tile, Ls, Lt;
};

__device__ inline EdgeGeom edge_geom(const Mol &m, const uint8_t *L, long long key) {
    EdgeGeom G;
    const int axis = (int)(key % 3);
    const long long idx = key / 3;
    const int nx = m.dims[0], ny = m.dims[1];
    int i0, i1, i2;
    grid_ijk(idx, nx, ny, i0, i1, i2);
    const long long step = axis == 0 ? 1 : axis == 1 ? (long long)nx : (long long)nx * ny;
    G.Ls = L[idx];
    G.Lt = L[idx + step];
    G.tile = i0 / m.tile + m.tdims[0] * (i1 / m.tile + m.tdims[1] * (i2 / m.tile));
    G.e[0] = axis == 0 ? 1.0 : 0.0;
    G.e[1] = axis == 1 ? 1.0 : 0.0;
    G.e[2] = axis == 2 ? 1.0 : 0.0;
    G.xs[0] = mol_coord(m, 0, i0);
    G.xs[1] = mol_coord(m, 1, i1);
    G.xs[2] = mol_coord(m, 2, i2);
    return G;
}

// The walk over the sorted roots u[0..n) (keys k[]) of one edge: the label
// is constant between consecutive distinct roots; the first interval has
// Inside[s] and the last Inside[t] unless a root sits exactly on that end,
// the others are evaluated at their midpoints.  Returns u*, the start of the
// first interval whose label differs from Inside[s] (1 if none: the change
// is at t itself), and the owner key of that position (the smallest key of
// the roots there).  LabelFn(x, y, z) evaluates eq. (2).
template <bool CNT, class RootAt, class LabelFn>
__device__ double walk_roots(int n, RootAt root_at, int Ls, int Lt, const double *xs,
                             const double *e, double h, LabelFn label, int *owner,
                             unsigned long long *cnt) {
    double u0 = 0.0, ulast = 0.0;
    int k0 = 0;
    if (n > 0) {
        root_at(0, u0, k0);
        root_at(n - 1, ulast, k0);
    }
    const bool root0 = n > 0 && u0 == 0.0;
    const bool root1 = n > 0 && ulast == 1.0;
    double prev = 0.0;
    int prev_key = -1;
    for (int r = 0; r <= n; ++r) {
        double next = 1.0;
        int kn = -1;
        if (r < n) root_at(r, next, kn);
        if (next > prev) {
            int lab;
            if (prev == 0.0 && !root0) {
                lab = Ls;
            } else if (r == n && !root1) {
                lab = Lt;
            } else {
                double um = 0.5 * (prev + next) * h;
                if (CNT) ++cnt[EC_LABEL];
                lab = label(xs[0] + um * e[0], xs[1] + um * e[1], xs[2] + um * e[2]);
            }
            if (lab != Ls) {
                *owner = prev_key;
                return prev;
            }
        }
        if (r < n && (prev_key < 0 || next > prev)) prev_key = kn;
        if (next > prev) prev = next;
    }
    *owner = prev_key;
    return 1.0;
}

// The record of edge q: lambda = 1 - u*, the outward unit normal of the
// owning surface at x(u*), its patch type and atoms (original indices).
__device__ inline void write_record(const Mol &m, long long q, const EdgeGeom &G, double ustar,
                                    int owner_key, double *lam, double *nrm, uint8_t *ptype,
                                    int *patoms) {
    const double us = ustar * m.h;
    const double xst[3] = {G.xs[0] + us * G.e[0], G.xs[1] + us * G.e[1], G.xs[2] + us * G.e[2]};
    double n3[3] = {0.0, 0.0, 0.0};
    int type = 0, at0 = -1, at1 = -1, at2 = -1;
    if (owner_key >= 0) {
        type = owner_key >> 28;
        const int id = owner_key & ((1 << 28) - 1);
        double y[3];
        if (type == 1) {
            const int ia = m.face_atom[id];
            double4 a = m.atom[ia];
            y[0] = xst[0] - a.x;
            y[1] = xst[1] - a.y;
            y[2] = xst[2] - a.z;
            at0 = m.orig[ia];
        } else if (type == 2) {
            int ci = m.ec_circ[id];
            double4 oR = m.circ_oR[ci];
            double4 nn = m.circ_n[ci];
            double wv[3] = {xst[0] - oR.x, xst[1] - oR.y, xst[2] - oR.z};
            double t = wv[0] * nn.x + wv[1] * nn.y + wv[2] * nn.z;
            double wp[3] = {wv[0] - t * nn.x, wv[1] - t * nn.y, wv[2] - t * nn.z};
            double b = sqrt(wp[0] * wp[0] + wp[1] * wp[1] + wp[2] * wp[2]);
            double u[3];
            if (b > 0.0) {
                u[0] = wp[0] / b;
                u[1] = wp[1] / b;
                u[2] = wp[2] / b;
            } else {
                perp_unit(nn.x, nn.y, nn.z, u[0], u[1], u[2]);
            }
            y[0] = oR.x + oR.w * u[0] - xst[0];
            y[1] = oR.y + oR.w * u[1] - xst[1];
            y[2] = oR.z + oR.w * u[2] - xst[2];
            at0 = min(m.orig[m.circ_i[ci]], m.orig[m.circ_j[ci]]);
            at1 = max(m.orig[m.circ_i[ci]], m.orig[m.circ_j[ci]]);
        } else {
            double4 p = m.vert_p[id];
            y[0] = p.x - xst[0];
            y[1] = p.y - xst[1];
            y[2] = p.z - xst[2];
            int4 v = m.vert_ijks[id];
            at0 = m.orig[v.x];
            at1 = m.orig[v.y];
            at2 = m.orig[v.z];
            sort3(at0, at1, at2);
        }
        double l = sqrt(y[0] * y[0] + y[1] * y[1] + y[2] * y[2]);
        if (l > 0.0)
            for (int a = 0; a < 3; ++a) n3[a] = y[a] / l;
    }
    if (owner_key < 0) atomicAdd(&m.diag[3], 1);  // no surface owns the change: reported
    lam[q] = 1.0 - ustar;
    nrm[3 * q] = n3[0];
    nrm[3 * q + 1] = n3[1];
    nrm[3 * q + 2] = n3[2];
    ptype[q] = (uint8_t)type;
    patoms[3 * q] = at0;
    patoms[3 * q + 1] = at1;
    patoms[3 * q + 2] = at2;
}

__device__ inline int edge_tile(const Mol &m, long long key) {
    int i, j, k;
    grid_ijk(key / 3, m.dims[0], m.dims[1], i, j, k);
    return i / m.tile + m.tdims[0] * (j / m.tile + m.tdims[1] * (k / m.tile));
}

// Surface count and the key of entry s of tile t's candidate surfaces:
// exposed faces, then probes, then exposed circles.
__device__ inline int tile_surfaces(const Mol &m, int t) {
    return (m.tF_off[t + 1] - m.tF_off[t]) + (m.tV_off[t + 1] - m.tV_off[t]) +
           (m.tC_off[t + 1] - m.tC_off[t]);
}

// (The lists' pointers are read before the branches, so that a per-thread
// choice selects among their values rather than among fields of m.)
__device__ inline int tile_surface_key(const Mol &m, int t, int s) {
    const int *tF = m.tF, *tV = m.tV, *tC = m.tC;
    const int f0 = m.tF_off[t], nf = m.tF_off[t + 1] - f0;
    const int v0 = m.tV_off[t], nv = m.tV_off[t + 1] - v0;
    const int c0 = m.tC_off[t];
    const int *p;
    int tag;
    if (s < nf) {
        p = tF + f0 + s;
        tag = 1;
    } else if (s < nf + nv) {
        p = tV + v0 + (s - nf);
        tag = 3;
    } else {
        p = tC + c0 + (s - nf - nv);
        tag = 2;
    }
    return (tag << 28) | *p;
}

// ------------------------------------------------ roots, chunks of one tile
//
// A workgroup takes up to CH_EDGES crossing edges of one tile (a chunk) and
// the tile's candidate surfaces, staged in LDS.  Threads run over the
// (edge, surface) pairs for the reach test; the pairs that pass are queued
// (tori and spheres apart, so that waves solve one kind), one thread per
// queued pair solves it and keeps its admissible roots; the roots are then
// grouped by edge and one thread per edge sorts its roots and walks the
// intervals, evaluating eq. (2) where an interval's label is not implied by
// the end labels.
constexpr int CH_EDGES = 64;
constexpr int CH_THREADS = 256;
constexpr int CH_SURF = 128;    // surfaces staged per pass
constexpr int CH_ROOTS = 512;   // admissible roots per chunk
constexpr int CH_SLOTS = 4;     // roots of one quartic before the admissibility test
constexpr int CH_ATOMS = 192;   // tile atoms staged for the labels
constexpr int CH_CUTS = 384;    // cut planes of the staged surfaces
constexpr int CH_Q = 256;       // label queries of a chunk evaluated together
constexpr int CH_TILE_UNITS = 3;  // tiles per block for whole-tile units

struct ChunkLds {
    SurfParams sp[CH_SURF];
    double4 atoms[CH_ATOMS];
    double4 cut[CH_CUTS];
    double xs[CH_EDGES][3];
    double mid[CH_EDGES][3];  // edge midpoints
    union {
        // staging: the surfaces' first global cut, the offsets of their
        // (surface, cut) pairs and the cursors of their kept cuts
        struct {
            int ccb[CH_SURF];
            int coff[CH_SURF + 1];
            int ccur[CH_SURF];
            // each surface's cone over the tile in FP32 (axis, sin; cos, or
            // -1 for every direction)
            float4 cna[CH_SURF];
            float cnc[CH_SURF];
        } st;
        // solve phase: roots of one quartic per thread
        double slot[CH_SLOTS][CH_THREADS];
        // walk phase: label queries (edge, midpoint parameter), their test
        // results (1 van der Waals ball, 2 SAS ball, 4 candidate within rho)
        // and the offsets of their (query, candidate) tests
        struct {
            double qu[CH_Q];
            int qflag[CH_Q];
            int qoff[CH_Q + 1];
            int qskip[CH_Q];  // mask bits before the query's tests of a phase
            unsigned char qe[CH_Q];
        } q;
    };
    double fu[CH_ROOTS];
    int fk[CH_ROOTS];
    int skey[CH_SURF];
    unsigned char sdead[CH_SURF];  // surface inadmissible throughout the tile
    int2 crange[CH_SURF];  // cut range in `cut`, or (-1 - begin, end) in global memory
    long long eq[CH_EDGES];
    int einfo[CH_EDGES];  // axis | Ls << 2 | Lt << 3
    int ecount[CH_EDGES + 1];
    int eoff[CH_EDGES + 1];
    int scan[CH_THREADS / WAVE + 1];
    // per wavefront: queued (edge, surface) pairs, spheres [0] and tori [1]
    unsigned short wq[CH_THREADS / WAVE][2][2 * WAVE];
    unsigned short perm[CH_ROOTS];
    unsigned char fe[CH_ROOTS];
    // per edge: the staged atoms and surfaces whose label test can hold
    // somewhere on the edge (bit masks over the staged arrays)
    unsigned long long amask[CH_EDGES][CH_ATOMS / 64];
    unsigned long long smask[CH_EDGES][CH_SURF / 64];
    int nf, ovf, tile, fb_base, nq;
};

// The cut tests of staged surface s, on its planes in LDS or, where they did
// not fit, in global memory.
template <bool CNT>
__device__ inline bool staged_cuts_pass(const Mol &m, const ChunkLds &S, int s, double px,
                                        double py, double pz, double sc,
                                        unsigned long long *cc) {
    const int2 r = S.crange[s];
    if (r.x >= 0) return cuts_pass<CNT>(S.cut, r.x, r.y, px, py, pz, sc, cc);
    const double4 *g = (S.skey[s] >> 28) == 1 ? m.face_cut : m.ec_cut;
    return cuts_pass<CNT>(g, -1 - r.x, r.y, px, py, pz, sc, cc);
}

// Inside/outside of x (eq. 2) from the staged tile data: the first nAst
// atoms of the tile's atom list in LDS (the rest read from global memory),
// the surfaces (exposed faces [0, nF), probes [nF, nF + nV), exposed
// circles [nF + nV, ns)) and their cuts.  The same tests as label_fp64_t.
template <bool CNT>
__device__ int label_chunk(const Mol &m, const ChunkLds &S, int tile, int nAst, int nF, int nV,
                           int ns, double x, double y, double z, unsigned long long *cnt) {
    const double rho = m.rho;
    const double rho2 = rho * rho;
    bool inU = false;
    for (int q = 0; q < nAst; ++q) {
        double4 a = S.atoms[q];
        double dx = x - a.x, dy = y - a.y, dz = z - a.z;
        double d2 = dx * dx + dy * dy + dz * dz;
        if (CNT) ++cnt[EC_L_ATOM];
        if (d2 <= a.w * a.w) return 1;
        double s = a.w + rho;
        inU |= d2 < s * s;
    }
    for (int q = m.tA_off[tile] + nAst, e = m.tA_off[tile + 1]; q < e; ++q) {
        double4 a = m.atom[m.tA[q]];
        double dx = x - a.x, dy = y - a.y, dz = z - a.z;
        double d2 = dx * dx + dy * dy + dz * dz;
        if (CNT) ++cnt[EC_L_ATOM];
        if (d2 <= a.w * a.w) return 1;
        double s = a.w + rho;
        inU |= d2 < s * s;
    }
    if (!inU) return 0;
    for (int q = nF; q < nF + nV; ++q) {
        double4 p = S.sp[q].c;
        double dx = x - p.x, dy = y - p.y, dz = z - p.z;
        if (CNT) ++cnt[EC_L_VERTEX];
        if (dx * dx + dy * dy + dz * dz < rho2) return 0;
    }
    for (int q = 0; q < nF; ++q) {
        double4 a = S.sp[q].c;
        double dx = x - a.x, dy = y - a.y, dz = z - a.z;
        double d2 = dx * dx + dy * dy + dz * dz;
        double sr = a.w + 2.0 * rho;
        if (CNT) ++cnt[EC_L_FACE];
        if (!(d2 < sr * sr)) continue;
        double d = sqrt(d2);
        if (staged_cuts_pass<CNT>(m, S, q, dx, dy, dz, d, CNT ? cnt + EC_L_FACE_CUT : nullptr))
            return 0;
    }
    for (int q = nF + nV; q < ns; ++q) {
        double4 oR = S.sp[q].c;
        double4 n = S.sp[q].n;
        double wx = x - oR.x, wy = y - oR.y, wz = z - oR.z;
        double t = wx * n.x + wy * n.y + wz * n.z;
        double ww = wx * wx + wy * wy + wz * wz;
        double b = sqrt(fmax(ww - t * t, 0.0));
        double R = oR.w;
        if (CNT) ++cnt[EC_L_CIRCLE];
        if (!(ww + R * R - rho2 < 2.0 * b * R)) continue;
        double px = wx, py = wy, pz = wz, pb = b;
        if (!(b > 0.0)) {
            perp_unit(n.x, n.y, n.z, px, py, pz);
            pb = 1.0;
        }
        if (staged_cuts_pass<CNT>(m, S, q, px, py, pz, pb, CNT ? cnt + EC_L_CIRCLE_CUT : nullptr))
            return 0;
    }
    return 1;
}

// label_chunk restricted to the atoms and surfaces of edge ei's masks: the
// others fail their tests everywhere on the edge (distance bounds from the
// edge's midpoint), so the result is the same.
template <bool CNT>
__device__ int label_masked(const Mol &m, const ChunkLds &S, int ei, int nF, int nV, double x,
                            double y, double z, unsigned long long *cnt) {
    const double rho = m.rho;
    const double rho2 = rho * rho;
    bool inU = false;
    for (int w = 0; w < CH_ATOMS / 64; ++w) {
        for (unsigned long long bits = S.amask[ei][w]; bits; bits &= bits - 1) {
            double4 a = S.atoms[w * 64 + __builtin_ctzll(bits)];
            double dx = x - a.x, dy = y - a.y, dz = z - a.z;
            double d2 = dx * dx + dy * dy + dz * dz;
            if (CNT) ++cnt[EC_L_ATOM];
            if (d2 <= a.w * a.w) return 1;
            double s = a.w + rho;
            inU |= d2 < s * s;
        }
    }
    if (!inU) return 0;
    for (int w = 0; w < CH_SURF / 64; ++w) {
        for (unsigned long long bits = S.smask[ei][w]; bits; bits &= bits - 1) {
            const int q = w * 64 + __builtin_ctzll(bits);
            if (q < nF) {
                double4 a = S.sp[q].c;
                double dx = x - a.x, dy = y - a.y, dz = z - a.z;
                double d2 = dx * dx + dy * dy + dz * dz;
                double sr = a.w + 2.0 * rho;
                if (CNT) ++cnt[EC_L_FACE];
                if (!(d2 < sr * sr)) continue;
                double d = sqrt(d2);
                if (staged_cuts_pass<CNT>(m, S, q, dx, dy, dz, d,
                                          CNT ? cnt + EC_L_FACE_CUT : nullptr))
                    return 0;
            } else if (q < nF + nV) {
                double4 p = S.sp[q].c;
                double dx = x - p.x, dy = y - p.y, dz = z - p.z;
                if (CNT) ++cnt[EC_L_VERTEX];
                if (dx * dx + dy * dy + dz * dz < rho2) return 0;
            } else {
                double4 oR = S.sp[q].c;
                double4 n = S.sp[q].n;
                double wx = x - oR.x, wy = y - oR.y, wz = z - oR.z;
                double t = wx * n.x + wy * n.y + wz * n.z;
                double ww = wx * wx + wy * wy + wz * wz;
                double b = sqrt(fmax(ww - t * t, 0.0));
                double R = oR.w;
                if (CNT) ++cnt[EC_L_CIRCLE];
                if (!(ww + R * R - rho2 < 2.0 * b * R)) continue;
                double px = wx, py = wy, pz = wz, pb = b;
                if (!(b > 0.0)) {
                    perp_unit(n.x, n.y, n.z, px, py, pz);
                    pb = 1.0;
                }
                if (staged_cuts_pass<CNT>(m, S, q, px, py, pz, pb,
                                          CNT ? cnt + EC_L_CIRCLE_CUT : nullptr))
                    return 0;
            }
        }
    }
    return 1;
}

// The intervals of one edge's sorted roots whose label walk_roots may
// evaluate, in its order: emit(u) with u the midpoint parameter.
template <class RootAt, class Emit>
__device__ inline void label_intervals(int n, RootAt root_at, Emit emit) {
    double u0 = 0.0, ulast = 0.0;
    int k0 = 0;
    if (n > 0) {
        root_at(0, u0, k0);
        root_at(n - 1, ulast, k0);
    }
    const bool root0 = n > 0 && u0 == 0.0;
    const bool root1 = n > 0 && ulast == 1.0;
    double prev = 0.0;
    for (int r = 0; r <= n; ++r) {
        double next = 1.0;
        int kn;
        if (r < n) root_at(r, next, kn);
        if (next > prev) {
            if (!(prev == 0.0 && !root0) && !(r == n && !root1)) emit(0.5 * (prev + next));
            prev = next;
        }
    }
}

// Position of the j-th (from 0) set bit of x, j < popcount(x): halves
// chosen by their popcounts.
__device__ inline int nth_bit(unsigned long long x, int j) {
    int pos = 0;
    unsigned v = (unsigned)x;
    const int c = __popc(v);
    if (j >= c) {
        j -= c;
        v = (unsigned)(x >> 32);
        pos = 32;
    }
#pragma unroll
    for (int w = 16; w >= 1; w >>= 1) {
        const int cw = __popc(v & ((1u << w) - 1u));
        if (j >= cw) {
            j -= cw;
            v >>= w;
            pos += w;
        }
    }
    return pos;
}

// Test j of the label query at parameter um on edge e: the j-th atom or
// surface of the edge's masks (atoms first).  Returns 1 if x lies in the
// atom's van der Waals ball, 2 if in its SAS ball only, 4 if the surface's
// candidate lies within rho; label_masked's tests, one at a time.
template <bool CNT>
__device__ int label_test(const Mol &m, const ChunkLds &S, int e, int j, double um, int nF,
                          int nV, unsigned long long *cnt) {
    const double rho = m.rho, rho2 = rho * rho, h = m.h;
    const int axis = S.einfo[e] & 3;
    const double us = um * h;
    const double x = S.xs[e][0] + us * (axis == 0 ? 1.0 : 0.0);
    const double y = S.xs[e][1] + us * (axis == 1 ? 1.0 : 0.0);
    const double z = S.xs[e][2] + us * (axis == 2 ? 1.0 : 0.0);
    int w = 0;
    unsigned long long bits = 0;
    for (; w < CH_ATOMS / 64 + CH_SURF / 64; ++w) {
        bits = w < CH_ATOMS / 64 ? S.amask[e][w] : S.smask[e][w - CH_ATOMS / 64];
        const int c = __popcll(bits);
        if (j < c) break;
        j -= c;
    }
    const int b = nth_bit(bits, j);
    if (w < CH_ATOMS / 64) {
        double4 a = S.atoms[w * 64 + b];
        double dx = x - a.x, dy = y - a.y, dz = z - a.z;
        double d2 = dx * dx + dy * dy + dz * dz;
        if (CNT) ++cnt[EC_L_ATOM];
        if (d2 <= a.w * a.w) return 1;
        double sr = a.w + rho;
        return d2 < sr * sr ? 2 : 0;
    }
    const int q = (w - CH_ATOMS / 64) * 64 + b;
    if (q < nF) {
        double4 a = S.sp[q].c;
        double dx = x - a.x, dy = y - a.y, dz = z - a.z;
        double d2 = dx * dx + dy * dy + dz * dz;
        double sr = a.w + 2.0 * rho;
        if (CNT) ++cnt[EC_L_FACE];
        if (!(d2 < sr * sr)) return 0;
        double d = sqrt(d2);
        return staged_cuts_pass<CNT>(m, S, q, dx, dy, dz, d, CNT ? cnt + EC_L_FACE_CUT : nullptr)
                   ? 4
                   : 0;
    }
    if (q < nF + nV) {
        double4 p = S.sp[q].c;
        double dx = x - p.x, dy = y - p.y, dz = z - p.z;
        if (CNT) ++cnt[EC_L_VERTEX];
        return dx * dx + dy * dy + dz * dz < rho2 ? 4 : 0;
    }
    double4 oR = S.sp[q].c;
    double4 nn = S.sp[q].n;
    double wx = x - oR.x, wy = y - oR.y, wz = z - oR.z;
    double t = wx * nn.x + wy * nn.y + wz * nn.z;
    double ww = wx * wx + wy * wy + wz * wz;
    double bb = sqrt(fmax(ww - t * t, 0.0));
    double R = oR.w;
    if (CNT) ++cnt[EC_L_CIRCLE];
    if (!(ww + R * R - rho2 < 2.0 * bb * R)) return 0;
    double px = wx, py = wy, pz = wz, pb = bb;
    if (!(bb > 0.0)) {
        perp_unit(nn.x, nn.y, nn.z, px, py, pz);
        pb = 1.0;
    }
    return staged_cuts_pass<CNT>(m, S, q, px, py, pz, pb, CNT ? cnt + EC_L_CIRCLE_CUT : nullptr)
               ? 4
               : 0;
}

// Directions of a face's or circle's candidate over a ball: the cone of
// half-angle theta (sin st, cos ct) around the unit axis; `all` when the
// ball holds the apex (every direction possible).
struct DirCone {
    double ax, ay, az, st, ct;
    bool all;
};

// The cone over ball (bc, rb): from the atom centre for a face, in the
// circle's plane from its centre for a circle (the in-plane part of a
// displacement is no longer than the displacement).
__device__ inline DirCone surface_cone(int type, const SurfParams &p, const double *bc, double rb) {
    double ax = bc[0] - p.c.x, ay = bc[1] - p.c.y, az = bc[2] - p.c.z;
    if (type == 2) {
        double t = ax * p.n.x + ay * p.n.y + az * p.n.z;
        ax -= t * p.n.x;
        ay -= t * p.n.y;
        az -= t * p.n.z;
    }
    DirCone c;
    const double L = sqrt(ax * ax + ay * ay + az * az);
    c.all = !(L > rb * (1.0 + 1e-9));
    if (c.all) {
        c.ax = c.ay = c.az = c.st = 0.0;
        c.ct = 1.0;
        return c;
    }
    c.ax = ax / L;
    c.ay = ay / L;
    c.az = az / L;
    c.st = rb / L;
    c.ct = sqrt(fmax(0.0, 1.0 - c.st * c.st));
    return c;
}

// A cut (v, tau) rejects the unit direction u iff u . v > tau.  Over the
// cone, u . v ranges between |v| cos(phi + theta) and |v| cos(phi - theta)
// (phi the angle between v and the axis, clamped to [0, pi]): cone_rejects_f
// tells whether the cut rejects every direction of the cone, cone_may_reject_f
// whether it rejects some.  The cone's parameters are rounded to FP32 (each
// within 2^-23 relative); the axis a' is rescaled by one Newton step for
// 1 / |a'| (exact to 1e-13, |a'|^2 being within 4e-7 of 1), so cp is the
// cosine, to 1e-13, of the angle between v and a direction within 2e-7 rad
// of the exact axis, and that angle is within 4e-7 rad of the exact one even
// where cp is near +-1.  Those extremes then move by less than 1e-6 |v|; a
// margin of that size, beside a small slack, keeps both decisions
// conservative (a surface is declared dead, or a cut dropped, only when the
// exact cone would do so too).
__device__ inline double cone_cos(float4 a, double4 v, double vn) {
    const double ax = a.x, ay = a.y, az = a.z;
    return (ax * v.x + ay * v.y + az * v.z) / vn * (1.5 - 0.5 * (ax * ax + ay * ay + az * az));
}

__device__ inline bool cone_rejects_f(float4 a, float ct, double4 v) {
    if (ct < 0.0f) return false;
    const double vn = sqrt(v.x * v.x + v.y * v.y + v.z * v.z);
    if (!(vn > 0.0)) return false;
    const double cp = cone_cos(a, v, vn);
    if (cp <= -(double)ct) return false;
    const double sp = sqrt(fmax(0.0, 1.0 - cp * cp));
    return vn * (cp * (double)ct - sp * (double)a.w) >
           v.w + 1e-9 * (vn + fabs(v.w)) + 1e-6 * vn;
}

__device__ inline bool cone_may_reject_f(float4 a, float ct, double4 v) {
    if (ct < 0.0f) return true;
    const double vn = sqrt(v.x * v.x + v.y * v.y + v.z * v.z);
    if (!(vn > 0.0)) return 0.0 > v.w - 1e-9;
    const double cp = cone_cos(a, v, vn);
    double best = vn;
    if (cp < (double)ct) {
        const double sp = sqrt(fmax(0.0, 1.0 - cp * cp));
        best = vn * (cp * (double)ct + sp * (double)a.w);
    }
    return best > v.w - 1e-9 * (vn + fabs(v.w)) - 1e-6 * vn;
}

// Whether some cut of staged face or circle si rejects its candidate at
// every point of the edge (the ball of radius `half` around mid).  The
// candidate's direction -- from the atom centre for a face, in the circle's
// plane from its centre for a circle -- stays within angle theta of its value
// at mid, sin theta = half / |a| (a the axis); a cut (v, tau) rejects the
// direction u iff u . v > tau, so it rejects the whole cone iff the cone does
// not reach the direction -v (phi + theta <= pi) and
//   |v| cos(phi + theta) = (a . v cos theta - |a x v| sin theta) / |a| > tau,
// phi the angle between v and a.  The test runs in FP32 on the rounded axis
// and cut: each of a . v and |a x v| is then within 1e-6 |a| |v| of its exact
// value and cos, sin theta within 1e-6, so the left side is within 1e-5 |v|;
// that margin (beside the FP64 slack of the exact test) keeps the decision
// conservative: a surface is declared dead only where the exact cone is.
template <bool CNT>
__device__ bool edge_cone_dead(const Mol &m, const ChunkLds &S, int si, int type,
                               const double *mid, double half, unsigned long long *cnt) {
    const SurfParams &p = S.sp[si];
    double ax = mid[0] - p.c.x, ay = mid[1] - p.c.y, az = mid[2] - p.c.z;
    if (type == 2) {
        double t = ax * p.n.x + ay * p.n.y + az * p.n.z;
        ax -= t * p.n.x;
        ay -= t * p.n.y;
        az -= t * p.n.z;
    }
    if (!(ax * ax + ay * ay + az * az > 4.0 * half * half)) return false;  // cone too wide
    const float fx = (float)ax, fy = (float)ay, fz = (float)az;
    const float L = sqrtf(fx * fx + fy * fy + fz * fz);
    const float iL = 1.0f / L;
    const float st = (float)half * iL, ct = sqrtf(1.0f - st * st);
    const int2 r = S.crange[si];
    const double4 *cuts = S.cut;
    int b = r.x, e = r.y;
    if (r.x < 0) {
        cuts = type == 1 ? m.face_cut : m.ec_cut;
        b = -1 - r.x;
    }
    for (int c = b; c < e; ++c) {
        const double4 v = cuts[c];
        if (CNT) ++cnt[EC_CONE];
        const float vx = (float)v.x, vy = (float)v.y, vz = (float)v.z, tau = (float)v.w;
        const float av = fx * vx + fy * vy + fz * vz;
        // u . v over the cone is at most its value on the axis
        if (!(av * iL > tau)) continue;
        const float vn = sqrtf(vx * vx + vy * vy + vz * vz);
        if (!(av > (1e-4f - ct) * L * vn)) continue;  // the cone may reach -v
        const float cx = fy * vz - fz * vy, cy = fz * vx - fx * vz, cz = fx * vy - fy * vx;
        const float axv = sqrtf(cx * cx + cy * cy + cz * cz);
        const float mn = (av * ct - axv * st) * iL;
        if ((double)mn > v.w + 1e-9 * ((double)vn + fabs(v.w)) + 1e-5 * (double)vn) return true;
    }
    return false;
}

// Thread t's item within a block-wide round: items 4k .. 4k+3 go to lane k
// of waves 0 .. 3, so that a short round still uses every SIMD.
__device__ inline int spread(int t) { return (t % WAVE) * (CH_THREADS / WAVE) + t / WAVE; }

template <bool CNT>
__device__ void edge_chunk(const Mol &m, const uint8_t *L, const long long *keys,
                           const int *order, int g0, int n, double *lam, double *nrm,
                           uint8_t *ptype, int *patoms, int *fallback, int *nfallback,
                           bool same_tile, ChunkLds &S, unsigned long long *cnt) {
    const int tid = threadIdx.x;
    const double h = m.h, rho = m.rho;
    const double half = 0.5 * h + 1e-9;
    if (tid < n) {
        long long q = order[g0 + tid];
        long long key = keys[q];
        EdgeGeom G = edge_geom(m, L, key);
        S.eq[tid] = q;
        const int axis = (int)(key % 3);
        for (int a = 0; a < 3; ++a) {
            S.xs[tid][a] = G.xs[a];
            S.mid[tid][a] = G.xs[a] + (a == axis ? 0.5 * h : 0.0);
        }
        S.einfo[tid] = axis | (G.Ls << 2) | (G.Lt << 3);
        S.ecount[tid] = 0;
        for (int w = 0; w < CH_ATOMS / 64; ++w) S.amask[tid][w] = 0;
        for (int w = 0; w < CH_SURF / 64; ++w) S.smask[tid][w] = 0;
        if (tid == 0) S.tile = G.tile;
    }
    if (tid == 0) {
        S.nf = 0;
        S.ovf = 0;
    }
    __syncthreads();
    const int tile = S.tile;
    const int a0 = m.tA_off[tile];
    const int nA = m.tA_off[tile + 1] - a0;
    const int nAst = min(CH_ATOMS, nA);
    // the previous chunk of this block covered the same tile: its staged
    // atoms, and its staged surfaces if the tile took one pass, still hold
    if (!same_tile)
        for (int q = tid; q < nAst; q += CH_THREADS) S.atoms[q] = m.atom[m.tA[a0 + q]];
    const int ns_all = tile_surfaces(m, tile);
    const bool restage = !same_tile || ns_all > CH_SURF;
    // one surface pass with every atom staged: labels from the per-edge masks
    const bool filt = ns_all > 0 && ns_all <= CH_SURF && nA <= CH_ATOMS;
    // ball holding every point of the tile's edges: points T t .. T t + T per axis
    double bc[3];
    const int T = m.tile;
    {
        const int t3[3] = {tile % m.tdims[0], (tile / m.tdims[0]) % m.tdims[1],
                           tile / (m.tdims[0] * m.tdims[1])};
        for (int a = 0; a < 3; ++a)
            bc[a] = m.lo[a] + (t3[a] * T + (a == 2 ? m.kz0 : 0) + 0.5 * T) * h;
    }
    const double rb = sqrt(3.0) * 0.5 * T * h * (1.0 + 1e-12) + 1e-9;
    // pair p -> (p / n, p % n) by a multiply: with n in [2, 64] and
    // p < 2^16, floor(p * ceil(2^32 / n) / 2^32) is p / n exactly
    const unsigned ninv = n > 1 ? 0xFFFFFFFFu / (unsigned)n + 1u : 0u;
    auto split = [&](int p, int &hi, int &lo) {
        hi = n > 1 ? (int)__umulhi((unsigned)p, ninv) : p;
        lo = p - hi * n;
    };
    for (int sb = 0; sb < ns_all; sb += CH_SURF) {
        const int ns = min(CH_SURF, ns_all - sb);
        // stage the pass's surfaces and, culled to the tile's direction cone,
        // their cut planes, every thread on a (surface, cut) pair: one sweep
        // marks the surfaces that one cut rejects over the whole cone (dead
        // in this tile) and counts the cuts kept, the next copies the kept
        // cuts of the surfaces that fit the pool; the others keep every cut
        // in global memory
        if (restage) {
            int ncut = 0;
            if (tid < ns) {
                const int key = tile_surface_key(m, tile, sb + tid);
                S.skey[tid] = key;
                S.sp[tid] = sphere_reach_bounds(surf_params(m, key), key >> 28, rho, half);
                int cb, ce;
                global_cuts(m, key, &cb, &ce);
                S.st.ccb[tid] = cb;
                S.st.ccur[tid] = 0;
                S.sdead[tid] = 0;
                ncut = ce - cb;
            }
            if (tid < ns) {
                const DirCone cone = surface_cone(S.skey[tid] >> 28, S.sp[tid], bc, rb);
                S.st.cna[tid] =
                    make_float4((float)cone.ax, (float)cone.ay, (float)cone.az, (float)cone.st);
                S.st.cnc[tid] = cone.all ? -1.0f : (float)cone.ct;
            }
            int total;
            const int off = block_excl_scan<int, CH_THREADS>(ncut, S.scan, &total);
            if (tid < ns) S.st.coff[tid] = off;
            if (tid == 0) S.st.coff[ns] = total;
            __syncthreads();
            for (int pass = 0; pass < 2; ++pass) {
                for (int p = tid; p < total; p += CH_THREADS) {
                    int lo = 0, hi = ns;
                    while (lo < hi) {
                        const int mid = (lo + hi) >> 1;
                        if (S.st.coff[mid + 1] <= p) lo = mid + 1;
                        else hi = mid;
                    }
                    const int q = lo;
                    if (pass == 1 && S.crange[q].x < 0) continue;  // not pooled
                    const int type = S.skey[q] >> 28;
                    const double4 *gc = type == 1 ? m.face_cut : m.ec_cut;
                    const double4 v = gc[S.st.ccb[q] + (p - S.st.coff[q])];
                    const float4 ca = S.st.cna[q];
                    const float cc = S.st.cnc[q];
                    if (pass == 0 && cone_rejects_f(ca, cc, v)) S.sdead[q] = 1;
                    if (!cone_may_reject_f(ca, cc, v)) continue;
                    const int k = atomicAdd(&S.st.ccur[q], 1);
                    if (pass == 1) S.cut[S.crange[q].x + k] = v;
                }
                if (pass == 1) break;
                __syncthreads();
                const bool dead = tid < ns && S.sdead[tid];
                const int kept = tid < ns && !dead ? S.st.ccur[tid] : 0;
                int ktot;
                const int koff = block_excl_scan<int, CH_THREADS>(kept, S.scan, &ktot);
                if (tid < ns) {
                    const int cb = S.st.ccb[tid];
                    const int ce = cb + S.st.coff[tid + 1] - S.st.coff[tid];
                    const bool fits = !dead && koff + kept <= CH_CUTS;
                    S.crange[tid] = fits ? make_int2(koff, koff + kept) : make_int2(-1 - cb, ce);
                    S.st.ccur[tid] = 0;
                }
                __syncthreads();
            }
            __syncthreads();
        }
        // atoms whose SAS ball can hold a point of an edge (label masks)
        if (filt && sb == 0) {
            for (int p = tid; p < n * nAst; p += CH_THREADS) {
                int ei, ai;
                split(p, ai, ei);
                const double4 a = S.atoms[ai];
                double dm2 = 0.0;
                for (int c = 0; c < 3; ++c) {
                    const double ac = c == 0 ? a.x : c == 1 ? a.y : a.z;
                    dm2 += sq(S.mid[ei][c] - ac);
                }
                if (dm2 < sq(a.w + rho + half)) atomicOr(&S.amask[ei][ai >> 6], 1ull << (ai & 63));
            }
        }
        // (edge, surface) pairs: wavefront w takes the staged surfaces s = w,
        // w + 4, ... and lane e the chunk's edge e, so a surface is read once
        // per wavefront (an LDS broadcast) and its type is uniform.  Pairs
        // that reach go to the wavefront's queue of their kind (tori apart
        // from spheres); a queue that holds a wavefront's worth is solved at
        // once, one pair per lane, without waiting for the other wavefronts.
        // Lane e gathers the label-mask bits of edge e.
        {
            const int wv = tid / WAVE, lane = tid % WAVE;
            const bool eact = lane < n;
            int nqs = 0, nqt = 0;  // queue lengths (uniform across the wavefront)
            for (int s0 = 0;;) {
                // a full queue is solved first; once every surface is
                // tested, the partial queues; one call site keeps the
                // solver inlined once
                int which = -1, count = 0;
                if (nqt >= WAVE) which = 1;
                else if (nqs >= WAVE) which = 0;
                else if (s0 >= ns) which = nqt ? 1 : nqs ? 0 : -1;
                if (which >= 0) {
                    count = which ? nqt : nqs;
                    const int left = count > WAVE ? count - WAVE : 0;
                    if (which) nqt = left;
                    else nqs = left;
                    // the pairs beyond the first WAVE move to the front
                    unsigned short *qu = S.wq[wv][which];
                    const unsigned short v = lane < count ? qu[lane] : (unsigned short)0;
                    if (lane < left) qu[lane] = qu[WAVE + lane];
                    if (lane < count) {
                        const int ei = v & 63, si = v >> 6;
                        const int skey = S.skey[si];
                        const SurfParams sp = S.sp[si];
                        const int axis = S.einfo[ei] & 3;
                        const double xs[3] = {S.xs[ei][0], S.xs[ei][1], S.xs[ei][2]};
                        const double e[3] = {axis == 0 ? 1.0 : 0.0, axis == 1 ? 1.0 : 0.0,
                                             axis == 2 ? 1.0 : 0.0};
                        int nr = 0;
                        surface_roots<CNT>(
                            skey >> 28, sp, h, rho, e, xs,
                            [&](double u) {
                                if (nr < CH_SLOTS) S.slot[nr][tid] = u;
                                ++nr;
                            },
                            cnt);
                        if (nr > CH_SLOTS) {
                            S.ovf = 1;
                            nr = CH_SLOTS;
                        }
                        auto pass = [&](double px, double py, double pz, double sc) {
                            return staged_cuts_pass<CNT>(m, S, si, px, py, pz, sc,
                                                         CNT ? cnt + EC_CUT : nullptr);
                        };
                        for (int r = 0; r < nr; ++r) {
                            const double u = S.slot[r][tid];
                            if (root_admissible(m, skey, sp, pass, u, e, xs)) {
                                const int pos = atomicAdd(&S.nf, 1);
                                if (pos < CH_ROOTS) {
                                    S.fu[pos] = u;
                                    S.fk[pos] = skey;
                                    S.fe[pos] = (unsigned char)ei;
                                }
                            }
                        }
                    }
                    continue;
                }
                if (s0 >= ns) break;
                const int si = s0 + wv;
                s0 += CH_THREADS / WAVE;
                if (si >= ns) continue;  // this wavefront's surfaces are done
                const int type = S.skey[si] >> 28;
                if (CNT && eact) ++cnt[type == 2 ? EC_REACH_TORUS : EC_REACH_SPHERE];
                if (S.sdead[si]) continue;
                bool rel = false, hit = false;
                if (eact) {
                    const double mid[3] = {S.mid[lane][0], S.mid[lane][1], S.mid[lane][2]};
                    hit = staged_reaches_rel(type, S.sp[si], rho, mid, half, &rel);
                    // a face or circle whose candidate is inadmissible on the
                    // whole edge has no kept root there and fails every
                    // label test
                    if (type != 3 && (hit || rel) &&
                        edge_cone_dead<CNT>(m, S, si, type, mid, half, cnt)) {
                        hit = false;
                        rel = false;
                    }
                }
                if (rel) atomicOr(&S.smask[lane][si >> 6], 1ull << (si & 63));
                const unsigned long long hb = __ballot(hit);
                if (!hb) continue;
                const int pos = __popcll(hb & ((1ull << lane) - 1ull));
                if (type == 2) {
                    if (hit) S.wq[wv][1][nqt + pos] = (unsigned short)(lane | (si << 6));
                    nqt += __popcll(hb);
                } else {
                    if (hit) S.wq[wv][0][nqs + pos] = (unsigned short)(lane | (si << 6));
                    nqs += __popcll(hb);
                }
            }
        }
        __syncthreads();
    }
    // too many roots for the chunk's lists: its edges go to the wavefront kernel
    if (S.ovf || S.nf > CH_ROOTS || m.edge_fallback) {
        if (tid == 0) S.fb_base = atomicAdd(nfallback, n);
        __syncthreads();
        if (tid < n) fallback[S.fb_base + tid] = (int)S.eq[tid];
        return;
    }
    // group the roots by edge (counting sort)
    const int nf = S.nf;
    for (int j = tid; j < nf; j += CH_THREADS) atomicAdd(&S.ecount[S.fe[j]], 1);
    __syncthreads();
    if (tid < WAVE) {
        int c = tid < n ? S.ecount[tid] : 0;
        int incl = wave_incl_scan(c);
        if (tid < n) {
            S.eoff[tid] = incl - c;
            S.ecount[tid] = incl - c;  // fill cursor
        }
    }
    __syncthreads();
    for (int j = tid; j < nf; j += CH_THREADS) S.perm[atomicAdd(&S.ecount[S.fe[j]], 1)] = (unsigned short)j;
    __syncthreads();
    // one thread per edge (edge e on wave e % 4): sort its roots by (u, key)
    const int ei = spread(tid);
    const bool act = ei < n;
    int o = 0, ne = 0;
    if (act) {
        o = S.eoff[ei];
        ne = S.ecount[ei] - o;
        for (int a = 1; a < ne; ++a) {
            unsigned short v = S.perm[o + a];
            double u = S.fu[v];
            int k = S.fk[v];
            int b = a - 1;
            while (b >= 0) {
                unsigned short w = S.perm[o + b];
                double uw = S.fu[w];
                if (uw < u || (uw == u && S.fk[w] <= k)) break;
                S.perm[o + b + 1] = w;
                --b;
            }
            S.perm[o + b + 1] = v;
        }
    }
    EdgeGeom G;
    const int info = act ? S.einfo[ei] : 0;
    const int axis = info & 3;
    for (int a = 0; a < 3; ++a) {
        G.xs[a] = act ? S.xs[ei][a] : 0.0;
        G.e[a] = a == axis ? 1.0 : 0.0;
    }
    G.tile = tile;
    G.Ls = (info >> 2) & 1;
    G.Lt = (info >> 3) & 1;
    auto root_at = [&](int r, double &u, int &k) {
        unsigned short v = S.perm[o + r];
        u = S.fu[v];
        k = S.fk[v];
    };
    // the staged surfaces serve the labels when the tile had a single pass
    const bool staged = ns_all <= CH_SURF;
    const int nF = m.tF_off[tile + 1] - m.tF_off[tile];
    const int nV = m.tV_off[tile + 1] - m.tV_off[tile];
    int owner = -1;
    double ustar = 1.0;
    bool done = false;
    if (filt) {
        // every interval whose label the walk may read becomes a query; the
        // block evaluates all (query, candidate) tests of the per-edge masks
        // at once, and the walk reads the combined results
        if (tid == 0) S.nq = 0;
        __syncthreads();
        int nqe = 0, q0 = 0;
        if (act) {
            label_intervals(ne, root_at, [&](double) { ++nqe; });
            q0 = atomicAdd(&S.nq, nqe);
        }
        __syncthreads();
        const int nq = S.nq;
        if (nq <= CH_Q) {
            if (act && nqe > 0) {
                int k = q0;
                label_intervals(ne, root_at, [&](double um) {
                    S.q.qu[k] = um;
                    S.q.qe[k] = (unsigned char)ei;
                    ++k;
                });
                if (CNT) cnt[EC_LABEL] += nqe;
            }
            __syncthreads();
            // the atoms' tests first: a query in a van der Waals ball (flag
            // 1) or in no SAS ball (no flag 2) is decided by them, and the
            // surfaces' tests run only for the others
            for (int phase = 0; phase < 2; ++phase) {
                int kq = 0;
                if (tid < nq) {
                    const int e = S.q.qe[tid];
                    int ka = 0;
                    for (int w = 0; w < CH_ATOMS / 64; ++w) ka += __popcll(S.amask[e][w]);
                    if (phase == 0) {
                        kq = ka;
                        S.q.qflag[tid] = 0;
                    } else if (S.q.qflag[tid] == 2) {
                        for (int w = 0; w < CH_SURF / 64; ++w) kq += __popcll(S.smask[e][w]);
                    }
                    S.q.qskip[tid] = phase == 0 ? 0 : ka;
                }
                int tot;
                const int off = block_excl_scan<int, CH_THREADS>(kq, S.scan, &tot);
                if (tid < nq) S.q.qoff[tid] = off;
                if (tid == 0) S.q.qoff[nq] = tot;
                __syncthreads();
                for (int p = tid; p < tot; p += CH_THREADS) {
                    int lo = 0, hi = nq;
                    while (lo < hi) {
                        int mid = (lo + hi) >> 1;
                        if (S.q.qoff[mid + 1] <= p) lo = mid + 1;
                        else hi = mid;
                    }
                    const int f = label_test<CNT>(m, S, S.q.qe[lo],
                                                  S.q.qskip[lo] + p - S.q.qoff[lo], S.q.qu[lo],
                                                  nF, nV, cnt);
                    if (f) atomicOr(&S.q.qflag[lo], f);
                }
                __syncthreads();
            }
            if (act) {
                int k = q0;
                ustar = walk_roots<false>(
                    ne, root_at, G.Ls, G.Lt, G.xs, G.e, h,
                    [&](double, double, double) {
                        const int f = S.q.qflag[k++];
                        return (f & 1) ? 1 : (!(f & 2) ? 0 : ((f & 4) ? 0 : 1));
                    },
                    &owner, cnt);
            }
            done = true;
        }
    }
    if (!act) return;
    if (!done)
        ustar = walk_roots<CNT>(
            ne, root_at, G.Ls, G.Lt, G.xs, G.e, h,
            [&](double x, double y, double z) {
                return filt     ? label_masked<CNT>(m, S, ei, nF, nV, x, y, z, cnt)
                       : staged ? label_chunk<CNT>(m, S, tile, nAst, nF, nV, ns_all, x, y, z, cnt)
                                : label_fp64_t<CNT>(m, tile, x, y, z, CNT ? cnt + EC_L_ATOM : nullptr);
            },
            &owner, cnt);
    if (CNT) {
        ++cnt[EC_EDGES];
        return;
    }
    write_record(m, S.eq[ei], G, ustar, owner, lam, nrm, ptype, patoms);
}

// Chunk c covers positions [CH_EDGES c, CH_EDGES c + n) of `order`, all in
// one tile (each tile's segment is padded to a multiple of CH_EDGES).  The
// grid is persistent: blocks take the units (tiles with edges, the ones with
// most chunks first) from one counter, and a block runs every chunk of its
// tile in a row, staging the tile once; when the tiles are fewer than the
// blocks, each chunk is a unit of its own.
template <bool CNT>
__global__ void __launch_bounds__(CH_THREADS) __attribute__((amdgpu_waves_per_eu(3)))
    k_edge_chunks(Mol m, const uint8_t *L, const long long *keys, const int *order,
                  const int *tcount, const int *coff, int *units, double *lam, double *nrm,
                  uint8_t *ptype, int *patoms, int *fallback, int *nfallback,
                  unsigned long long *work) {
    __shared__ ChunkLds S;
    __shared__ int next;
    unsigned long long cnt[CNT ? EC_COUNT + 1 : 1];
    for (int c = 0; c < (CNT ? (int)EC_COUNT + 1 : 1); ++c) cnt[c] = 0;
    // with too few tiles to balance the blocks (fewer than CH_TILE_UNITS per
    // block), the units are the chunks themselves, so that a tile's chunks
    // run side by side
    const int nunits = units[EU_COUNT];
    const bool per_chunk = nunits < CH_TILE_UNITS * (int)gridDim.x;
    const int nq = per_chunk ? coff[m.ntiles] : nunits;
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(&units[EU_QUEUE], 1);
        __syncthreads();
        const int u = next;
        __syncthreads();
        if (u >= nq) break;
        int t, cb, ce;
        if (per_chunk) {
            cb = u;
            ce = u + 1;
            t = edge_tile(m, keys[order[u * CH_EDGES]]);
        } else {
            t = units[EU_LIST + u];
            cb = coff[t];
            ce = coff[t + 1];
        }
        for (int c = cb; c < ce; ++c) {
            const int g0 = c * CH_EDGES;
            const int n = min(CH_EDGES, tcount[t] - (c - coff[t]) * CH_EDGES);
            edge_chunk<CNT>(m, L, keys, order, g0, n, lam, nrm, ptype, patoms, fallback,
                            nfallback, c != cb, S, cnt);
            __syncthreads();
        }
    }
    if (CNT)
        for (int c = 0; c < EC_COUNT; ++c)
            if (cnt[c]) atomicAdd(&work[c], cnt[c]);
}

// ------------------------------------------------ roots of a batch, one launch

// Global unit offsets of the jobs' unit lists (one block).
__global__ void __launch_bounds__(256) k_edge_batch_prefix(const EdgeJob *jobs, int nj,
                                                           int *prefix) {
    __shared__ int lds[256 / WAVE + 1];
    int carry = 0;
    for (int b = 0; b < nj; b += 256) {
        const int j = b + (int)threadIdx.x;
        const int v = j < nj ? jobs[j].units[EU_COUNT] : 0;
        int tot;
        const int off = block_excl_scan<int, 256>(v, lds, &tot);
        if (j < nj) prefix[j] = carry + off;
        carry += tot;
    }
    if (threadIdx.x == 0) prefix[nj] = carry;
}

// The chunk kernel over the tiles of every job: global unit u belongs to
// the last job whose offset is at most u.
__global__ void __launch_bounds__(CH_THREADS) __attribute__((amdgpu_waves_per_eu(3)))
    k_edge_chunks_batch(const Mol *mols, const EdgeJob *jobs, int nj, const int *prefix,
                        int *queue) {
    __shared__ ChunkLds S;
    __shared__ int next;
    unsigned long long cnt[1] = {0};
    const int total = prefix[nj];
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(queue, 1);
        __syncthreads();
        const int u = next;
        __syncthreads();
        if (u >= total) break;
        int lo = 0, hi = nj - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (prefix[mid] <= u) lo = mid;
            else hi = mid - 1;
        }
        const int j = __builtin_amdgcn_readfirstlane(lo);
        const EdgeJob &J = jobs[j];
        const int t = J.units[EU_LIST + (u - prefix[j])];
        const int c0 = J.coff[t], c1 = J.coff[t + 1];
        for (int c = c0; c < c1; ++c) {
            const int n = min(CH_EDGES, J.tcount[t] - (c - c0) * CH_EDGES);
            edge_chunk<false>(uniform_mol(mols, J.mol), J.L, J.keys, J.order, c * CH_EDGES, n,
                              J.lam, J.nrm, J.ptype, J.patoms, J.fallback, J.nfallback, c != c0,
                              S, cnt);
            __syncthreads();
        }
    }
}

// ------------------------------------------------ roots, one wavefront per edge
//
// For the edges of chunks whose root lists overflow: one wavefront per edge,
// with up to EW_SURF reaching surfaces and EW_ROOTS roots.  Lanes gather the
// reaching surfaces, each lane solves one surface, one lane per root tests
// admissibility, the roots are rank-sorted in LDS and the walk runs on every
// lane (uniformly).  The arithmetic is that of the chunk path.
constexpr int EW_WAVES = 4;
constexpr int EW_THREADS = EW_WAVES * WAVE;
constexpr int EW_SURF = 256;
constexpr int EW_ROOTS = 256;

struct EdgeWaveLds {
    int surf[EW_SURF];
    double u[EW_ROOTS];
    int k[EW_ROOTS];
    double su[EW_ROOTS];
    int sk[EW_ROOTS];
    int nroot;
};

template <bool CNT>
__device__ void edge_wave(const Mol &m, const uint8_t *L, const long long *keys, long long q,
                          double *lam, double *nrm, uint8_t *ptype, int *patoms, int *overflow,
                          EdgeWaveLds &S, unsigned long long *cnt) {
    const int lane = lane_id();
    const long long key = keys[q];
    const EdgeGeom G = edge_geom(m, L, key);
    const int tile = G.tile;
    const double h = m.h, rho = m.rho;
    const double hh = 0.5 * h;
    const double mid[3] = {G.xs[0] + hh * G.e[0], G.xs[1] + hh * G.e[1], G.xs[2] + hh * G.e[2]};
    const double half = 0.5 * h + 1e-9;
    bool ovf = false;
    if (lane == 0) S.nroot = 0;
    // 1. reaching surfaces, compacted with ballots
    const int ns_all = tile_surfaces(m, tile);
    int ns = 0;
    for (int base = 0; base < ns_all; base += WAVE) {
        int s = base + lane;
        bool r = false;
        int key = 0;
        if (s < ns_all) {
            key = tile_surface_key(m, tile, s);
            int type = key >> 28;
            if (CNT) ++cnt[type == 2 ? EC_REACH_TORUS : EC_REACH_SPHERE];
            r = surf_reaches(type, surf_params(m, key), rho, mid, half);
        }
        unsigned long long bm = __ballot(r);
        int pos = ns + mask_prefix(bm);
        if (r && pos < EW_SURF) S.surf[pos] = key;
        ns += __popcll(bm);
    }
    if (ns > EW_SURF) {
        ovf = true;
        ns = EW_SURF;
    }
    wave_sync();
    // 2. one surface per lane, every root in [0, 1] appended
    for (int sb = 0; sb < ns; sb += WAVE) {
        int si = sb + lane;
        if (si < ns) {
            const int key = S.surf[si];
            surface_roots<CNT>(
                key >> 28, surf_params(m, key), h, rho, G.e, G.xs,
                [&](double u) {
                    int pos = atomicAdd(&S.nroot, 1);
                    if (pos < EW_ROOTS) {
                        S.u[pos] = u;
                        S.k[pos] = key;
                    }
                },
                cnt);
        }
    }
    wave_sync();
    int nraw = S.nroot;
    if (nraw > EW_ROOTS) {
        ovf = true;
        nraw = EW_ROOTS;
    }
    // 3. one root per lane: admissible ones compacted into (su, sk)
    int nr = 0;
    for (int b = 0; b < nraw; b += WAVE) {
        int r = b + lane;
        bool keep = false;
        double u = 0.0;
        int k = 0;
        if (r < nraw) {
            u = S.u[r];
            k = S.k[r];
            int cb, ce;
            const double4 *cuts = global_cuts(m, k, &cb, &ce);
            auto pass = [&](double px, double py, double pz, double sc) {
                return cuts_pass<CNT>(cuts, cb, ce, px, py, pz, sc, CNT ? cnt + EC_CUT : nullptr);
            };
            keep = root_admissible(m, k, surf_params(m, k), pass, u, G.e, G.xs);
        }
        unsigned long long bm = __ballot(keep);
        if (keep) {
            int pos = nr + mask_prefix(bm);
            S.su[pos] = u;
            S.sk[pos] = k;
        }
        nr += __popcll(bm);
    }
    wave_sync();
    // 4. rank sort by (u, key) from (su, sk) into (u, k)
    for (int b = 0; b < nr; b += WAVE) {
        int r = b + lane;
        if (r < nr) {
            double u = S.su[r];
            int k = S.sk[r];
            int rank = 0;
            for (int p = 0; p < nr; ++p) {
                double up = S.su[p];
                int kp = S.sk[p];
                rank += (up < u || (up == u && (kp < k || (kp == k && p < r)))) ? 1 : 0;
            }
            S.u[rank] = u;
            S.k[rank] = k;
        }
    }
    wave_sync();
    // 5. the walk, the same on every lane; lane 0 counts and writes
    unsigned long long dummy[EC_COUNT + 1];
    unsigned long long *lc = lane == 0 ? cnt : dummy;
    int owner = -1;
    const double ustar = walk_roots<CNT>(
        nr,
        [&](int r, double &u, int &k) {
            u = S.u[r];
            k = S.k[r];
        },
        G.Ls, G.Lt, G.xs, G.e, h,
        [&](double x, double y, double z) {
            return label_fp64_t<CNT>(m, tile, x, y, z, lc + EC_L_ATOM);
        },
        &owner, lc);
    if (__any(ovf) && lane == 0) *overflow = 1;
    if (CNT) {
        if (lane == 0) ++cnt[EC_EDGES];
        return;
    }
    if (lane == 0) write_record(m, q, G, ustar, owner, lam, nrm, ptype, patoms);
}

template <bool CNT>
__global__ void __launch_bounds__(EW_THREADS)
    k_edge_wave(Mol m, const uint8_t *L, const long long *keys, const int *list,
                const int *nlist, double *lam, double *nrm, uint8_t *ptype, int *patoms,
                int *overflow, unsigned long long *work) {
    __shared__ EdgeWaveLds lds[EW_WAVES];
    const int w = threadIdx.x / WAVE;
    unsigned long long cnt[CNT ? EC_COUNT + 1 : 1];
    for (int c = 0; c < (CNT ? (int)EC_COUNT + 1 : 1); ++c) cnt[c] = 0;
    const int n = *nlist;
    for (int g = blockIdx.x * EW_WAVES + w; g < n; g += gridDim.x * EW_WAVES) {
        edge_wave<CNT>(m, L, keys, list[g], lam, nrm, ptype, patoms, overflow, lds[w], cnt);
        wave_sync();
    }
    if (CNT)
        for (int c = 0; c < EC_COUNT; ++c)
            if (cnt[c]) atomicAdd(&work[c], cnt[c]);
}

// ------------------------------------------------ grouping by tile, launches

// Chunks per tile, and the tiles with edges counted by class min(chunks,
// EU_CLASSES) (in LDS, then one global add per class and block); block blk
// takes tiles from 256 blk on.
__device__ inline void edge_chunk_count_block(const int *tcount, int ntiles, int *ccount,
                                              int *units, int blk, int *cls) {
    const int t = blk * 256 + threadIdx.x;
    if (threadIdx.x < EU_CLASSES) cls[threadIdx.x] = 0;
    __syncthreads();
    if (t < ntiles) {
        const int c = (tcount[t] + CH_EDGES - 1) / CH_EDGES;
        ccount[t] = c;
        if (c > 0) atomicAdd(&cls[min(c, EU_CLASSES) - 1], 1);
    }
    __syncthreads();
    if (threadIdx.x < EU_CLASSES && cls[threadIdx.x] > 0)
        atomicAdd(&units[EU_CLASS + threadIdx.x], cls[threadIdx.x]);
}

__global__ void __launch_bounds__(256) k_edge_chunk_count(const int *tcount, int ntiles,
                                                          int *ccount, int *units) {
    __shared__ int cls[EU_CLASSES];
    edge_chunk_count_block(tcount, ntiles, ccount, units, blockIdx.x, cls);
}

// The unit list: tiles with edges, classes of more chunks first.  A block
// ranks its tiles per class in LDS and reserves each class's run with one
// global add.
__device__ inline void edge_unit_order_block(const int *ccount, int ntiles, int *units, int blk,
                                             int *cls, int *base) {
    const int t = blk * 256 + threadIdx.x;
    if (t == 0) {
        int tot = 0;
        for (int b = 0; b < EU_CLASSES; ++b) tot += units[EU_CLASS + b];
        units[EU_COUNT] = tot;
    }
    if (threadIdx.x < EU_CLASSES) cls[threadIdx.x] = 0;
    __syncthreads();
    int b = -1, r = 0;
    if (t < ntiles) {
        const int c = ccount[t];
        if (c > 0) {
            b = min(c, EU_CLASSES) - 1;
            r = atomicAdd(&cls[b], 1);
        }
    }
    __syncthreads();
    if (threadIdx.x < EU_CLASSES && cls[threadIdx.x] > 0) {
        int off = 0;
        for (int k = threadIdx.x + 1; k < EU_CLASSES; ++k) off += units[EU_CLASS + k];
        base[threadIdx.x] = off + atomicAdd(&units[EU_FILL + threadIdx.x], cls[threadIdx.x]);
    }
    __syncthreads();
    if (b >= 0) units[EU_LIST + base[b] + r] = t;
}

__global__ void __launch_bounds__(256) k_edge_unit_order(const int *ccount, int ntiles,
                                                         int *units) {
    __shared__ int cls[EU_CLASSES], base[EU_CLASSES];
    edge_unit_order_block(ccount, ntiles, units, blockIdx.x, cls, base);
}

__device__ inline void edge_tile_scatter_at(const Mol &m, const long long *keys, long long q,
                                            const int *coff, const int *rank, int *order) {
    const int t = edge_tile(m, keys[q]);
    order[(long long)coff[t] * CH_EDGES + rank[q]] = (int)q;
}

__global__ void k_edge_tile_scatter(Mol m, const long long *keys, long long count,
                                    const int *coff, const int *rank, int *order) {
    long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (q < count) edge_tile_scatter_at(m, keys, q, coff, rank, order);
}

// ------------------------------------- crossing edges of a batch, batched
//
// The passes above over every molecule of a batch at once: block b of a
// batched pass works for molecule q with start[q] <= b < start[q + 1] (the
// largest such q, so molecules with no blocks in the pass are skipped), as
// that molecule's block b - start[q].

__device__ inline int batch_mol_of(const int *start, int nm, int b) {
    int lo = 0, hi = nm - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (start[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ void __launch_bounds__(EDGE_BLOCK) k_edge_count_batch(const Mol *mols,
                                                                 const EdgeDetectJob *jobs,
                                                                 const int *start, int nm) {
    __shared__ int lds[EDGE_BLOCK / WAVE + 1];
    const int q = batch_mol_of(start, nm, blockIdx.x);
    const Mol &m = mols[q];
    edge_count_block(jobs[q].L, m.dims[0], m.dims[1], m.dims[2], m.npts,
                     (int)blockIdx.x - start[q], jobs[q].bcount, lds);
}

__global__ void __launch_bounds__(EDGE_BLOCK) k_edge_write_batch(const Mol *mols,
                                                                 const EdgeDetectJob *jobs,
                                                                 const int *start, int nm) {
    __shared__ int lds[EDGE_BLOCK / WAVE + 1];
    const int q = batch_mol_of(start, nm, blockIdx.x);
    const Mol &m = mols[q];
    const EdgeDetectJob &J = jobs[q];
    const int blk = (int)blockIdx.x - start[q];
    edge_write_block(J.L, m.dims[0], m.dims[1], m.dims[2], m.npts, blk, J.boff[blk], J.nw,
                     J.keys, J.tcount, J.rank, m.tile, m.tdims[0], m.tdims[1], lds);
}

__global__ void __launch_bounds__(256) k_edge_chunk_count_batch(const Mol *mols,
                                                                const EdgeDetectJob *jobs,
                                                                const int *start, int nm) {
    __shared__ int cls[EU_CLASSES];
    const int q = batch_mol_of(start, nm, blockIdx.x);
    const EdgeDetectJob &J = jobs[q];
    edge_chunk_count_block(J.tcount, mols[q].ntiles, J.ccount, J.units,
                           (int)blockIdx.x - start[q], cls);
}

__global__ void __launch_bounds__(256) k_edge_unit_order_batch(const Mol *mols,
                                                               const EdgeDetectJob *jobs,
                                                               const int *start, int nm) {
    __shared__ int cls[EU_CLASSES], base[EU_CLASSES];
    const int q = batch_mol_of(start, nm, blockIdx.x);
    const EdgeDetectJob &J = jobs[q];
    edge_unit_order_block(J.ccount, mols[q].ntiles, J.units, (int)blockIdx.x - start[q], cls,
                          base);
}

__global__ void __launch_bounds__(256) k_edge_tile_scatter_batch(const Mol *mols,
                                                                 const EdgeDetectJob *jobs,
                                                                 const int *start, int nm) {
    const int q = batch_mol_of(start, nm, blockIdx.x);
    const EdgeDetectJob &J = jobs[q];
    const long long e = ((long long)blockIdx.x - start[q]) * 256 + threadIdx.x;
    if (e < J.nw) edge_tile_scatter_at(mols[q], J.keys, e, J.coff, J.rank, J.order);
}

// Diagnostic word k of every molecule of a batch set to v.
__global__ void k_diag_set(const Mol *mols, int nm, int k, int v) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < nm) mols[q].diag[k] = v;
}

static hipError_t batch_grid(const int *start_host, int nm, unsigned *nb) {
    const long long n = start_host[nm];
    if (n < 0 || n > 0x7fffffffLL) return hipErrorInvalidValue;
    *nb = (unsigned)n;
    return hipSuccess;
}

hipError_t launch_edge_detect_count_batch(const Mol *mols, const EdgeDetectJob *jobs,
                                          const int *start, const int *start_host, int nm,
                                          hipStream_t st) {
    unsigned nb = 0;
    hipError_t e = batch_grid(start_host, nm, &nb);
    if (e != hipSuccess || nb == 0) return e;
    hipLaunchKernelGGL(k_edge_count_batch, dim3(nb), dim3(EDGE_BLOCK), 0, st, mols, jobs, start,
                       nm);
    return hipGetLastError();
}

hipError_t launch_edge_detect_write_batch(const Mol *mols, const EdgeDetectJob *jobs,
                                          const EdgeBatchStarts &s, int nm, hipStream_t st) {
    unsigned nb = 0;
    hipError_t e = hipSuccess;
    if (nm > 0) e = launch_diag_set(mols, nm, 3, 0, st);  // ownerless records
    if (e == hipSuccess) e = batch_grid(s.write_host, nm, &nb);
    if (e != hipSuccess || nb == 0) return e;
    hipLaunchKernelGGL(k_edge_write_batch, dim3(nb), dim3(EDGE_BLOCK), 0, st, mols, jobs, s.write,
                       nm);
    return hipGetLastError();
}

hipError_t launch_edge_group_batch(const Mol *mols, const EdgeDetectJob *jobs,
                                   const EdgeBatchStarts &s, const ScanSeg *coff_scan,
                                   int nscan, long long nchunks, int *sums, int nm,
                                   hipStream_t st) {
    unsigned nt = 0, ne = 0;
    hipError_t e = batch_grid(s.tile_host, nm, &nt);
    if (e == hipSuccess) e = batch_grid(s.edge_host, nm, &ne);
    if (e != hipSuccess || nt == 0) return e;
    hipLaunchKernelGGL(k_edge_chunk_count_batch, dim3(nt), dim3(256), 0, st, mols, jobs, s.tile,
                       nm);
    e = scan_seg(coff_scan, nscan, nchunks, sums, st);
    if (e != hipSuccess) return e;
    if (ne > 0)
        hipLaunchKernelGGL(k_edge_tile_scatter_batch, dim3(ne), dim3(256), 0, st, mols, jobs,
                           s.edge, nm);
    hipLaunchKernelGGL(k_edge_unit_order_batch, dim3(nt), dim3(256), 0, st, mols, jobs, s.tile,
                       nm);
    return hipGetLastError();
}

hipError_t launch_diag_set(const Mol *mols, int nm, int k, int v, hipStream_t st) {
    if (nm <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_diag_set, dim3((nm + 255) / 256), dim3(256), 0, st, mols, nm, k, v);
    return hipGetLastError();
}

long long edge_order_capacity(const Mol &m, long long count) {
    return count + (long long)(CH_EDGES - 1) * std::min<long long>(m.ntiles, count);
}

long long edge_units_capacity(const Mol &m) { return EU_LIST + (long long)m.ntiles; }

hipError_t launch_edge_group(const Mol &m, const long long *keys, long long count, int *tcount,
                             int *ccount, int *coff, const int *rank, int *order, int *units,
                             int *tmp, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    unsigned nb = (unsigned)((count + 255) / 256);
    const unsigned tb = (unsigned)((m.ntiles + 255) / 256);
    hipError_t e = fill_i32(units, EU_LIST, 0, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_edge_chunk_count, dim3(tb), dim3(256), 0, st, tcount, m.ntiles, ccount,
                       units);
    e = scan_i32(ccount, m.ntiles, coff, tmp, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_edge_tile_scatter, dim3(nb), dim3(256), 0, st, m, keys, count, coff,
                       rank, order);
    hipLaunchKernelGGL(k_edge_unit_order, dim3(tb), dim3(256), 0, st, ccount, m.ntiles, units);
    return hipGetLastError();
}

long long edge_detect_blocks(const Mol &m) {
    const long long per = (long long)EDGE_BLOCK * EDGE_PPT;
    const long long nb = (m.npts + per - 1) / per;
    return nb < 1 ? 1 : nb;
}

hipError_t launch_edge_detect_count(const uint8_t *L, const Mol &m, int *bcount, long long *nblk,
                                    hipStream_t st) {
    *nblk = edge_detect_blocks(m);
    hipLaunchKernelGGL(k_edge_count, dim3((unsigned)*nblk), dim3(EDGE_BLOCK), 0, st, L, m.dims[0],
                       m.dims[1], m.dims[2], m.npts, bcount);
    return hipGetLastError();
}

hipError_t launch_edge_detect_write(const uint8_t *L, const Mol &m, const long long *boff,
                                    long long cap, long long *keys, int *tcount, int *rank,
                                    hipStream_t st) {
    hipError_t e = fill_i32(tcount, m.ntiles + 1, 0, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_edge_write, dim3((unsigned)edge_detect_blocks(m)), dim3(EDGE_BLOCK), 0, st,
                       L, m.dims[0], m.dims[1], m.dims[2], m.npts, boff, cap, keys, tcount, rank,
                       m.tile, m.tdims[0], m.tdims[1]);
    return hipGetLastError();
}

// Chunk kernel over every chunk, then the wavefront kernel over the edges of
// chunks that overflowed (normally none).  With work != nullptr the
// statistics variants run and no record is written.
// Resident blocks of the chunk kernel on the current device (its persistent grid).
static int edge_chunk_slots() {
    static std::atomic<int> slots[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
    int v = slots[dev].load(std::memory_order_relaxed);
    if (v > 0) return v;
    int ncu = 0, per = 0;
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_edge_chunks<false>, CH_THREADS, 0);
    v = std::max(1, ncu) * std::max(1, per);
    slots[dev].store(v, std::memory_order_relaxed);
    return v;
}

static hipError_t edge_roots_impl(const Mol &m, const uint8_t *L, const long long *keys,
                                  long long count, const int *order, const int *tcount,
                                  const int *coff, int *units, double *lam, double *nrm,
                                  uint8_t *ptype, int *patoms, int *fallback, int *nfallback,
                                  int *overflow, unsigned long long *work, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipError_t e = fill_i32(nfallback, 1, 0, st);
    if (e == hipSuccess) e = fill_i32(units + EU_QUEUE, 1, 0, st);
    if (e != hipSuccess) return e;
    // no more blocks than chunks or than fit on the device
    const long long chunks_max =
        (count + CH_EDGES - 1) / CH_EDGES + std::min<long long>(m.ntiles, count);
    const long long grid = std::min<long long>(chunks_max, edge_chunk_slots());
    if (work)
        hipLaunchKernelGGL(k_edge_chunks<true>, dim3((unsigned)grid), dim3(CH_THREADS), 0, st, m,
                           L, keys, order, tcount, coff, units, lam, nrm, ptype, patoms,
                           fallback, nfallback, work);
    else
        hipLaunchKernelGGL(k_edge_chunks<false>, dim3((unsigned)grid), dim3(CH_THREADS), 0, st,
                           m, L, keys, order, tcount, coff, units, lam, nrm, ptype, patoms,
                           fallback, nfallback, work);
    if (work)
        hipLaunchKernelGGL(k_edge_wave<true>, dim3(256), dim3(EW_THREADS), 0, st, m, L, keys,
                           fallback, nfallback, lam, nrm, ptype, patoms, overflow, work);
    else
        hipLaunchKernelGGL(k_edge_wave<false>, dim3(256), dim3(EW_THREADS), 0, st, m, L, keys,
                           fallback, nfallback, lam, nrm, ptype, patoms, overflow, work);
    return hipGetLastError();
}

// The fallback edges of every job of a batch.
__global__ void __launch_bounds__(EW_THREADS)
    k_edge_wave_batch(const Mol *mols, const EdgeJob *jobs, int nj, int *overflow) {
    __shared__ EdgeWaveLds lds[EW_WAVES];
    const int w = threadIdx.x / WAVE;
    unsigned long long cnt[1] = {0};
    for (int j = 0; j < nj; ++j) {
        const EdgeJob &J = jobs[j];
        const int n = *J.nfallback;
        for (int g = blockIdx.x * EW_WAVES + w; g < n; g += gridDim.x * EW_WAVES) {
            edge_wave<false>(mols[J.mol], J.L, J.keys, J.fallback[g], J.lam, J.nrm, J.ptype,
                             J.patoms, overflow, lds[w], cnt);
            wave_sync();
        }
    }
}

// Slab views (out-of-core form): the records of the slab's own planes are
// the keys below `limit` (a prefix, keys being ascending); their number goes
// to *n_own and those keys are moved to the whole grid's numbering.
__global__ void k_key_lower_bound(const long long *keys, long long count, long long limit,
                                  long long *n_own) {
    long long lo = 0, hi = count;
    while (lo < hi) {
        const long long mid = (lo + hi) >> 1;
        if (keys[mid] < limit) lo = mid + 1;
        else hi = mid;
    }
    *n_own = lo;
}

__global__ void k_key_shift(long long *keys, long long count, long long limit, long long shift) {
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < count;
         q += (long long)gridDim.x * blockDim.x)
        if (keys[q] < limit) keys[q] += shift;
}

hipError_t launch_slab_keys(long long *keys, long long count, long long limit, long long shift,
                            long long *n_own, hipStream_t st) {
    hipLaunchKernelGGL(k_key_lower_bound, dim3(1), dim3(1), 0, st, keys, count, limit, n_own);
    if (count > 0) {
        const long long nb = std::min<long long>((count + 255) / 256, 4096);
        hipLaunchKernelGGL(k_key_shift, dim3((unsigned)nb), dim3(256), 0, st, keys, count, limit,
                           shift);
    }
    return hipGetLastError();
}

hipError_t launch_edge_roots_batch(const Mol *mols, const EdgeJob *jobs, int nj, int *prefix,
                                   int *queue, int *overflow, hipStream_t st) {
    if (nj <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_edge_batch_prefix, dim3(1), dim3(256), 0, st, jobs, nj, prefix);
    hipLaunchKernelGGL(k_edge_chunks_batch, dim3((unsigned)edge_chunk_slots()), dim3(CH_THREADS),
                       0, st, mols, jobs, nj, prefix, queue);
    hipLaunchKernelGGL(k_edge_wave_batch, dim3(256), dim3(EW_THREADS), 0, st, mols, jobs, nj,
                       overflow);
    return hipGetLastError();
}

hipError_t launch_edge_roots(const Mol &m, const uint8_t *L, const long long *keys,
                             long long count, const int *order, const int *tcount,
                             const int *coff, int *units, double *lam, double *nrm,
                             uint8_t *ptype, int *patoms, int *fallback, int *nfallback,
                             int *overflow, hipStream_t st) {
    return edge_roots_impl(m, L, keys, count, order, tcount, coff, units, lam, nrm, ptype,
                           patoms, fallback, nfallback, overflow, nullptr, st);
}

hipError_t launch_edge_work(const Mol &m, const uint8_t *L, const long long *keys,
                            long long count, const int *order, const int *tcount,
                            const int *coff, int *units, int *fallback, int *nfallback,
                            int *overflow, unsigned long long *work, hipStream_t st) {
    return edge_roots_impl(m, L, keys, count, order, tcount, coff, units, nullptr, nullptr,
                           nullptr, nullptr, fallback, nfallback, overflow, work, st);
}

}  // namespace eses
