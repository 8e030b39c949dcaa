// Stage 3: intersections of the SES with grid edges (eq. 3-4).
//
// (a) Crossing edges: a streaming pass over the label array finds every axis
//     edge whose end labels differ; a block-level prefix sum plus a scan of
//     block counts gives each edge its slot, so keys come out ascending.
// (b) Roots: one lane per crossing edge collects, along s + u h e_axis, the
//     roots in [0, 1] of every surface that can carry the boundary of M
//     there -- van der Waals spheres (convex), tori of radius rho around
//     exposed circles (saddle), probe spheres around exposed concave probe
//     positions (concave) -- sorts them, and walks the intervals from s.
//     u* is the start of the first interval whose label differs from
//     Inside[s]; lambda = 1 - u*.
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
    EC_COUNT
};

__device__ inline int edge_flags(const uint8_t *L, long long idx, int i, int j, int k, int nx,
                                 int ny, int nz) {
    uint8_t a = L[idx];
    int f = 0;
    if (i + 1 < nx && L[idx + 1] != a) f |= 1;
    if (j + 1 < ny && L[idx + nx] != a) f |= 2;
    if (k + 1 < nz && L[idx + (long long)nx * ny] != a) f |= 4;
    return f;
}

__global__ void __launch_bounds__(EDGE_BLOCK) k_edge_count(const uint8_t *L, int nx, int ny,
                                                           int nz, long long npts, int *bcount) {
    __shared__ int lds[EDGE_BLOCK / WAVE + 1];
    long long idx = (long long)blockIdx.x * EDGE_BLOCK + threadIdx.x;
    int c = 0;
    if (idx < npts) {
        int i = (int)(idx % nx);
        long long r = idx / nx;
        int j = (int)(r % ny);
        int k = (int)(r / ny);
        c = __popc(edge_flags(L, idx, i, j, k, nx, ny, nz));
    }
    int tot;
    block_excl_scan<int, EDGE_BLOCK>(c, lds, &tot);
    if (threadIdx.x == 0) bcount[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(EDGE_BLOCK) k_edge_write(const uint8_t *L, int nx, int ny,
                                                           int nz, long long npts,
                                                           const long long *boff, long long cap,
                                                           long long *keys) {
    __shared__ int lds[EDGE_BLOCK / WAVE + 1];
    long long idx = (long long)blockIdx.x * EDGE_BLOCK + threadIdx.x;
    int f = 0;
    if (idx < npts) {
        int i = (int)(idx % nx);
        long long r = idx / nx;
        int j = (int)(r % ny);
        int k = (int)(r / ny);
        f = edge_flags(L, idx, i, j, k, nx, ny, nz);
    }
    int tot;
    long long w = boff[blockIdx.x] + block_excl_scan<int, EDGE_BLOCK>(__popc(f), lds, &tot);
    for (int a = 0; a < 3; ++a)
        if (f & (1 << a)) {
            if (w < cap) keys[w] = 3 * idx + a;
            ++w;
        }
}

// ------------------------------------------------------------ root finding

__device__ inline double horner(const double *c, int deg, double u) {
    double v = c[deg];
    for (int q = deg - 1; q >= 0; --q) v = v * u + c[q];
    return v;
}

// Root of the polynomial c (degree deg) in [lo, hi] where its values at the
// ends have opposite signs: Newton steps kept inside a shrinking bracket,
// bisection when a step leaves it.
template <bool CNT>
__device__ double bracket_root(const double *c, int deg, double lo, double hi, double flo,
                               unsigned long long *cnt) {
    double d[4];
    for (int q = 1; q <= deg; ++q) d[q - 1] = q * c[q];
    double x = 0.5 * (lo + hi);
    for (int it = 0; it < 128; ++it) {
        if (CNT) cnt[EC_HORNER_FLOPS] += 4 * deg + 4;  // f, f' and the step
        double f = horner(c, deg, x);
        if (f == 0.0) return x;
        if ((f < 0.0) == (flo < 0.0)) lo = x;
        else hi = x;
        double df = horner(d, deg - 1, x);
        double xn = x - f / df;
        if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
        if (fabs(xn - x) <= 1e-17 || hi - lo <= 2e-16) return xn;
        x = xn;
    }
    return x;
}

// Real roots in [0, 1] of a u^2 + b u + c (a > 0), numerically stable form.
__device__ inline int quad01(double a, double b, double c, double *r) {
    double disc = b * b - 4.0 * a * c;
    if (disc < 0.0) return 0;
    double sd = sqrt(disc);
    double q = -0.5 * (b + copysign(sd, b));
    double r1 = q / a;
    double r2 = q != 0.0 ? c / q : r1;
    int n = 0;
    if (r1 >= 0.0 && r1 <= 1.0) r[n++] = r1;
    if (r2 >= 0.0 && r2 <= 1.0 && r2 != r1) r[n++] = r2;
    return n;
}

// Real roots in [0, 1] of the quartic g (ascending coefficients), passed to
// emit in increasing order: the roots of g'' split [0, 1] into intervals
// where g' is monotone, the root of g' found in each splits it further into
// intervals where g is monotone, and each sign change of g on those is
// refined by bracket_root.  Both stages run in one loop, without lists, so
// that each refinement is a single call site.
template <bool CNT, class Emit>
__device__ void quartic01(const double *g, Emit emit, unsigned long long *cnt) {
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
    double fca = horner(g, 4, 0.0);  // g there
    if (fca == 0.0) emit(0.0);
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
                double fa = horner(d1, 3, a), fb = horner(d1, 3, b);
                if (CNT) cnt[EC_HORNER_FLOPS] += 12;
                if (fa == 0.0 && a > 0.0) {
                    cp = a;
                    have = true;
                } else if (fa != 0.0 && fb != 0.0 && ((fa < 0.0) != (fb < 0.0))) {
                    cp = bracket_root<CNT>(d1, 3, a, b, fa, cnt);
                    have = true;
                }
            }
        }
        if (!have || !(cp > ca)) continue;
        double fb = horner(g, 4, cp);
        if (CNT) cnt[EC_HORNER_FLOPS] += 16;
        if (fb == 0.0) emit(cp);
        else if (fca != 0.0 && ((fca < 0.0) != (fb < 0.0)))
            emit(bracket_root<CNT>(g, 4, ca, cp, fca, cnt));
        if (interior && fb != 0.0 && fabs(fb) <= tol) emit(cp);
        ca = cp;
        fca = fb;
    }
}

// ------------------------------------------------ roots, one wavefront per edge
//
// One wavefront per crossing edge.  Lanes gather the surfaces that reach the
// edge (distance from the edge's midpoint within h/2 of the surface: distance
// to a set is 1-Lipschitz), each lane solves one surface, the roots are
// rank-sorted across lanes in LDS, and the labels of the intervals between
// roots are evaluated cooperatively (lanes split the atoms and candidate
// features, ballots combine).  The walk from s stops at the first interval
// whose label differs from Inside[s]; its start is u*, lambda = 1 - u*.

// A point y of the sphere S_i seen from x along c_i -> x is admissible iff
// (x - c_i) . v_k <= |x - c_i| tau_k for every cut of the face.
template <bool CNT>
__device__ inline bool face_admissible(const Mol &m, int f, double dx, double dy, double dz,
                                       unsigned long long *cnt) {
    double d = sqrt(dx * dx + dy * dy + dz * dz);
    for (int c = m.face_cut_off[f], ce = m.face_cut_off[f + 1]; c < ce; ++c) {
        double4 v = m.face_cut[c];
        if (CNT) ++cnt[EC_CUT];
        if (dx * v.x + dy * v.y + dz * v.z > d * v.w) return false;
    }
    return true;
}

// The circle point nearest to x (w = x - o) is admissible iff
// w_perp . u_k <= |w_perp| T_k for every cut of the circle.
template <bool CNT>
__device__ inline bool circle_admissible(const Mol &m, int ec, double4 n, double wx, double wy,
                                         double wz, unsigned long long *cnt) {
    double t = wx * n.x + wy * n.y + wz * n.z;
    double px = wx - t * n.x, py = wy - t * n.y, pz = wz - t * n.z;
    double b = sqrt(px * px + py * py + pz * pz);
    if (!(b > 0.0)) {
        perp_unit(n.x, n.y, n.z, px, py, pz);
        b = 1.0;
    }
    for (int c = m.ec_cut_off[ec], ce = m.ec_cut_off[ec + 1]; c < ce; ++c) {
        double4 u = m.ec_cut[c];
        if (CNT) ++cnt[EC_CUT];
        if (px * u.x + py * u.y + pz * u.z > b * u.w) return false;
    }
    return true;
}

__device__ inline void sort3(int &a, int &b, int &c) {
    int t;
    if (a > b) { t = a; a = b; b = t; }
    if (b > c) { t = b; b = c; c = t; }
    if (a > b) { t = a; a = b; b = t; }
}

// Visibility of LDS writes of a wavefront to its other lanes.
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline bool face_reaches(const Mol &m, int f, const double *mid, double half) {
    double4 a = m.atom[m.face_atom[f]];
    double dm2 = sq(mid[0] - a.x) + sq(mid[1] - a.y) + sq(mid[2] - a.z);
    return !(dm2 > sq(a.w + half) || (a.w > half && dm2 < sq(a.w - half)));
}

__device__ inline bool probe_reaches(const Mol &m, int v, const double *mid, double half) {
    double4 c = m.vert_p[v];
    double dm2 = sq(mid[0] - c.x) + sq(mid[1] - c.y) + sq(mid[2] - c.z);
    return !(dm2 > sq(m.rho + half) || (m.rho > half && dm2 < sq(m.rho - half)));
}

__device__ inline bool torus_reaches(const Mol &m, int ec, const double *mid, double half) {
    int ci = m.ec_circ[ec];
    double4 oR = m.circ_oR[ci];
    double4 nn = m.circ_n[ci];
    double dm0 = mid[0] - oR.x, dm1 = mid[1] - oR.y, dm2 = mid[2] - oR.z;
    double tm = dm0 * nn.x + dm1 * nn.y + dm2 * nn.z;
    double bm = sqrt(fmax(0.0, dm0 * dm0 + dm1 * dm1 + dm2 * dm2 - tm * tm));
    double dc2 = tm * tm + sq(bm - oR.w);  // squared distance of the midpoint from the circle
    return !(dc2 > sq(m.rho + half) || (m.rho > half && dc2 < sq(m.rho - half)));
}

constexpr int EW_WAVES = 4;      // edges (wavefronts) per workgroup
constexpr int EW_THREADS = EW_WAVES * WAVE;
constexpr int EW_SURF = 128;     // reaching surfaces kept per edge
constexpr int EW_ROOTS = 128;    // roots kept per edge

struct EdgeWaveLds {
    int surf[EW_SURF];
    double u[EW_ROOTS];
    int k[EW_ROOTS];
    double su[EW_ROOTS];
    int sk[EW_ROOTS];
    int nroot;
};

// Appends a root (position u along the edge, owner key) to the wavefront's
// list; the order of appends is irrelevant (the list is rank-sorted).
__device__ inline void push_root(EdgeWaveLds &S, double u, int key) {
    int pos = atomicAdd(&S.nroot, 1);
    if (pos < EW_ROOTS) {
        S.u[pos] = u;
        S.k[pos] = key;
    }
}

// Roots in [0, 1] of one surface (type 1 face f, 3 probe v, 2 exposed circle
// ec) along the edge x(u) = xs + u h e, appended to the wavefront's list with
// the key (type << 28) | id.
template <bool CNT>
__device__ void surface_roots(const Mol &m, int key, const double *e, const double *xs,
                              EdgeWaveLds &S, unsigned long long *cnt) {
    const double h = m.h, rho = m.rho;
    const int type = key >> 28, id = key & ((1 << 28) - 1);
    if (type != 2) {
        // sphere |x(u) - c|^2 = r^2: a van der Waals face or a probe
        double4 c = type == 1 ? m.atom[m.face_atom[id]] : m.vert_p[id];
        double r = type == 1 ? c.w : rho;
        if (CNT) ++cnt[EC_QUAD];
        double w0[3] = {xs[0] - c.x, xs[1] - c.y, xs[2] - c.z};
        double we = w0[0] * e[0] + w0[1] * e[1] + w0[2] * e[2];
        double tmp[2];
        int n = quad01(h * h, 2.0 * h * we,
                       w0[0] * w0[0] + w0[1] * w0[1] + w0[2] * w0[2] - r * r, tmp);
        if (n > 0) push_root(S, tmp[0], key);
        if (n > 1) push_root(S, tmp[1], key);
        return;
    }
    // torus (|w|^2 + R^2 - rho^2)^2 = 4 R^2 |w_perp|^2 of the circle's
    // points at distance rho; both branches (the far one is dropped later)
    const int ci = m.ec_circ[id];
    const double4 oR = m.circ_oR[ci];
    const double4 nn = m.circ_n[ci];
    const double R = oR.w;
    const double w0[3] = {xs[0] - oR.x, xs[1] - oR.y, xs[2] - oR.z};
    const double ww = w0[0] * w0[0] + w0[1] * w0[1] + w0[2] * w0[2];
    const double t0 = w0[0] * nn.x + w0[1] * nn.y + w0[2] * nn.z;
    const double we = w0[0] * e[0] + w0[1] * e[1] + w0[2] * e[2];
    const double ne = nn.x * e[0] + nn.y * e[1] + nn.z * e[2];
    const double RR = R * R;
    const double a0 = ww + RR - rho * rho, a1 = 2.0 * h * we, a2 = h * h;
    const double b0 = ww - t0 * t0, b1 = 2.0 * h * (we - t0 * ne), b2 = h * h * (1.0 - ne * ne);
    const double g[5] = {a0 * a0 - 4.0 * RR * b0, 2.0 * a0 * a1 - 4.0 * RR * b1,
                         a1 * a1 + 2.0 * a0 * a2 - 4.0 * RR * b2, 2.0 * a1 * a2, a2 * a2};
    if (CNT) ++cnt[EC_QUARTIC];
    quartic01<CNT>(g, [&](double u) { push_root(S, u, key); }, cnt);
}

// Whether a root is kept: only if the point of A that would put it on the
// boundary is admissible, the radial projection onto the exposed face (van
// der Waals roots) or the nearest point of the exposed circle on the near
// branch of the torus (torus roots).  Every label change lies on such a
// point, so dropping the others is exact.  Probe roots are always kept.
template <bool CNT>
__device__ bool root_admissible(const Mol &m, int key, double u, const double *e,
                                const double *xs, unsigned long long *cnt) {
    const int type = key >> 28, id = key & ((1 << 28) - 1);
    if (type == 3) return true;
    const double s = u * m.h;
    if (type == 1) {
        double4 a = m.atom[m.face_atom[id]];
        return face_admissible<CNT>(m, id, xs[0] - a.x + s * e[0], xs[1] - a.y + s * e[1],
                                    xs[2] - a.z + s * e[2], cnt);
    }
    const int ci = m.ec_circ[id];
    const double4 oR = m.circ_oR[ci];
    const double4 nn = m.circ_n[ci];
    const double R = oR.w, rho = m.rho;
    double x0 = xs[0] - oR.x + s * e[0], x1 = xs[1] - oR.y + s * e[1],
           x2 = xs[2] - oR.z + s * e[2];
    double tt = x0 * nn.x + x1 * nn.y + x2 * nn.z;
    double bb = sqrt(fmax(0.0, x0 * x0 + x1 * x1 + x2 * x2 - tt * tt));
    double near = fabs(sq(bb - R) + tt * tt - rho * rho);
    double far = fabs(sq(bb + R) + tt * tt - rho * rho);
    return near <= far && circle_admissible<CNT>(m, id, nn, x0, x1, x2, cnt);
}

// Inside/outside of x (eq. 2) evaluated by the whole wavefront: the three
// cases of the classification with lanes splitting the tile's atoms and
// candidate features.
template <bool CNT>
__device__ int label_wave(const Mol &m, int tile, double x, double y, double z,
                          unsigned long long *cnt) {
    const int lane = lane_id();
    const double rho = m.rho, rho2 = rho * rho;
    bool inU = false;
    for (int base = m.tA_off[tile], e = m.tA_off[tile + 1]; base < e; base += WAVE) {
        int q = base + lane;
        bool v = false, u = false;
        if (q < e) {
            double4 a = m.atom[m.tA[q]];
            double dx = x - a.x, dy = y - a.y, dz = z - a.z;
            double d2 = dx * dx + dy * dy + dz * dz;
            if (CNT) ++cnt[EC_L_ATOM];
            v = d2 <= a.w * a.w;
            u = d2 < sq(a.w + rho);
        }
        if (__any(v)) return 1;
        inU = inU || __any(u);
    }
    if (!inU) return 0;
    for (int base = m.tV_off[tile], e = m.tV_off[tile + 1]; base < e; base += WAVE) {
        int q = base + lane;
        bool hit = false;
        if (q < e) {
            double4 p = m.vert_p[m.tV[q]];
            if (CNT) ++cnt[EC_L_VERTEX];
            hit = sq(x - p.x) + sq(y - p.y) + sq(z - p.z) < rho2;
        }
        if (__any(hit)) return 0;
    }
    for (int base = m.tF_off[tile], e = m.tF_off[tile + 1]; base < e; base += WAVE) {
        int q = base + lane;
        bool hit = false;
        if (q < e) {
            int f = m.tF[q];
            double4 a = m.atom[m.face_atom[f]];
            double dx = x - a.x, dy = y - a.y, dz = z - a.z;
            double d2 = dx * dx + dy * dy + dz * dz;
            if (CNT) ++cnt[EC_L_FACE];
            if (d2 < sq(a.w + 2.0 * rho)) {
                double d = sqrt(d2);
                hit = true;
                for (int c = m.face_cut_off[f], ce = m.face_cut_off[f + 1]; c < ce; ++c) {
                    double4 v = m.face_cut[c];
                    if (CNT) ++cnt[EC_L_FACE_CUT];
                    if (dx * v.x + dy * v.y + dz * v.z > d * v.w) {
                        hit = false;
                        break;
                    }
                }
            }
        }
        if (__any(hit)) return 0;
    }
    for (int base = m.tC_off[tile], e = m.tC_off[tile + 1]; base < e; base += WAVE) {
        int q = base + lane;
        bool hit = false;
        if (q < e) {
            int ec = m.tC[q];
            int ci = m.ec_circ[ec];
            double4 oR = m.circ_oR[ci];
            double4 n = m.circ_n[ci];
            double wx = x - oR.x, wy = y - oR.y, wz = z - oR.z;
            double t = wx * n.x + wy * n.y + wz * n.z;
            double ww = wx * wx + wy * wy + wz * wz;
            double b = sqrt(fmax(ww - t * t, 0.0));
            double R = oR.w;
            if (CNT) ++cnt[EC_L_CIRCLE];
            if (ww + R * R - rho2 < 2.0 * b * R) {
                double px = wx, py = wy, pz = wz, pb = b;
                if (!(b > 0.0)) {
                    perp_unit(n.x, n.y, n.z, px, py, pz);
                    pb = 1.0;
                }
                hit = true;
                for (int c = m.ec_cut_off[ec], ce = m.ec_cut_off[ec + 1]; c < ce; ++c) {
                    double4 u = m.ec_cut[c];
                    if (CNT) ++cnt[EC_L_CIRCLE_CUT];
                    if (px * u.x + py * u.y + pz * u.z > pb * u.w) {
                        hit = false;
                        break;
                    }
                }
            }
        }
        if (__any(hit)) return 0;
    }
    return 1;
}

// CNT: the statistics pass (not timed); it tallies the work into
// `work[EC_COUNT]` and writes no record.
template <bool CNT>
__global__ void __launch_bounds__(EW_THREADS)
    k_edge_roots(Mol m, const uint8_t *L, const long long *keys, long long count, double *lam,
                 double *nrm, uint8_t *ptype, int *patoms, int *overflow, const int *order,
                 int nblocks, unsigned long long *work) {
    __shared__ EdgeWaveLds lds[EW_WAVES];
    const int w = threadIdx.x / WAVE, lane = lane_id();
    // edges grouped by tile (order); consecutive groups stay on one XCD
    const int blk = xcd_tile(blockIdx.x, nblocks, (int)((count + EW_WAVES - 1) / EW_WAVES));
    if (blk < 0) return;  // uniform across the workgroup
    const long long g = (long long)blk * EW_WAVES + w;
    if (g >= count) return;  // uniform across the wavefront; no workgroup barrier below
    EdgeWaveLds &S = lds[w];
    unsigned long long cnt[CNT ? EC_COUNT : 1];
    for (int c = 0; c < (CNT ? (int)EC_COUNT : 1); ++c) cnt[c] = 0;

    const long long q = order[g];
    const long long key = keys[q];
    const int axis = (int)(key % 3);
    const long long idx = key / 3;
    const int nx = m.dims[0], ny = m.dims[1];
    const int i0 = (int)(idx % nx), i1 = (int)((idx / nx) % ny),
              i2 = (int)(idx / ((long long)nx * ny));
    const long long step = axis == 0 ? 1 : axis == 1 ? (long long)nx : (long long)nx * ny;
    const int Ls = L[idx], Lt = L[idx + step];
    const int tile = i0 / m.tile + m.tdims[0] * (i1 / m.tile + m.tdims[1] * (i2 / m.tile));
    const double h = m.h;
    // the edge x(u) = xs + u h e, u in [0, 1]
    const double e[3] = {axis == 0 ? 1.0 : 0.0, axis == 1 ? 1.0 : 0.0, axis == 2 ? 1.0 : 0.0};
    const double xs[3] = {grid_coord(m.lo[0], h, i0), grid_coord(m.lo[1], h, i1),
                          grid_coord(m.lo[2], h, i2)};
    const double hh = 0.5 * h;
    const double mid[3] = {xs[0] + hh * e[0], xs[1] + hh * e[1], xs[2] + hh * e[2]};
    const double half = 0.5 * h + 1e-9;
    bool ovf = false;
    if (lane == 0) S.nroot = 0;

    // 1. surfaces reaching the edge, compacted with ballots
    int ns = 0;
    for (int base = m.tF_off[tile], end = m.tF_off[tile + 1]; base < end; base += WAVE) {
        int p = base + lane;
        int f = p < end ? m.tF[p] : 0;
        bool r = p < end && face_reaches(m, f, mid, half);
        if (CNT && p < end) ++cnt[EC_REACH_SPHERE];
        unsigned long long bm = __ballot(r);
        int pos = ns + mask_prefix(bm);
        if (r && pos < EW_SURF) S.surf[pos] = (1 << 28) | f;
        ns += __popcll(bm);
    }
    for (int base = m.tV_off[tile], end = m.tV_off[tile + 1]; base < end; base += WAVE) {
        int p = base + lane;
        int v = p < end ? m.tV[p] : 0;
        bool r = p < end && probe_reaches(m, v, mid, half);
        if (CNT && p < end) ++cnt[EC_REACH_SPHERE];
        unsigned long long bm = __ballot(r);
        int pos = ns + mask_prefix(bm);
        if (r && pos < EW_SURF) S.surf[pos] = (3 << 28) | v;
        ns += __popcll(bm);
    }
    for (int base = m.tC_off[tile], end = m.tC_off[tile + 1]; base < end; base += WAVE) {
        int p = base + lane;
        int ec = p < end ? m.tC[p] : 0;
        bool r = p < end && torus_reaches(m, ec, mid, half);
        if (CNT && p < end) ++cnt[EC_REACH_TORUS];
        unsigned long long bm = __ballot(r);
        int pos = ns + mask_prefix(bm);
        if (r && pos < EW_SURF) S.surf[pos] = (2 << 28) | ec;
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
        if (si < ns) surface_roots<CNT>(m, S.surf[si], e, xs, S, cnt);
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
            keep = root_admissible<CNT>(m, k, u, e, xs, cnt);
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

    // 5. walk the intervals from s (uniform across the wavefront).  The label
    // is constant between consecutive roots; the first interval has
    // Inside[s] and the last Inside[t] unless a root sits exactly on that end.
    const bool root0 = nr > 0 && S.u[0] == 0.0;
    const bool root1 = nr > 0 && S.u[nr - 1] == 1.0;
    double ustar = 1.0, prev = 0.0;
    int prev_key = -1, owner_key = -1;
    bool found = false;
    for (int r = 0; r <= nr; ++r) {
        double next = r < nr ? S.u[r] : 1.0;
        if (next > prev) {
            int lab;
            if (prev == 0.0 && !root0) {
                lab = Ls;
            } else if (r == nr && !root1) {
                lab = Lt;
            } else {
                double um = 0.5 * (prev + next) * h;
                if (CNT && lane == 0) ++cnt[EC_LABEL];
                lab = label_wave<CNT>(m, tile, xs[0] + um * e[0], xs[1] + um * e[1],
                                      xs[2] + um * e[2], cnt);
            }
            if (lab != Ls) {
                ustar = prev;
                owner_key = prev_key;
                found = true;
                break;
            }
        }
        // owner of a position: the smallest key among the roots there
        if (r < nr && (prev_key < 0 || next > prev)) prev_key = S.k[r];
        if (next > prev) prev = next;
    }
    // no change inside the edge: it happens at t itself (the last root)
    if (!found) owner_key = prev_key;
    if (__any(ovf) && lane == 0) *overflow = 1;
    if (CNT) {
        if (lane == 0) cnt[EC_EDGES] = 1;
        // untimed statistics pass: one atomic per lane and counter
        for (int c = 0; c < EC_COUNT; ++c)
            if (cnt[c]) atomicAdd(&work[c], cnt[c]);
        return;
    }
    if (lane != 0) return;

    // 6. the record: normal of the owning surface at x(u*), atoms of its patch
    const double us = ustar * h;
    const double xst[3] = {xs[0] + us * e[0], xs[1] + us * e[1], xs[2] + us * e[2]};
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
    lam[q] = 1.0 - ustar;
    nrm[3 * q] = n3[0];
    nrm[3 * q + 1] = n3[1];
    nrm[3 * q + 2] = n3[2];
    ptype[q] = (uint8_t)type;
    patoms[3 * q] = at0;
    patoms[3 * q + 1] = at1;
    patoms[3 * q + 2] = at2;
}


// Permutation of the crossing edges grouping them by the tile owning s
// (counting sort; the order inside a tile is not used by any result).
__device__ inline int edge_tile(const Mol &m, long long key) {
    long long idx = key / 3;
    const int nx = m.dims[0], ny = m.dims[1];
    int i = (int)(idx % nx), j = (int)((idx / nx) % ny), k = (int)(idx / ((long long)nx * ny));
    return i / m.tile + m.tdims[0] * (j / m.tile + m.tdims[1] * (k / m.tile));
}

__global__ void k_edge_tile_count(Mol m, const long long *keys, long long count, int *tcount) {
    long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (q >= count) return;
    atomicAdd(&tcount[edge_tile(m, keys[q])], 1);
}

__global__ void k_edge_tile_scatter(Mol m, const long long *keys, long long count, int *tfill,
                                    int *order) {
    long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (q >= count) return;
    order[atomicAdd(&tfill[edge_tile(m, keys[q])], 1)] = (int)q;
}

hipError_t launch_edge_group(const Mol &m, const long long *keys, long long count, int *tcount,
                             int *tfill, int *order, int *tmp, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    unsigned nb = (unsigned)((count + 255) / 256);
    hipError_t e = fill_i32(tcount, m.ntiles + 1, 0, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_edge_tile_count, dim3(nb), dim3(256), 0, st, m, keys, count, tcount);
    e = scan_i32(tcount, m.ntiles, tfill, tmp, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_edge_tile_scatter, dim3(nb), dim3(256), 0, st, m, keys, count, tfill,
                       order);
    return hipGetLastError();
}

hipError_t launch_edge_detect_count(const uint8_t *L, const Mol &m, int *bcount, long long *nblk,
                                    hipStream_t st) {
    long long nb = (m.npts + EDGE_BLOCK - 1) / EDGE_BLOCK;
    if (nb < 1) nb = 1;
    *nblk = nb;
    hipLaunchKernelGGL(k_edge_count, dim3((unsigned)nb), dim3(EDGE_BLOCK), 0, st, L, m.dims[0],
                       m.dims[1], m.dims[2], m.npts, bcount);
    return hipGetLastError();
}

hipError_t launch_edge_detect_write(const uint8_t *L, const Mol &m, const long long *boff,
                                    long long cap, long long *keys, hipStream_t st) {
    long long nb = (m.npts + EDGE_BLOCK - 1) / EDGE_BLOCK;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_edge_write, dim3((unsigned)nb), dim3(EDGE_BLOCK), 0, st, L, m.dims[0],
                       m.dims[1], m.dims[2], m.npts, boff, cap, keys);
    return hipGetLastError();
}

hipError_t launch_edge_roots(const Mol &m, const uint8_t *L, const long long *keys,
                             long long count, double *lam, double *nrm, uint8_t *ptype,
                             int *patoms, int *overflow, const int *order, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    int nb = (int)((count + EW_WAVES - 1) / EW_WAVES);
    nb = (nb + NXCD - 1) / NXCD * NXCD;
    hipLaunchKernelGGL(k_edge_roots<false>, dim3(nb), dim3(EW_THREADS), 0, st, m, L, keys, count,
                       lam, nrm, ptype, patoms, overflow, order, nb, nullptr);
    return hipGetLastError();
}

hipError_t launch_edge_work(const Mol &m, const uint8_t *L, const long long *keys,
                            long long count, const int *order, int *overflow,
                            unsigned long long *work, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    int nb = (int)((count + EW_WAVES - 1) / EW_WAVES);
    nb = (nb + NXCD - 1) / NXCD * NXCD;
    hipLaunchKernelGGL(k_edge_roots<true>, dim3(nb), dim3(EW_THREADS), 0, st, m, L, keys, count,
                       nullptr, nullptr, nullptr, nullptr, overflow, order, nb, work);
    return hipGetLastError();
}

}  // namespace eses
