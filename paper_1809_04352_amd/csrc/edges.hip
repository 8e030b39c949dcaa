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
__device__ double bracket_root(const double *c, int deg, double lo, double hi, double flo) {
    double d[4];
    for (int q = 1; q <= deg; ++q) d[q - 1] = q * c[q];
    double x = 0.5 * (lo + hi);
    for (int it = 0; it < 128; ++it) {
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

// Real roots in [0, 1] of the quartic g (ascending coefficients): the roots
// of g'' split [0, 1] into intervals where g' is monotone, the roots of g'
// found there split it into intervals where g is monotone, and each sign
// change of g on those is refined by bracket_root.
__device__ int quartic01(const double *g, double *out) {
    double br[4];
    int nb = 0;
    br[nb++] = 0.0;
    {
        double a = 12.0 * g[4], b = 6.0 * g[3], c = 2.0 * g[2];
        double r[2];
        int n = 0;
        if (a != 0.0) {
            double disc = b * b - 4.0 * a * c;
            if (disc > 0.0) {
                double sd = sqrt(disc);
                double q = -0.5 * (b + copysign(sd, b));
                r[n++] = q / a;
                if (q != 0.0) r[n++] = c / q;
            }
        } else if (b != 0.0) {
            r[n++] = -c / b;
        }
        if (n == 2 && r[1] < r[0]) {
            double t = r[0];
            r[0] = r[1];
            r[1] = t;
        }
        for (int q = 0; q < n; ++q)
            if (r[q] > 0.0 && r[q] < 1.0) br[nb++] = r[q];
    }
    br[nb++] = 1.0;
    double d1[4] = {g[1], 2.0 * g[2], 3.0 * g[3], 4.0 * g[4]};
    double cp[6];
    int ncp = 0;
    cp[ncp++] = 0.0;
    for (int q = 0; q + 1 < nb; ++q) {
        double a = br[q], b = br[q + 1];
        if (!(b > a)) continue;
        double fa = horner(d1, 3, a), fb = horner(d1, 3, b);
        if (fa == 0.0 && a > 0.0) cp[ncp++] = a;
        else if (fa != 0.0 && fb != 0.0 && ((fa < 0.0) != (fb < 0.0)))
            cp[ncp++] = bracket_root(d1, 3, a, b, fa);
    }
    cp[ncp++] = 1.0;
    // An interior critical point where g vanishes to within rounding is a
    // root of even multiplicity: a line through the self-intersection of a
    // spindle torus on its axis, where the quartic is a perfect square.
    const double tol =
        1e-12 * (fabs(g[0]) + fabs(g[1]) + fabs(g[2]) + fabs(g[3]) + fabs(g[4]));
    int nr = 0;
    double f0 = horner(g, 4, 0.0);
    if (f0 == 0.0) out[nr++] = 0.0;
    for (int q = 0; q + 1 < ncp; ++q) {
        double a = cp[q], b = cp[q + 1];
        if (!(b > a)) continue;
        double fa = horner(g, 4, a), fb = horner(g, 4, b);
        if (fb == 0.0) out[nr++] = b;
        else if (fa != 0.0 && ((fa < 0.0) != (fb < 0.0))) out[nr++] = bracket_root(g, 4, a, b, fa);
        if (q + 2 < ncp && fb != 0.0 && fabs(fb) <= tol) out[nr++] = b;
    }
    return nr;
}

constexpr int MAXR = 12;   // roots per page of the walk

// Sorted insertion by (u, type, id) keeping the MAXR smallest roots; a root
// that does not fit marks the list truncated.
__device__ inline void push_root(double *ru, int *rt, int &nr, bool &truncated, double u, int type,
                                 int id) {
    int key = (type << 28) | id;
    if (nr == MAXR) {
        truncated = true;
        if (ru[MAXR - 1] < u || (ru[MAXR - 1] == u && rt[MAXR - 1] <= key)) return;
        --nr;
    }
    int p = nr++;
    while (p > 0 && (ru[p - 1] > u || (ru[p - 1] == u && rt[p - 1] > key))) {
        ru[p] = ru[p - 1];
        rt[p] = rt[p - 1];
        --p;
    }
    ru[p] = u;
    rt[p] = key;
}

// A point y of the sphere S_i seen from x along c_i -> x is admissible iff
// (x - c_i) . v_k <= |x - c_i| tau_k for every cut of the face.
__device__ inline bool face_admissible(const Mol &m, int f, double dx, double dy, double dz) {
    double d = sqrt(dx * dx + dy * dy + dz * dz);
    for (int c = m.face_cut_off[f], ce = m.face_cut_off[f + 1]; c < ce; ++c) {
        double4 v = m.face_cut[c];
        if (dx * v.x + dy * v.y + dz * v.z > d * v.w) return false;
    }
    return true;
}

// The circle point nearest to x (w = x - o) is admissible iff
// w_perp . u_k <= |w_perp| T_k for every cut of the circle.
__device__ inline bool circle_admissible(const Mol &m, int ec, double4 n, double wx, double wy,
                                         double wz) {
    double t = wx * n.x + wy * n.y + wz * n.z;
    double px = wx - t * n.x, py = wy - t * n.y, pz = wz - t * n.z;
    double b = sqrt(px * px + py * py + pz * pz);
    if (!(b > 0.0)) {
        perp_unit(n.x, n.y, n.z, px, py, pz);
        b = 1.0;
    }
    for (int c = m.ec_cut_off[ec], ce = m.ec_cut_off[ec + 1]; c < ce; ++c) {
        double4 u = m.ec_cut[c];
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

// Surfaces whose distance from the edge's midpoint is within h/2 of zero
// (distance to a set is 1-Lipschitz, so only these can cross the edge) are
// first gathered per lane, so the solves below run over each lane's own short
// list instead of every lane waiting on every other lane's solves.
constexpr int EDGE_THREADS = 256;
constexpr int MAXS = 32;  // surfaces listed per edge; more are solved in place

struct EdgeSurf {
    int n;
    bool more;  // more than MAXS surfaces: the lists are scanned again
};

__device__ inline int surf_slot(int q) { return q * EDGE_THREADS + (int)threadIdx.x; }

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

// Roots u > lower (in [0, 1]) of one surface (type 1 face atom f, 3 probe v,
// 2 exposed circle ec), kept only if the point of A that would put the root
// on the boundary is admissible: the radial projection onto the exposed face
// (van der Waals roots) or the nearest point of the exposed circle (torus
// roots).  Every label change lies on such a point, so dropping the others
// is exact.
__device__ void surface_roots(const Mol &m, int type, int id, int axis,
                                          const double *xs,
                              double lower, double *ru, int *rt, int &nr, bool &truncated) {
    const double h = m.h, rho = m.rho;
    double tmp[4];
    if (type == 1) {
        int f = id;
        int i = m.face_atom[f];
        double4 a = m.atom[i];
        double w0[3] = {xs[0] - a.x, xs[1] - a.y, xs[2] - a.z};
        int n = quad01(h * h, 2.0 * h * w0[axis],
                       w0[0] * w0[0] + w0[1] * w0[1] + w0[2] * w0[2] - a.w * a.w, tmp);
        for (int t = 0; t < n; ++t) {
            if (!(tmp[t] > lower)) continue;
            double x[3] = {w0[0], w0[1], w0[2]};
            x[axis] += tmp[t] * h;
            if (face_admissible(m, f, x[0], x[1], x[2]))
                push_root(ru, rt, nr, truncated, tmp[t], 1, i);
        }
    } else if (type == 3) {
        int v = id;
        double4 c = m.vert_p[v];
        double w0[3] = {xs[0] - c.x, xs[1] - c.y, xs[2] - c.z};
        int n = quad01(h * h, 2.0 * h * w0[axis],
                       w0[0] * w0[0] + w0[1] * w0[1] + w0[2] * w0[2] - rho * rho, tmp);
        for (int t = 0; t < n; ++t)
            if (tmp[t] > lower) push_root(ru, rt, nr, truncated, tmp[t], 3, v);
    } else {
        // torus (|w|^2 + R^2 - rho^2)^2 = 4 R^2 |w_perp|^2, the branch at
        // distance rho from the near circle point
        int ec = id;
        int ci = m.ec_circ[ec];
        double4 oR = m.circ_oR[ci];
        double4 nn = m.circ_n[ci];
        double R = oR.w;
        double w0[3] = {xs[0] - oR.x, xs[1] - oR.y, xs[2] - oR.z};
        double nv[3] = {nn.x, nn.y, nn.z};
        double ww = w0[0] * w0[0] + w0[1] * w0[1] + w0[2] * w0[2];
        double t0 = w0[0] * nv[0] + w0[1] * nv[1] + w0[2] * nv[2];
        double RR = R * R;
        double a0 = ww + RR - rho * rho, a1 = 2.0 * h * w0[axis], a2 = h * h;
        double b0 = ww - t0 * t0, b1 = 2.0 * h * (w0[axis] - t0 * nv[axis]),
               b2 = h * h * (1.0 - nv[axis] * nv[axis]);
        double g[5] = {a0 * a0 - 4.0 * RR * b0, 2.0 * a0 * a1 - 4.0 * RR * b1,
                       a1 * a1 + 2.0 * a0 * a2 - 4.0 * RR * b2, 2.0 * a1 * a2, a2 * a2};
        double r4[10];
        int n = quartic01(g, r4);
        for (int t = 0; t < n; ++t) {
            if (!(r4[t] > lower)) continue;
            double x[3] = {w0[0], w0[1], w0[2]};
            x[axis] += r4[t] * h;
            double tt = x[0] * nv[0] + x[1] * nv[1] + x[2] * nv[2];
            double bb = sqrt(fmax(0.0, x[0] * x[0] + x[1] * x[1] + x[2] * x[2] - tt * tt));
            double near = fabs(sq(bb - R) + tt * tt - rho * rho);
            double far = fabs(sq(bb + R) + tt * tt - rho * rho);
            if (near <= far && circle_admissible(m, ec, nn, x[0], x[1], x[2]))
                push_root(ru, rt, nr, truncated, r4[t], 2, ec);
        }
    }
}

// The edge's reaching surfaces with index in [skip, skip + MAXS), packed
// (type << 28 | id) in LDS; `more` if there are further ones.
__device__ EdgeSurf gather_surfaces(const Mol &m, int tile, const double *mid, int *slots,
                                    int skip) {
    const double half = 0.5 * m.h + 1e-9;
    EdgeSurf es = {0, false};
    int seen = 0;
    for (int p = m.tF_off[tile], e = m.tF_off[tile + 1]; p < e; ++p) {
        int f = m.tF[p];
        if (!face_reaches(m, f, mid, half) || seen++ < skip) continue;
        if (es.n < MAXS) slots[surf_slot(es.n++)] = (1 << 28) | f;
        else es.more = true;
    }
    for (int p = m.tV_off[tile], e = m.tV_off[tile + 1]; p < e; ++p) {
        int v = m.tV[p];
        if (!probe_reaches(m, v, mid, half) || seen++ < skip) continue;
        if (es.n < MAXS) slots[surf_slot(es.n++)] = (3 << 28) | v;
        else es.more = true;
    }
    for (int p = m.tC_off[tile], e = m.tC_off[tile + 1]; p < e; ++p) {
        int ec = m.tC[p];
        if (!torus_reaches(m, ec, mid, half) || seen++ < skip) continue;
        if (es.n < MAXS) slots[surf_slot(es.n++)] = (2 << 28) | ec;
        else es.more = true;
    }
    return es;
}

// All roots u > lower of the edge's reaching surfaces (the MAXR smallest).
// `es` describes the first window of surfaces in `slots`; further windows
// (rare) are gathered in turn and the first one is restored at the end.
__device__ void collect_roots(const Mol &m, int tile, int axis, const double *xs,
                              const double *mid, int *slots, EdgeSurf es, double lower,
                              double *ru, int *rt, int &nr, bool &truncated) {
    nr = 0;
    truncated = false;
    int skip = 0;
    for (;;) {
        for (int q = 0; q < es.n; ++q) {
            int s = slots[surf_slot(q)];
            surface_roots(m, s >> 28, s & ((1 << 28) - 1), axis, xs, lower, ru, rt, nr, truncated);
        }
        if (!es.more) break;
        skip += MAXS;
        es = gather_surfaces(m, tile, mid, slots, skip);
    }
    if (skip > 0) gather_surfaces(m, tile, mid, slots, 0);
}

__global__ void __launch_bounds__(EDGE_THREADS) k_edge_roots(Mol m, const uint8_t *L, const long long *keys,
                                                    long long count, double *lam, double *nrm,
                                                    uint8_t *ptype, int *patoms, int *overflow,
                                                    const int *order, int nblocks) {
    // edges grouped by tile (order), consecutive groups on one XCD
    int blk = xcd_tile(blockIdx.x, nblocks, (int)((count + EDGE_THREADS - 1) / EDGE_THREADS));
    if (blk < 0) return;
    long long g = (long long)blk * EDGE_THREADS + threadIdx.x;
    if (g >= count) return;
    const long long q = order[g];
    long long key = keys[q];
    int axis = (int)(key % 3);
    long long idx = key / 3;
    const int nx = m.dims[0], ny = m.dims[1];
    int ii[3] = {(int)(idx % nx), (int)((idx / nx) % ny), (int)(idx / ((long long)nx * ny))};
    const long long stride[3] = {1, nx, (long long)nx * ny};
    int Ls = L[idx], Lt = L[idx + stride[axis]];
    int tile = ii[0] / m.tile + m.tdims[0] * (ii[1] / m.tile + m.tdims[1] * (ii[2] / m.tile));
    double xs[3];
    for (int a = 0; a < 3; ++a) xs[a] = grid_coord(m.lo[a], m.h, ii[a]);
    const double h = m.h, rho = m.rho;
    double mid[3] = {xs[0], xs[1], xs[2]};
    mid[axis] += 0.5 * h;

    __shared__ int slots[MAXS * EDGE_THREADS];
    const EdgeSurf es = gather_surfaces(m, tile, mid, slots, 0);
    double ru[MAXR];
    int rt[MAXR];
    int nr = 0;
    bool truncated = false;

    // Walk the intervals from s.  The label is constant between consecutive
    // roots; the first interval has Inside[s] and the last Inside[t] unless a
    // root sits exactly on that end.  Roots come in pages of the MAXR smallest
    // above the last one walked; a page that ends before t is followed by the
    // next one.
    double ustar = 1.0;
    double prev = 0.0;
    int prev_key = -1, owner_key = -1;
    bool found = false;
    for (int page = 0; page < 64; ++page) {
        const bool first = page == 0;
        collect_roots(m, tile, axis, xs, mid, slots, es, first ? -1.0 : prev, ru, rt, nr,
                      truncated);
        bool root0 = first && nr > 0 && ru[0] == 0.0;
        bool root1 = !truncated && nr > 0 && ru[nr - 1] == 1.0;
        for (int r = 0; r <= nr; ++r) {
            if (r == nr && truncated) break;
            double next = r < nr ? ru[r] : 1.0;
            if (next > prev) {
                int lab;
                if (first && prev == 0.0 && !root0) lab = Ls;
                else if (r == nr && !root1) lab = Lt;
                else {
                    double x[3] = {xs[0], xs[1], xs[2]};
                    x[axis] += 0.5 * (prev + next) * h;
                    lab = label_fp64(m, tile, x[0], x[1], x[2]);
                }
                if (lab != Ls) {
                    ustar = prev;
                    owner_key = prev_key;
                    found = true;
                    break;
                }
            }
            if (r < nr && (prev_key < 0 || next > prev)) prev_key = rt[r];
            if (next > prev) prev = next;
        }
        if (found || !truncated) break;
        if (page == 63) *overflow = 1;
    }
    // no change inside the edge: it happens at t itself (the last root)
    if (!found) owner_key = prev_key;
    double xst[3] = {xs[0], xs[1], xs[2]};
    xst[axis] += ustar * h;
    double n3[3] = {0.0, 0.0, 0.0};
    int type = 0, at[3] = {-1, -1, -1};
    if (owner_key >= 0) {
        type = owner_key >> 28;
        int id = owner_key & ((1 << 28) - 1);
        double y[3];
        if (type == 1) {
            double4 a = m.atom[id];
            y[0] = xst[0] - a.x;
            y[1] = xst[1] - a.y;
            y[2] = xst[2] - a.z;
            at[0] = m.orig[id];
        } else if (type == 2) {
            int ci = m.ec_circ[id];
            double4 oR = m.circ_oR[ci];
            double4 nn = m.circ_n[ci];
            double w[3] = {xst[0] - oR.x, xst[1] - oR.y, xst[2] - oR.z};
            double t = w[0] * nn.x + w[1] * nn.y + w[2] * nn.z;
            double wp[3] = {w[0] - t * nn.x, w[1] - t * nn.y, w[2] - t * nn.z};
            double b = sqrt(wp[0] * wp[0] + wp[1] * wp[1] + wp[2] * wp[2]);
            double u[3];
            if (b > 0.0) {
                u[0] = wp[0] / b;
                u[1] = wp[1] / b;
                u[2] = wp[2] / b;
            } else {
                perp_unit(nn.x, nn.y, nn.z, u[0], u[1], u[2]);
            }
            for (int a = 0; a < 3; ++a)
                y[a] = ((a == 0 ? oR.x : a == 1 ? oR.y : oR.z) + oR.w * u[a]) - xst[a];
            at[0] = m.orig[m.circ_i[ci]];
            at[1] = m.orig[m.circ_j[ci]];
            if (at[0] > at[1]) {
                int t2 = at[0];
                at[0] = at[1];
                at[1] = t2;
            }
        } else {
            double4 p = m.vert_p[id];
            y[0] = p.x - xst[0];
            y[1] = p.y - xst[1];
            y[2] = p.z - xst[2];
            int4 v = m.vert_ijks[id];
            at[0] = m.orig[v.x];
            at[1] = m.orig[v.y];
            at[2] = m.orig[v.z];
            sort3(at[0], at[1], at[2]);
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
    patoms[3 * q] = at[0];
    patoms[3 * q + 1] = at[1];
    patoms[3 * q + 2] = at[2];
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
    int nb = (int)((count + EDGE_THREADS - 1) / EDGE_THREADS);
    nb = (nb + NXCD - 1) / NXCD * NXCD;
    hipLaunchKernelGGL(k_edge_roots, dim3(nb), dim3(EDGE_THREADS), 0, st, m, L, keys, count, lam, nrm,
                       ptype, patoms, overflow, order, nb);
    return hipGetLastError();
}

}  // namespace eses
