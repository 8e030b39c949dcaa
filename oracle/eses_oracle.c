/*
 * eses_oracle.c -- plain FP64 CPU oracle for the Eulerian solvent-excluded
 * surface (ESES) hot path.  TEST INFRASTRUCTURE ONLY: it is called by the
 * tests, by the smoke check and by the CPU-baseline leg of the benchmark, never
 * by the product path, and it shares no code with the HIP library.
 *
 * What it computes (Zhao, Wang, Tong, Wei, "Divide-and-Conquer Strategy for
 * Large-Scale Eulerian Solvent Excluded Surface", arXiv 1809.04352):
 *
 *   input   atoms (c_i, r_i), eq. (1); probe radius rho; grid spacing h; box.
 *   labels  Inside[i,j,k] = 1 iff the grid point lies in M, the volume enclosed
 *           by the SES, eq. (2).  The SES is the boundary of the union of all
 *           probe balls that do not overlap an atom (section 1), so with SAS
 *           radii s_i = r_i + rho, U = union of open balls B(c_i, s_i) and
 *           A = R^3 \ U (the admissible probe centres, a closed set):
 *               M = { x : dist(x, A) >= rho }   (closed: the surface is inside).
 *   vertices the concave-patch probe positions: points on three SAS spheres
 *           that lie in A (a probe touching three atoms and overlapping none,
 *           section 1).
 *   edges   for each axis edge st with Inside[s] != Inside[t] (eq. 3), the
 *           first point where the label changes walking from s to t, written
 *           p = lambda s + (1 - lambda) t (eq. 4), with the outward unit
 *           normal and the patch that carries it (section 1: convex, saddle,
 *           concave; section 4.1: the nearby atoms of each intersection).
 *
 * How the distance is evaluated.  For x in U the nearest point of A lies on
 * the boundary of U, i.e. on some SAS sphere S_i outside every other open ball.
 * On the exposed part of S_i the minimum of |x - y| is either the radial
 * projection of x onto S_i or lies on a bounding circle S_i ^ S_j; on an
 * exposed arc it is either the nearest circle point or an arc end, which is a
 * point on three spheres.  Hence
 *     dist(x, A) = min |x - y| over the candidates y in A among
 *       (F) radial projections onto each S_i,
 *       (E) nearest points of each circle S_i ^ S_j,
 *       (V) the exposed three-sphere points,
 * and a candidate is "in A" iff |y - c_k| >= s_k for every atom k.  The label
 * follows the definition: 1 inside a closed van der Waals ball (every point
 * of A is then at least rho away), 0 outside U (x itself is in A), otherwise
 * [dist(x, A) >= rho].
 *
 * Readings of points the paper leaves open: interior probe-accessible
 * cavities count as solvent (no flood fill); a point at distance exactly rho
 * is inside (M is closed); a probe touching a fourth atom is still admissible
 * (|p - c| >= s, non-strict); grid point (i,j,k) is lo + (i,j,k) h evaluated
 * as fl(lo + fl(i h)); edges are the six-neighbour axis edges; s is the lower
 * index end, lambda weights s; on an edge with several crossings the first
 * change walking from s is reported; normals point from M into the solvent.
 *
 * Numbers: FP64 throughout; edge roots of tori are isolated and bisected in
 * long double.  Atoms near a point are found with a uniform cell list that
 * only narrows the search to a superset; every decision is an exact-distance
 * comparison.
 *
 * Certification of labels: the grid labels of orc_labels_*_cert carry every
 * comparison's FP64 margin together with a bound on its rounding error (the
 * bounds are stated beside each test below).  A comparison whose margin lies
 * within its bound is undecided; a label that depends on an undecided
 * comparison is returned as 2, and the Python side (oracle/exact.py)
 * re-decides it in exact rational arithmetic on the input doubles.  The
 * labels the oracle reports are therefore those of exact real arithmetic on
 * the given doubles, including points that lie exactly on a sphere, at
 * exactly rho from a probe, or exactly on the boundary of an admissible
 * patch.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int n;
    double rho;
    double *cx, *cy, *cz, *r, *s;
    double smax;
    /* uniform cell list over the atom box */
    double cell, lo[3];
    int nc[3];
    int *cstart; /* [ncell+1] */
    int *catom;  /* [n] */
    /* per-atom SAS neighbours: j != i with |c_i - c_j| < s_i + s_j */
    int *nstart;
    int *nbr;
    /* exposed three-sphere points */
    int nv;
    double *vp;   /* [nv][3] */
    int *vatom;   /* [nv][3], ascending atom ids */
    int *vsign;   /* +1 / -1 */
    double *veps; /* [nv] bound on the rounding error of each position (angstrom) */
    double cmag;  /* max |coordinate| of any centre */
    int *vcstart; /* vertex cell list */
    int *vcidx;
} oracle_t;

static double sq(double a) { return a * a; }

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

static int cell_coord(const oracle_t *o, double x, int a) {
    return clampi((int)floor((x - o->lo[a]) / o->cell), 0, o->nc[a] - 1);
}

/* Indices of atoms (or vertices) in the cells overlapping the cube
 * [x - d, x + d]; a superset of those within distance d. */
typedef struct {
    int *idx;
    int n, cap;
} ibuf_t;

static void ibuf_push(ibuf_t *b, int v) {
    if (b->n == b->cap) {
        b->cap = b->cap ? 2 * b->cap : 256;
        b->idx = (int *)realloc(b->idx, sizeof(int) * (size_t)b->cap);
    }
    b->idx[b->n++] = v;
}

static void query_cells(const oracle_t *o, const int *start, const int *list, const double x[3],
                        double d, ibuf_t *out) {
    int a0[3], a1[3];
    out->n = 0;
    for (int a = 0; a < 3; a++) {
        a0[a] = cell_coord(o, x[a] - d, a);
        a1[a] = cell_coord(o, x[a] + d, a);
    }
    for (int k = a0[2]; k <= a1[2]; k++)
        for (int j = a0[1]; j <= a1[1]; j++)
            for (int i = a0[0]; i <= a1[0]; i++) {
                int c = i + o->nc[0] * (j + o->nc[1] * k);
                for (int q = start[c]; q < start[c + 1]; q++) ibuf_push(out, list[q]);
            }
}

static void build_cells(const oracle_t *o, int count, const double *px, const double *py,
                        const double *pz, int **start_out, int **list_out) {
    int ncell = o->nc[0] * o->nc[1] * o->nc[2];
    int *start = (int *)calloc((size_t)ncell + 1, sizeof(int));
    int *list = (int *)malloc(sizeof(int) * (size_t)(count > 0 ? count : 1));
    int *cid = (int *)malloc(sizeof(int) * (size_t)(count > 0 ? count : 1));
    for (int q = 0; q < count; q++) {
        int c = cell_coord(o, px[q], 0) +
                o->nc[0] * (cell_coord(o, py[q], 1) + o->nc[1] * cell_coord(o, pz[q], 2));
        cid[q] = c;
        start[c + 1]++;
    }
    for (int c = 0; c < ncell; c++) start[c + 1] += start[c];
    int *fill = (int *)malloc(sizeof(int) * (size_t)ncell);
    memcpy(fill, start, sizeof(int) * (size_t)ncell);
    for (int q = 0; q < count; q++) list[fill[cid[q]]++] = q;
    free(fill);
    free(cid);
    *start_out = start;
    *list_out = list;
}

static double dist2_pt(const oracle_t *o, int i, const double x[3]) {
    return sq(x[0] - o->cx[i]) + sq(x[1] - o->cy[i]) + sq(x[2] - o->cz[i]);
}

/* y is in A (no atom other than skip0..2 has y strictly inside its SAS ball).
 * A point on S_i can only lie inside ball k if S_i and S_k overlap, so the
 * SAS neighbours of `owner` are a superset of the atoms to test. */
static int in_A(const oracle_t *o, const double y[3], int owner, int skip1, int skip2) {
    for (int q = o->nstart[owner]; q < o->nstart[owner + 1]; q++) {
        int k = o->nbr[q];
        if (k == skip1 || k == skip2) continue;
        if (dist2_pt(o, k, y) < sq(o->s[k])) return 0;
    }
    return 1;
}

/* Circle S_i ^ S_j: centre oc, unit axis n (c_i -> c_j), radius R.
 * Exists iff |s_i - s_j| < d < s_i + s_j. */
static int circle_of(const oracle_t *o, int i, int j, double oc[3], double n[3], double *R) {
    double v[3] = {o->cx[j] - o->cx[i], o->cy[j] - o->cy[i], o->cz[j] - o->cz[i]};
    double d = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    if (!(d < o->s[i] + o->s[j]) || !(d > fabs(o->s[i] - o->s[j]))) return 0;
    double a = (sq(o->s[i]) - sq(o->s[j]) + d * d) / (2.0 * d);
    double R2 = sq(o->s[i]) - a * a;
    if (!(R2 > 0.0)) return 0;
    for (int t = 0; t < 3; t++) n[t] = v[t] / d;
    oc[0] = o->cx[i] + a * n[0];
    oc[1] = o->cy[i] + a * n[1];
    oc[2] = o->cz[i] + a * n[2];
    *R = sqrt(R2);
    return 1;
}

/* Any unit vector perpendicular to n. */
static void perp_unit(const double n[3], double u[3]) {
    double e[3] = {0, 0, 0};
    int m = 0;
    if (fabs(n[1]) < fabs(n[m])) m = 1;
    if (fabs(n[2]) < fabs(n[m])) m = 2;
    e[m] = 1.0;
    double dn = e[0] * n[0] + e[1] * n[1] + e[2] * n[2];
    for (int t = 0; t < 3; t++) u[t] = e[t] - dn * n[t];
    double l = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    for (int t = 0; t < 3; t++) u[t] /= l;
}

/* Nearest point of circle (oc, n, R) to x; uses an arbitrary circle point
 * when x is on the axis (all circle points are then equally far). */
static void circle_nearest(const double x[3], const double oc[3], const double n[3], double R,
                           double q[3]) {
    double w[3] = {x[0] - oc[0], x[1] - oc[1], x[2] - oc[2]};
    double t = w[0] * n[0] + w[1] * n[1] + w[2] * n[2];
    double wp[3] = {w[0] - t * n[0], w[1] - t * n[1], w[2] - t * n[2]};
    double b = sqrt(wp[0] * wp[0] + wp[1] * wp[1] + wp[2] * wp[2]);
    double u[3];
    if (b > 0.0) {
        for (int k = 0; k < 3; k++) u[k] = wp[k] / b;
    } else {
        perp_unit(n, u);
    }
    for (int k = 0; k < 3; k++) q[k] = oc[k] + R * u[k];
}

static double norm3(const double a[3]) { return sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]); }

/* Which candidate attained the minimum (for normals and tags). */
typedef struct {
    int type; /* 1 face (convex), 2 circle (saddle), 3 vertex (concave), 0 none */
    int a[3];
    double y[3];
} owner_t;

/* min(cap, dist(x, A)) for x in U (0 if x is not in U), from the candidate
 * theorem above.  Candidates farther than the running minimum are skipped
 * before their membership test, which does not change the minimum. */
static double dist_to_A(const oracle_t *o, const double x[3], double cap, owner_t *own,
                        ibuf_t *buf) {
    double best = cap;
    if (own) own->type = 0;
    /* atoms whose sphere comes within cap of x (a candidate on S_i within cap
     * of x needs |x - c_i| < s_i + cap) */
    query_cells(o, o->cstart, o->catom, x, o->smax + cap, buf);
    int inU = 0, m = 0;
    for (int q = 0; q < buf->n; q++) {
        int i = buf->idx[q];
        double d2 = dist2_pt(o, i, x);
        if (d2 < sq(o->s[i])) inU = 1;
        if (d2 < sq(o->s[i] + cap)) buf->idx[m++] = i;
    }
    buf->n = m;
    if (!inU) return 0.0;
    /* (V) exposed three-sphere points */
    {
        ibuf_t vb = {0, 0, 0};
        query_cells(o, o->vcstart, o->vcidx, x, cap, &vb);
        for (int q = 0; q < vb.n; q++) {
            int v = vb.idx[q];
            const double *p = o->vp + 3 * v;
            double d[3] = {x[0] - p[0], x[1] - p[1], x[2] - p[2]};
            double dv = norm3(d);
            if (dv < best) {
                best = dv;
                if (own) {
                    own->type = 3;
                    for (int t = 0; t < 3; t++) {
                        own->a[t] = o->vatom[3 * v + t];
                        own->y[t] = p[t];
                    }
                }
            }
        }
        free(vb.idx);
    }
    /* (F) radial projections */
    for (int q = 0; q < buf->n; q++) {
        int i = buf->idx[q];
        double dv[3] = {x[0] - o->cx[i], x[1] - o->cy[i], x[2] - o->cz[i]};
        double d = norm3(dv);
        if (!(d > 0.0)) continue;
        double y[3];
        for (int t = 0; t < 3; t++) y[t] = (t == 0 ? o->cx[i] : t == 1 ? o->cy[i] : o->cz[i]) + o->s[i] * dv[t] / d;
        double e[3] = {x[0] - y[0], x[1] - y[1], x[2] - y[2]};
        double dy = norm3(e);
        if (dy < best && in_A(o, y, i, i, i)) {
            best = dy;
            if (own) {
                own->type = 1;
                own->a[0] = i;
                own->a[1] = own->a[2] = -1;
                memcpy(own->y, y, sizeof(y));
            }
        }
    }
    /* (E) nearest circle points */
    for (int q1 = 0; q1 < buf->n; q1++) {
        int i = buf->idx[q1];
        for (int qq = o->nstart[i]; qq < o->nstart[i + 1]; qq++) {
            int j = o->nbr[qq];
            if (j <= i) continue;
            if (!(dist2_pt(o, j, x) < sq(o->s[j] + cap))) continue;
            double oc[3], n[3], R;
            if (!circle_of(o, i, j, oc, n, &R)) continue;
            double qp[3];
            circle_nearest(x, oc, n, R, qp);
            double e[3] = {x[0] - qp[0], x[1] - qp[1], x[2] - qp[2]};
            double dq = norm3(e);
            if (dq < best && in_A(o, qp, i, i, j)) {
                best = dq;
                if (own) {
                    own->type = 2;
                    own->a[0] = i;
                    own->a[1] = j;
                    own->a[2] = -1;
                    memcpy(own->y, qp, sizeof(qp));
                }
            }
        }
    }
    return best;
}

/* Inside(x) = [dist(x, A) >= rho], eq. (2), via the three cases above. */
static int label_at(const oracle_t *o, const double x[3], ibuf_t *buf) {
    query_cells(o, o->cstart, o->catom, x, o->smax, buf);
    int inU = 0;
    for (int q = 0; q < buf->n; q++) {
        int i = buf->idx[q];
        double d2 = dist2_pt(o, i, x);
        if (d2 <= sq(o->r[i])) return 1;
        if (d2 < sq(o->s[i])) inU = 1;
    }
    if (!inU) return 0;
    return dist_to_A(o, x, o->rho, NULL, buf) >= o->rho;
}

/* ------------------------------------------------- certified labels */

/* Width of the undecided band of a comparison, relative to the squared length
 * scale of its terms: 2^-40, at least 2^12 times the few-ulp rounding error of
 * the sums of squares and products below (u = 2^-53). */
#define CERT_BAND 9.094947017729282e-13
#define U_RND 1.1102230246251565e-16

enum { T_NO = 0, T_YES = 1, T_UNSURE = 2 };

/* Three-valued "m < 0" (or "m <= 0": the two differ only at m = 0, which is
 * undecided either way) for a margin m computed with |error| <= err. */
static int tri_neg(double m, double err) {
    if (m < -err) return T_YES;
    if (m > err) return T_NO;
    return T_UNSURE;
}

static double absmax3(const double v[3]) {
    return fmax(fabs(v[0]), fmax(fabs(v[1]), fabs(v[2])));
}

/* Circle S_i ^ S_j as circle_of, with a bound eps on the rounding error of
 * each component of its centre and of its radius (first order, safety 4):
 * d within 4u d; a = (s_i^2 - s_j^2 + d^2) / 2d within
 * da = 2u (s_i^2 + s_j^2 + 3 d^2) / d + 5u |a|; R^2 = s_i^2 - a^2 within
 * 3u s_i^2 + 2 |a| da + u a^2, hence R within that over 2R plus u R; the unit
 * axis within 6u per component, so o = c_i + a n within
 * 2u (|c_i| + |a| + s_i) + da + 6u |a|. */
static int circle_cert(const oracle_t *o, int i, int j, double oc[3], double n[3], double *R,
                       double *eps) {
    if (!circle_of(o, i, j, oc, n, R)) return 0;
    const double u = U_RND;
    double v[3] = {o->cx[j] - o->cx[i], o->cy[j] - o->cy[i], o->cz[j] - o->cz[i]};
    double d = norm3(v);
    double si = o->s[i], sj = o->s[j];
    double a = (sq(si) - sq(sj) + d * d) / (2.0 * d);
    double ci[3] = {o->cx[i], o->cy[i], o->cz[i]};
    double da = 2.0 * u * (sq(si) + sq(sj) + 3.0 * d * d) / d + 5.0 * u * fabs(a);
    double dR = (3.0 * u * sq(si) + 2.0 * fabs(a) * da + u * a * a) / (2.0 * *R) + u * *R;
    *eps = 4.0 * (2.0 * u * (absmax3(ci) + fabs(a) + si) + da + 6.0 * u * fabs(a) + dR);
    return 1;
}

/* Certified case 3 for x in U and in no van der Waals ball (both certain):
 * 0 if some admissible candidate certainly lies closer than rho, 1 if
 * certainly none does, 2 if that depends on an undecided comparison. */
static int shell_cert(const oracle_t *o, const double x[3], ibuf_t *buf) {
    const double rho = o->rho, rho2 = rho * rho, u = U_RND;
    int unsure = 0;
    /* (V) concave probe positions: |x - p|^2 < rho^2.  p is within veps of
     * its exact value, so |x - p|^2 within 2 |x - p| veps (+ rounding);
     * 2 |x - p| <= |x - p|^2 / rho + rho. */
    {
        ibuf_t vb = {0, 0, 0};
        query_cells(o, o->vcstart, o->vcidx, x, rho + 1e-6, &vb);
        for (int q = 0; q < vb.n; q++) {
            int v = vb.idx[q];
            const double *p = o->vp + 3 * v;
            double d2 = sq(x[0] - p[0]) + sq(x[1] - p[1]) + sq(x[2] - p[2]);
            double err = 2.0 * o->veps[v] * (d2 / rho + rho) + CERT_BAND * (d2 + rho2);
            int t = tri_neg(d2 - rho2, err);
            if (t == T_YES) {
                free(vb.idx);
                return 0;
            }
            if (t == T_UNSURE) unsure = 1;
        }
        free(vb.idx);
    }
    query_cells(o, o->cstart, o->catom, x, o->smax + rho + 1e-6, buf);
    {
        int m = 0;
        for (int q = 0; q < buf->n; q++) {
            int i = buf->idx[q];
            if (dist2_pt(o, i, x) < sq(o->s[i] + rho + 1e-6)) buf->idx[m++] = i;
        }
        buf->n = m;
    }
    /* (F) radial projections y_i = c_i + s_i (x - c_i) / |x - c_i|, within rho
     * iff |x - c_i| < s_i + rho (x is outside the van der Waals ball); y_i is
     * within eps_y = 4u (2 |c_i| + 3 s_i) of its exact value, so |y - c_k|^2 is
     * within 2 |y - c_k| eps_y (+ rounding). */
    for (int q = 0; q < buf->n; q++) {
        int i = buf->idx[q];
        double ci[3] = {o->cx[i], o->cy[i], o->cz[i]};
        double d2 = dist2_pt(o, i, x);
        double sr = o->s[i] + rho;
        int w = tri_neg(d2 - sq(sr), CERT_BAND * (d2 + sq(sr)));
        if (w == T_NO) continue;
        double dv[3] = {x[0] - ci[0], x[1] - ci[1], x[2] - ci[2]};
        double d = sqrt(d2);
        double y[3];
        for (int t = 0; t < 3; t++) y[t] = ci[t] + o->s[i] * dv[t] / d;
        double eps_y = 4.0 * u * (2.0 * absmax3(ci) + 3.0 * o->s[i]);
        int adm = T_YES;
        for (int qq = o->nstart[i]; qq < o->nstart[i + 1] && adm != T_NO; qq++) {
            int k = o->nbr[qq];
            double dk2 = dist2_pt(o, k, y);
            double err = 4.0 * sqrt(dk2) * eps_y + CERT_BAND * (dk2 + sq(o->s[k]));
            int in = tri_neg(dk2 - sq(o->s[k]), err); /* y strictly inside ball k */
            if (in == T_YES) adm = T_NO;
            else if (in == T_UNSURE) adm = T_UNSURE;
        }
        if (adm == T_NO) continue;
        if (w == T_YES && adm == T_YES) return 0;
        unsure = 1;
    }
    /* (E) nearest circle points.  With w = x - o, t = w.n, b = |w - t n|:
     * |x - q|^2 = |w|^2 + R^2 - 2 b R, whose error is below
     * 8 (|w| + R)(eps + 8u |w|) (+ rounding); q = o + R (w - t n) / b is within
     * eps_q = 2 eps + 4 R (eps + 13u |w|) / b (the direction is undetermined on
     * the axis, b = 0).  A neighbour k whose ball certainly misses the whole
     * circle (distance from c_k to the circle above s_k) cannot make q
     * inadmissible; one that certainly holds the whole circle always does. */
    for (int q1 = 0; q1 < buf->n; q1++) {
        int i = buf->idx[q1];
        for (int qq = o->nstart[i]; qq < o->nstart[i + 1]; qq++) {
            int j = o->nbr[qq];
            if (j <= i) continue;
            if (!(dist2_pt(o, j, x) < sq(o->s[j] + rho + 1e-6))) continue;
            double oc[3], n[3], R, eps;
            if (!circle_cert(o, i, j, oc, n, &R, &eps)) continue;
            double w[3] = {x[0] - oc[0], x[1] - oc[1], x[2] - oc[2]};
            double ww = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
            double t = w[0] * n[0] + w[1] * n[1] + w[2] * n[2];
            double wp[3] = {w[0] - t * n[0], w[1] - t * n[1], w[2] - t * n[2]};
            double b = norm3(wp);
            double wl = sqrt(ww);
            double m = ww + R * R - rho2 - 2.0 * b * R;
            double err = 8.0 * (wl + R) * (eps + 8.0 * u * wl) +
                         CERT_BAND * (ww + R * R + rho2 + 2.0 * b * R);
            int within = tri_neg(m, err);
            if (within == T_NO) continue;
            double eps_q = b > 0.0 ? 2.0 * eps + 4.0 * R * (eps + 13.0 * u * wl) / b : INFINITY;
            double qp[3];
            circle_nearest(x, oc, n, R, qp);
            int adm = T_YES;
            for (int q3 = o->nstart[i]; q3 < o->nstart[i + 1] && adm != T_NO; q3++) {
                int k = o->nbr[q3];
                if (k == j) continue;
                double ck[3] = {o->cx[k], o->cy[k], o->cz[k]};
                double wk[3] = {ck[0] - oc[0], ck[1] - oc[1], ck[2] - oc[2]};
                double wkk = wk[0] * wk[0] + wk[1] * wk[1] + wk[2] * wk[2];
                double tk = wk[0] * n[0] + wk[1] * n[1] + wk[2] * n[2];
                double bk = sqrt(fmax(0.0, wkk - tk * tk));
                double sk2 = sq(o->s[k]);
                double wkl = sqrt(wkk);
                double errk = 8.0 * (wkl + R) * (eps + 8.0 * u * wkl) +
                              CERT_BAND * (wkk + R * R + sk2 + 2.0 * bk * R);
                /* nearest and farthest circle points from c_k */
                int miss = tri_neg(sk2 - (tk * tk + sq(bk - R)), errk);
                if (miss == T_YES) continue;
                int hold = tri_neg(tk * tk + sq(bk + R) - sk2, errk);
                if (hold == T_YES) {
                    adm = T_NO;
                    break;
                }
                double dk2 = sq(qp[0] - ck[0]) + sq(qp[1] - ck[1]) + sq(qp[2] - ck[2]);
                double e2 = isinf(eps_q) ? INFINITY
                                         : 4.0 * sqrt(dk2) * eps_q + CERT_BAND * (dk2 + sk2);
                int in = tri_neg(dk2 - sk2, e2);
                if (in == T_YES) adm = T_NO;
                else if (in == T_UNSURE) adm = T_UNSURE;
            }
            if (adm == T_NO) continue;
            if (within == T_YES && adm == T_YES) return 0;
            unsure = 1;
        }
    }
    return unsure ? 2 : 1;
}

/* Certified label: 1 inside, 0 outside, 2 undecided in FP64 (the cases of
 * label_at, each comparison three-valued; |x - c|^2, r^2 and s^2 are each
 * within 4u of their exact values, relative). */
static int label_cert(const oracle_t *o, const double x[3], ibuf_t *buf) {
    query_cells(o, o->cstart, o->catom, x, o->smax + 1e-6, buf);
    int vdw_unsure = 0, inU = 0, inU_unsure = 0;
    for (int q = 0; q < buf->n; q++) {
        int i = buf->idx[q];
        double d2 = dist2_pt(o, i, x);
        double s2 = sq(o->s[i]);
        double err = CERT_BAND * (d2 + s2);
        int v = tri_neg(d2 - sq(o->r[i]), err);
        if (v == T_YES) return 1;
        if (v == T_UNSURE) vdw_unsure = 1;
        int us = tri_neg(d2 - s2, err);
        if (us == T_YES) inU = 1;
        else if (us == T_UNSURE) inU_unsure = 1;
    }
    if (vdw_unsure) return 2;
    if (!inU) return inU_unsure ? 2 : 0;
    return shell_cert(o, x, buf);
}

/* ---------------------------------------------------------------- setup */

/* Relative tolerance of the admissibility test of a three-sphere point
 * (section 1: a probe touching three or more atoms).  A probe that touches a
 * fourth atom exactly sits at distance s_l from it in exact arithmetic, but the
 * rounded point may land a few ulps inside that SAS ball; the test keeps points
 * with |p - c_l|^2 >= s_l^2 (1 - VERTEX_TOL), so that every triple of a
 * cospherical set reports the probe. */
#define VERTEX_TOL 1e-9

/* Points on three SAS spheres by trilateration in the frame e_x || c_j - c_i,
 * e_y towards c_k, e_z = e_x x e_y.  Returns 0 if the centres are collinear or
 * the spheres share no point (z^2 < 0). */
static int trilaterate(const oracle_t *o, int i, int j, int k, double pp[3], double pm[3],
                       double *eps) {
    double ci[3] = {o->cx[i], o->cy[i], o->cz[i]};
    double dj[3] = {o->cx[j] - ci[0], o->cy[j] - ci[1], o->cz[j] - ci[2]};
    double dk[3] = {o->cx[k] - ci[0], o->cy[k] - ci[1], o->cz[k] - ci[2]};
    double d = norm3(dj);
    double ex[3] = {dj[0] / d, dj[1] / d, dj[2] / d};
    double ii = ex[0] * dk[0] + ex[1] * dk[1] + ex[2] * dk[2];
    double ey[3] = {dk[0] - ii * ex[0], dk[1] - ii * ex[1], dk[2] - ii * ex[2]};
    double jj = norm3(ey);
    if (!(jj > 1e-12 * d)) return 0;
    for (int t = 0; t < 3; t++) ey[t] /= jj;
    double ez[3] = {ex[1] * ey[2] - ex[2] * ey[1], ex[2] * ey[0] - ex[0] * ey[2],
                    ex[0] * ey[1] - ex[1] * ey[0]};
    double si2 = sq(o->s[i]), sj2 = sq(o->s[j]), sk2 = sq(o->s[k]);
    double X = (si2 - sj2 + d * d) / (2.0 * d);
    double Y = (si2 - sk2 + ii * ii + jj * jj) / (2.0 * jj) - (ii / jj) * X;
    double Z2 = si2 - X * X - Y * Y;
    if (Z2 < 0.0) return 0;
    double Z = sqrt(Z2);
    for (int t = 0; t < 3; t++) {
        pp[t] = ci[t] + X * ex[t] + Y * ey[t] + Z * ez[t];
        pm[t] = ci[t] + X * ex[t] + Y * ey[t] - Z * ez[t];
    }
    /* Rounding-error bound of the positions (first order, with a safety factor
     * of at least 4).  With L the sum of the lengths that enter (radii, d, |dk|)
     * and q = 1 + L / jj the amplification by a nearly collinear triple: the
     * frame vectors are off by <= 8u q, X by <= 4u L^2 / d, Y by <= 8u L^2 q^2 / jj
     * -- hence |X ex + Y ey| by <= 16u L q^2 (L / jj + L / d) -- and Z by the
     * error of Z^2 (<= 8u L^2 q^2 (1 + L / d)) over 2 Z, or by its square root
     * where that is smaller; the centre adds u |c_i|. */
    {
        const double u = 1.1102230246251565e-16;
        const double L = o->s[i] + o->s[j] + o->s[k] + d + norm3(dk);
        const double q = 1.0 + L / jj;
        const double cm = fmax(fabs(ci[0]), fmax(fabs(ci[1]), fabs(ci[2])));
        const double ez2 = 8.0 * u * L * L * q * q * (1.0 + L / d);
        /* |sqrt(a) - sqrt(b)| <= min(sqrt(|a - b|), |a - b| / (2 sqrt(b))) */
        *eps = 16.0 * (u * cm + 16.0 * u * L * q * q * (1.0 + L / jj + L / d) +
                       (Z > 0.0 ? fmin(sqrt(ez2), ez2 / (2.0 * Z)) : sqrt(ez2)));
    }
    return 1;
}

void orc_destroy(void *h) {
    oracle_t *o = (oracle_t *)h;
    if (!o) return;
    free(o->cx); free(o->cy); free(o->cz); free(o->r); free(o->s);
    free(o->cstart); free(o->catom); free(o->nstart); free(o->nbr);
    free(o->vp); free(o->vatom); free(o->vsign); free(o->veps); free(o->vcstart); free(o->vcidx);
    free(o);
}

void *orc_create(int n, const double *centres, const double *radii, double rho) {
    if (n < 1 || !(rho > 0.0)) return NULL;
    oracle_t *o = (oracle_t *)calloc(1, sizeof(oracle_t));
    o->n = n;
    o->rho = rho;
    o->cx = (double *)malloc(sizeof(double) * (size_t)n);
    o->cy = (double *)malloc(sizeof(double) * (size_t)n);
    o->cz = (double *)malloc(sizeof(double) * (size_t)n);
    o->r = (double *)malloc(sizeof(double) * (size_t)n);
    o->s = (double *)malloc(sizeof(double) * (size_t)n);
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    o->smax = 0.0;
    for (int i = 0; i < n; i++) {
        o->cx[i] = centres[3 * i];
        o->cy[i] = centres[3 * i + 1];
        o->cz[i] = centres[3 * i + 2];
        o->r[i] = radii[i];
        o->s[i] = radii[i] + rho;
        if (o->s[i] > o->smax) o->smax = o->s[i];
        for (int a = 0; a < 3; a++) o->cmag = fmax(o->cmag, fabs(centres[3 * i + a]));
        for (int a = 0; a < 3; a++) {
            if (centres[3 * i + a] < lo[a]) lo[a] = centres[3 * i + a];
            if (centres[3 * i + a] > hi[a]) hi[a] = centres[3 * i + a];
        }
    }
    o->cell = o->smax + rho;
    for (int a = 0; a < 3; a++) {
        o->lo[a] = lo[a];
        o->nc[a] = (int)floor((hi[a] - lo[a]) / o->cell) + 1;
    }
    build_cells(o, n, o->cx, o->cy, o->cz, &o->cstart, &o->catom);

    /* SAS neighbours */
    o->nstart = (int *)calloc((size_t)n + 1, sizeof(int));
    ibuf_t buf = {0, 0, 0};
    ibuf_t all = {0, 0, 0};
    for (int i = 0; i < n; i++) {
        double x[3] = {o->cx[i], o->cy[i], o->cz[i]};
        query_cells(o, o->cstart, o->catom, x, 2.0 * o->smax, &buf);
        for (int q = 0; q < buf.n; q++) {
            int j = buf.idx[q];
            if (j != i && dist2_pt(o, j, x) == 0.0) {
                /* two atoms share a centre: rejected (atoms are distinct balls) */
                free(buf.idx);
                free(all.idx);
                orc_destroy(o);
                return NULL;
            }
            if (j != i && dist2_pt(o, j, x) < sq(o->s[i] + o->s[j])) ibuf_push(&all, j);
        }
        o->nstart[i + 1] = all.n;
    }
    o->nbr = all.idx ? all.idx : (int *)malloc(sizeof(int));

    /* exposed three-sphere points, triples i < j < k with pairwise overlap */
    ibuf_t vat = {0, 0, 0}, vsg = {0, 0, 0};
    double *vp = NULL, *ve = NULL;
    int nv = 0, vcap = 0;
    for (int i = 0; i < n; i++) {
        for (int q1 = o->nstart[i]; q1 < o->nstart[i + 1]; q1++) {
            int j = o->nbr[q1];
            if (j <= i) continue;
            for (int q2 = o->nstart[i]; q2 < o->nstart[i + 1]; q2++) {
                int k = o->nbr[q2];
                if (k <= j) continue;
                double cj[3] = {o->cx[j], o->cy[j], o->cz[j]};
                if (!(dist2_pt(o, k, cj) < sq(o->s[j] + o->s[k]))) continue;
                double pp[3], pm[3], peps;
                if (!trilaterate(o, i, j, k, pp, pm, &peps)) continue;
                for (int sgn = 0; sgn < 2; sgn++) {
                    double *p = sgn == 0 ? pp : pm;
                    /* in A: every atom other than i, j, k at least its SAS radius away,
                     * up to VERTEX_TOL (a probe touching four or more atoms stays
                     * admissible whatever the rounding of p) */
                    int ok = 1;
                    for (int q3 = o->nstart[i]; q3 < o->nstart[i + 1] && ok; q3++) {
                        int l = o->nbr[q3];
                        if (l == j || l == k) continue;
                        if (dist2_pt(o, l, p) < sq(o->s[l]) * (1.0 - VERTEX_TOL)) ok = 0;
                    }
                    if (!ok) continue;
                    if (nv == vcap) {
                        vcap = vcap ? 2 * vcap : 1024;
                        vp = (double *)realloc(vp, sizeof(double) * 3 * (size_t)vcap);
                        ve = (double *)realloc(ve, sizeof(double) * (size_t)vcap);
                    }
                    memcpy(vp + 3 * nv, p, 3 * sizeof(double));
                    ve[nv] = peps;
                    ibuf_push(&vat, i);
                    ibuf_push(&vat, j);
                    ibuf_push(&vat, k);
                    ibuf_push(&vsg, sgn == 0 ? 1 : -1);
                    nv++;
                }
            }
        }
    }
    o->nv = nv;
    o->vp = vp ? vp : (double *)malloc(sizeof(double) * 3);
    o->veps = ve ? ve : (double *)malloc(sizeof(double));
    o->vatom = vat.idx ? vat.idx : (int *)malloc(sizeof(int) * 3);
    o->vsign = vsg.idx ? vsg.idx : (int *)malloc(sizeof(int));
    {
        double *px = (double *)malloc(sizeof(double) * (size_t)(nv > 0 ? nv : 1));
        double *py = (double *)malloc(sizeof(double) * (size_t)(nv > 0 ? nv : 1));
        double *pz = (double *)malloc(sizeof(double) * (size_t)(nv > 0 ? nv : 1));
        for (int v = 0; v < nv; v++) {
            px[v] = o->vp[3 * v];
            py[v] = o->vp[3 * v + 1];
            pz[v] = o->vp[3 * v + 2];
        }
        build_cells(o, nv, px, py, pz, &o->vcstart, &o->vcidx);
        free(px); free(py); free(pz);
    }
    free(buf.idx);
    return o;
}

int orc_num_vertices(void *h) { return ((oracle_t *)h)->nv; }

void orc_get_vertices(void *h, double *p, int *atoms, int *sign) {
    oracle_t *o = (oracle_t *)h;
    memcpy(p, o->vp, sizeof(double) * 3 * (size_t)o->nv);
    memcpy(atoms, o->vatom, sizeof(int) * 3 * (size_t)o->nv);
    memcpy(sign, o->vsign, sizeof(int) * (size_t)o->nv);
}

int orc_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------- labels */

static double grid_coord(double lo, double h, long i) {
    volatile double ih = (double)i * h; /* fl(i h), then fl(lo + fl(i h)) */
    return lo + ih;
}

void orc_labels_points(void *h, long count, const double *x, uint8_t *out) {
    oracle_t *o = (oracle_t *)h;
#pragma omp parallel
    {
        ibuf_t buf = {0, 0, 0};
#pragma omp for schedule(dynamic, 64)
        for (long q = 0; q < count; q++) out[q] = (uint8_t)label_at(o, x + 3 * q, &buf);
        free(buf.idx);
    }
}

/* Labels of grid points with k in [k0, k1); out[(k-k0)*ny*nx + j*nx + i]. */
void orc_labels_grid(void *h, const double lo[3], double hs, const int dims[3], int k0, int k1,
                     uint8_t *out) {
    oracle_t *o = (oracle_t *)h;
    long nx = dims[0], ny = dims[1];
    long rows = (long)(k1 - k0) * ny;
#pragma omp parallel
    {
        ibuf_t buf = {0, 0, 0};
#pragma omp for schedule(dynamic, 1)
        for (long row = 0; row < rows; row++) {
            long k = k0 + row / ny, j = row % ny;
            double x[3];
            x[1] = grid_coord(lo[1], hs, j);
            x[2] = grid_coord(lo[2], hs, k);
            for (long i = 0; i < nx; i++) {
                x[0] = grid_coord(lo[0], hs, i);
                out[row * nx + i] = (uint8_t)label_at(o, x, &buf);
            }
        }
        free(buf.idx);
    }
}

/* Certified labels (1, 0, or 2 = undecided in FP64) of points, and of the grid
 * points with k in [k0, k1) as orc_labels_grid. */
void orc_labels_points_cert(void *h, long count, const double *x, uint8_t *out) {
    oracle_t *o = (oracle_t *)h;
#pragma omp parallel
    {
        ibuf_t buf = {0, 0, 0};
#pragma omp for schedule(dynamic, 64)
        for (long q = 0; q < count; q++) out[q] = (uint8_t)label_cert(o, x + 3 * q, &buf);
        free(buf.idx);
    }
}

void orc_labels_grid_cert(void *h, const double lo[3], double hs, const int dims[3], int k0,
                          int k1, uint8_t *out) {
    oracle_t *o = (oracle_t *)h;
    long nx = dims[0], ny = dims[1];
    long rows = (long)(k1 - k0) * ny;
#pragma omp parallel
    {
        ibuf_t buf = {0, 0, 0};
#pragma omp for schedule(dynamic, 1)
        for (long row = 0; row < rows; row++) {
            long k = k0 + row / ny, j = row % ny;
            double x[3];
            x[1] = grid_coord(lo[1], hs, j);
            x[2] = grid_coord(lo[2], hs, k);
            for (long i = 0; i < nx; i++) {
                x[0] = grid_coord(lo[0], hs, i);
                out[row * nx + i] = (uint8_t)label_cert(o, x, &buf);
            }
        }
        free(buf.idx);
    }
}

/* min(cap, dist(x, A)) for each point (0 outside U), with the owner type. */
void orc_dist_points(void *h, long count, const double *x, double cap, double *out, int *type) {
    oracle_t *o = (oracle_t *)h;
#pragma omp parallel
    {
        ibuf_t buf = {0, 0, 0};
#pragma omp for schedule(dynamic, 64)
        for (long q = 0; q < count; q++) {
            owner_t own;
            out[q] = dist_to_A(o, x + 3 * q, cap, &own, &buf);
            if (type) type[q] = own.type;
        }
        free(buf.idx);
    }
}

/* -------------------------------------------------------------- edges */

/* Real roots in [0, 1] of a polynomial of degree n <= 4 (coefficients c[0..n],
 * ascending), isolated by subdividing its Bernstein form on [0, 1] (the
 * number of sign changes of the Bernstein coefficients bounds the number of
 * roots) and refined by bisection.  Long double throughout. */
typedef long double ld;

static ld horner(const ld *c, int n, ld u) {
    ld v = c[n];
    for (int q = n - 1; q >= 0; q--) v = v * u + c[q];
    return v;
}

static int sign_changes(const ld *b, int n) {
    int v = 0, last = 0;
    for (int q = 0; q <= n; q++) {
        int sg = b[q] > 0 ? 1 : (b[q] < 0 ? -1 : 0);
        if (sg == 0) continue;
        if (last != 0 && sg != last) v++;
        last = sg;
    }
    return v;
}

static void add_root(double *roots, int *nr, int cap, ld u) {
    if (*nr < cap) roots[(*nr)++] = (double)u;
}

static void isolate(const ld *c, int n, const ld *b, ld a, ld w, int depth, double *roots,
                    int *nr, int cap) {
    int v = sign_changes(b, n);
    if (v == 0) return;
    if (v == 1 && b[0] != 0 && b[n] != 0) {
        ld x0 = a, x1 = a + w;
        ld f0 = horner(c, n, x0);
        for (int it = 0; it < 200 && x1 - x0 > 0; it++) {
            ld m = 0.5L * (x0 + x1);
            if (m <= x0 || m >= x1) break;
            ld fm = horner(c, n, m);
            if (fm == 0) {
                x0 = x1 = m;
                break;
            }
            if ((fm < 0) == (f0 < 0)) {
                x0 = m;
                f0 = fm;
            } else {
                x1 = m;
            }
        }
        add_root(roots, nr, cap, 0.5L * (x0 + x1));
        return;
    }
    if (depth > 60 || w < 1e-17L) {
        /* a cluster narrower than the resolution: one (multiple) root */
        add_root(roots, nr, cap, a + 0.5L * w);
        return;
    }
    /* de Casteljau split at the midpoint */
    ld t[5][5];
    for (int q = 0; q <= n; q++) t[0][q] = b[q];
    for (int r = 1; r <= n; r++)
        for (int q = 0; q <= n - r; q++) t[r][q] = 0.5L * (t[r - 1][q] + t[r - 1][q + 1]);
    ld L[5], Rb[5];
    for (int q = 0; q <= n; q++) {
        L[q] = t[q][0];
        Rb[q] = t[n - q][q];
    }
    ld mid = a + 0.5L * w;
    ld fmid = horner(c, n, mid);
    if (fmid == 0) add_root(roots, nr, cap, mid);
    L[n] = fmid;
    Rb[0] = fmid;
    isolate(c, n, L, a, 0.5L * w, depth + 1, roots, nr, cap);
    isolate(c, n, Rb, mid, 0.5L * w, depth + 1, roots, nr, cap);
}

static int poly_roots01(const ld *c, int n, double *roots, int cap) {
    static const ld binom[5][5] = {{1, 0, 0, 0, 0}, {1, 1, 0, 0, 0}, {1, 2, 1, 0, 0},
                                   {1, 3, 3, 1, 0}, {1, 4, 6, 4, 1}};
    ld b[5];
    for (int k = 0; k <= n; k++) {
        b[k] = 0;
        for (int i = 0; i <= k; i++) b[k] += binom[k][i] / binom[n][i] * c[i];
    }
    int nr = 0;
    if (c[0] == 0) add_root(roots, &nr, cap, 0.0L);
    ld f1 = horner(c, n, 1.0L);
    if (f1 == 0) add_root(roots, &nr, cap, 1.0L);
    b[0] = c[0];
    b[n] = f1;
    isolate(c, n, b, 0.0L, 1.0L, 0, roots, &nr, cap);
    return nr;
}

/* Roots in [0, 1] of the quartic g: its sign changes, plus every critical
 * point (root of g') where g vanishes to within rounding -- a root of even
 * multiplicity, which is where a line runs through the self-intersection of
 * a spindle torus on its axis (the torus quartic is then a perfect square). */
static int quartic_roots01(const ld c[5], double *roots, int cap) {
    int nr = poly_roots01(c, 4, roots, cap);
    ld d[4] = {c[1], 2 * c[2], 3 * c[3], 4 * c[4]};
    double cp[4];
    int nc = poly_roots01(d, 3, cp, 4);
    ld scale = fabsl(c[0]) + fabsl(c[1]) + fabsl(c[2]) + fabsl(c[3]) + fabsl(c[4]);
    for (int q = 0; q < nc; q++)
        if (fabsl(horner(c, 4, (ld)cp[q])) <= 1e-15L * scale) add_root(roots, &nr, cap, cp[q]);
    /* an end where g vanishes to within rounding: the segment starts or ends on
     * the torus */
    ld g0 = c[0], g1 = horner(c, 4, 1.0L);
    if (g0 != 0 && fabsl(g0) <= 1e-15L * scale) add_root(roots, &nr, cap, 0.0L);
    if (g1 != 0 && fabsl(g1) <= 1e-15L * scale) add_root(roots, &nr, cap, 1.0L);
    return nr;
}

/* A root within END_SLACK (of the edge's length) outside an end is taken as
 * a root at that end: a surface through an end point then owns a crossing
 * there even where rounding puts its computed root just outside the edge. */
#define END_SLACK 1e-9

/* Real roots in [0,1] of a u^2 + b u + c (stable quadratic formula). */
static int quad_roots01(double a, double b, double c, double *roots) {
    double disc = b * b - 4.0 * a * c;
    if (disc < 0.0) return 0;
    double sd = sqrt(disc);
    double qv = -0.5 * (b + (b >= 0 ? sd : -sd));
    int nr = 0;
    double r1 = qv / a;
    double r2 = qv != 0.0 ? c / qv : r1;
    int in1 = r1 >= -END_SLACK && r1 <= 1.0 + END_SLACK;
    int in2 = r2 >= -END_SLACK && r2 <= 1.0 + END_SLACK;
    r1 = fmin(1.0, fmax(0.0, r1));
    r2 = fmin(1.0, fmax(0.0, r2));
    if (in1) roots[nr++] = r1;
    if (in2 && !(in1 && r2 == r1)) roots[nr++] = r2;
    return nr;
}

typedef struct {
    double u;
    int type; /* 1 vdW sphere, 2 torus, 3 probe sphere */
    int a[3];
    int v;    /* vertex index for type 3 */
} root_t;

static int root_cmp(const void *pa, const void *pb) {
    const root_t *x = (const root_t *)pa, *y = (const root_t *)pb;
    if (x->u != y->u) return x->u < y->u ? -1 : 1;
    if (x->type != y->type) return x->type - y->type;
    for (int t = 0; t < 3; t++)
        if (x->a[t] != y->a[t]) return x->a[t] - y->a[t];
    return 0;
}

static void push_root(root_t **rs, int *nr, int *cap, double u, int type, int a0, int a1, int a2,
                      int v) {
    if (*nr == *cap) {
        *cap = *cap ? 2 * *cap : 64;
        *rs = (root_t *)realloc(*rs, sizeof(root_t) * (size_t)*cap);
    }
    root_t *r = *rs + (*nr)++;
    r->u = u;
    r->type = type;
    r->a[0] = a0;
    r->a[1] = a1;
    r->a[2] = a2;
    r->v = v;
}

/* One edge: key = 3 * (i + nx (j + ny k)) + axis, t = s + e_axis.
 * Returns 1 with the record if the endpoint labels differ, 0 otherwise,
 * -1 if the key is not an edge of the grid. */
static int edge_record(const oracle_t *o, const double lo[3], double hs, const int dims[3],
                       long key, const int *ends, double *lambda, double nrm[3], int *type,
                       int atoms[3], ibuf_t *buf) {
    long axis = key % 3, idx = key / 3;
    long nx = dims[0], ny = dims[1], nz = dims[2];
    if (key < 0 || idx >= nx * ny * nz) return -1;
    long ii[3] = {idx % nx, (idx / nx) % ny, idx / (nx * ny)};
    if (ii[axis] + 1 >= dims[axis]) return -1;
    (void)nz;
    double xs[3], xt[3];
    for (int a = 0; a < 3; a++) {
        xs[a] = grid_coord(lo[a], hs, ii[a]);
        xt[a] = grid_coord(lo[a], hs, ii[a] + (a == axis ? 1 : 0));
    }
    /* end labels: the caller's (exact) ones when given, else FP64 */
    int Ls = ends ? ends[0] : label_at(o, xs, buf), Lt = ends ? ends[1] : label_at(o, xt, buf);
    if (Ls == Lt) return 0;

    /* surfaces that can carry the boundary of M on the segment:
     * van der Waals spheres, tori of radius rho around every circle, and
     * probe spheres of radius rho around the exposed three-sphere points */
    root_t *rs = NULL;
    int nr = 0, rcap = 0;
    double mid[3];
    for (int a = 0; a < 3; a++) mid[a] = 0.5 * (xs[a] + xt[a]);
    double reach = 0.5 * hs + 1e-9;
    query_cells(o, o->cstart, o->catom, mid, o->smax + o->rho + reach, buf);
    {
        int m = 0;
        for (int q = 0; q < buf->n; q++) {
            int i = buf->idx[q];
            if (dist2_pt(o, i, mid) < sq(o->s[i] + o->rho + reach)) buf->idx[m++] = i;
        }
        buf->n = m;
    }
    double tmp[4];
    for (int q = 0; q < buf->n; q++) {
        int i = buf->idx[q];
        double c[3] = {o->cx[i], o->cy[i], o->cz[i]};
        double w0[3] = {xs[0] - c[0], xs[1] - c[1], xs[2] - c[2]};
        int nq = quad_roots01(hs * hs, 2.0 * hs * w0[axis],
                              w0[0] * w0[0] + w0[1] * w0[1] + w0[2] * w0[2] - sq(o->r[i]), tmp);
        for (int t = 0; t < nq; t++) push_root(&rs, &nr, &rcap, tmp[t], 1, i, -1, -1, -1);
    }
    for (int q1 = 0; q1 < buf->n; q1++) {
        int i = buf->idx[q1];
        for (int qq = o->nstart[i]; qq < o->nstart[i + 1]; qq++) {
            int j = o->nbr[qq];
            if (j <= i) continue;
            if (!(dist2_pt(o, j, mid) < sq(o->s[j] + o->rho + reach))) continue;
            double oc[3], n[3], R;
            if (!circle_of(o, i, j, oc, n, &R)) continue;
            double dm[3] = {mid[0] - oc[0], mid[1] - oc[1], mid[2] - oc[2]};
            if (norm3(dm) > R + o->rho + reach) continue;
            /* (|w|^2 + R^2 - rho^2)^2 - 4 R^2 (|w|^2 - (w.n)^2) along w = w0 + u h e */
            ld w0[3] = {(ld)xs[0] - oc[0], (ld)xs[1] - oc[1], (ld)xs[2] - oc[2]};
            ld H = hs, RR = (ld)R * R, rr = (ld)o->rho * o->rho;
            ld ww = w0[0] * w0[0] + w0[1] * w0[1] + w0[2] * w0[2];
            ld t0 = w0[0] * n[0] + w0[1] * n[1] + w0[2] * n[2];
            ld a0 = ww + RR - rr, a1 = 2 * H * w0[axis], a2 = H * H;
            ld b0 = ww - t0 * t0, b1 = 2 * H * w0[axis] - 2 * t0 * H * n[axis],
               b2 = H * H - H * H * (ld)n[axis] * n[axis];
            ld cf[5] = {a0 * a0 - 4 * RR * b0, 2 * a0 * a1 - 4 * RR * b1,
                        a1 * a1 + 2 * a0 * a2 - 4 * RR * b2, 2 * a1 * a2, a2 * a2};
            double qr[12];
            int nq = quartic_roots01(cf, qr, 12);
            for (int t = 0; t < nq; t++) {
                /* keep the branch at distance rho from the near circle point */
                double x[3];
                for (int a = 0; a < 3; a++) x[a] = xs[a];
                x[axis] += qr[t] * hs;
                double w[3] = {x[0] - oc[0], x[1] - oc[1], x[2] - oc[2]};
                double tt = w[0] * n[0] + w[1] * n[1] + w[2] * n[2];
                double bb = sqrt(fmax(0.0, w[0] * w[0] + w[1] * w[1] + w[2] * w[2] - tt * tt));
                double near = fabs(sq(bb - R) + tt * tt - sq(o->rho));
                double far = fabs(sq(bb + R) + tt * tt - sq(o->rho));
                if (near <= far) push_root(&rs, &nr, &rcap, qr[t], 2, i, j, -1, -1);
            }
        }
    }
    {
        ibuf_t vb = {0, 0, 0};
        query_cells(o, o->vcstart, o->vcidx, mid, o->rho + reach, &vb);
        for (int q = 0; q < vb.n; q++) {
            int v = vb.idx[q];
            const double *p = o->vp + 3 * v;
            double w0[3] = {xs[0] - p[0], xs[1] - p[1], xs[2] - p[2]};
            int nq = quad_roots01(hs * hs, 2.0 * hs * w0[axis],
                                  w0[0] * w0[0] + w0[1] * w0[1] + w0[2] * w0[2] - sq(o->rho), tmp);
            for (int t = 0; t < nq; t++)
                push_root(&rs, &nr, &rcap, tmp[t], 3, o->vatom[3 * v], o->vatom[3 * v + 1],
                          o->vatom[3 * v + 2], v);
        }
        free(vb.idx);
    }
    if (nr > 1) qsort(rs, (size_t)nr, sizeof(root_t), root_cmp);

    /* walk the intervals between breakpoints from s; the first interval whose
     * label differs from Inside[s] starts at u* */
    double ustar = 1.0;
    int found = 0;
    double prev = 0.0;
    for (int m = 0; m <= nr && !found; m++) {
        double next = m < nr ? rs[m].u : 1.0;
        if (next > prev) {
            double um = 0.5 * (prev + next);
            double x[3] = {xs[0], xs[1], xs[2]};
            x[axis] = xs[axis] + um * hs;
            if (label_at(o, x, buf) != Ls) {
                ustar = prev;
                found = 1;
            }
        }
        prev = next > prev ? next : prev;
    }
    if (!found) ustar = 1.0; /* the change happens at t itself */
    /* owner: the breakpoint at u* (closest root; ties by type then atoms) */
    int best = -1;
    double bd = INFINITY;
    for (int m = 0; m < nr; m++) {
        double dd = fabs(rs[m].u - ustar);
        if (dd < bd) {
            bd = dd;
            best = m;
        }
    }
    *lambda = 1.0 - ustar;
    double x[3] = {xs[0], xs[1], xs[2]};
    x[axis] = xs[axis] + ustar * hs;
    if (best < 0) {
        *type = 0;
        atoms[0] = atoms[1] = atoms[2] = -1;
        nrm[0] = nrm[1] = nrm[2] = 0.0;
    } else {
        root_t *r = rs + best;
        *type = r->type;
        double y[3];
        if (r->type == 1) {
            double c[3] = {o->cx[r->a[0]], o->cy[r->a[0]], o->cz[r->a[0]]};
            for (int a = 0; a < 3; a++) y[a] = x[a] - c[a]; /* outward: away from the atom */
        } else if (r->type == 2) {
            double oc[3], n[3], R, qp[3];
            circle_of(o, r->a[0], r->a[1], oc, n, &R);
            circle_nearest(x, oc, n, R, qp);
            for (int a = 0; a < 3; a++) y[a] = qp[a] - x[a]; /* towards the probe centre */
        } else {
            const double *p = o->vp + 3 * r->v;
            for (int a = 0; a < 3; a++) y[a] = p[a] - x[a];
        }
        double l = norm3(y);
        for (int a = 0; a < 3; a++) nrm[a] = l > 0 ? y[a] / l : 0.0;
        for (int a = 0; a < 3; a++) atoms[a] = r->a[a];
    }
    free(rs);
    return 1;
}

/* Records for a list of edge keys.  status[q]: 1 crossing, 0 same labels,
 * -1 not an edge.  Atom ids are the caller's atom indices.  ends (NULL or
 * [count][2]): the labels of each edge's two end points, as certified and
 * exactly re-decided by the caller; without them the ends are labelled in
 * FP64. */
void orc_edges(void *h, const double lo[3], double hs, const int dims[3], long count,
               const long *keys, const int *ends, int *status, double *lambda, double *normal,
               int *type, int *atoms) {
    oracle_t *o = (oracle_t *)h;
#pragma omp parallel
    {
        ibuf_t buf = {0, 0, 0};
#pragma omp for schedule(dynamic, 16)
        for (long q = 0; q < count; q++) {
            status[q] = edge_record(o, lo, hs, dims, keys[q], ends ? ends + 2 * q : NULL,
                                    lambda + q, normal + 3 * q, type + q, atoms + 3 * q, &buf);
        }
        free(buf.idx);
    }
}
