/*
 * globule.c -- seeded protein-like globules (input generation only).
 *
 * Recipe: a bonded random walk of 1.5 A steps inside a confinement ball of
 * radius (3N / (4 pi density))^(1/3) around the origin, starting at the
 * origin.  Each step draws up to 64 directions uniformly on the sphere and
 * takes the first that stays in the ball and keeps `min_sep` from every
 * placed atom other than its bonded predecessor.  If all 64 fail the walk
 * restarts from a uniformly drawn placed atom; after 200 consecutive failed
 * restarts the ball grows by 2 %.  Radii are drawn i.i.d. afterwards from a
 * table of values and probabilities.
 *
 * Random numbers: splitmix64 (Steele, Lea, Flood 2014) seeded with the
 * caller's seed; uniform doubles from the top 53 bits; directions by
 * Archimedes' theorem (z uniform in [-1, 1], azimuth uniform).
 */
#include <math.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    uint64_t s;
} rng_t;

static uint64_t splitmix64(rng_t *r) {
    uint64_t z = (r->s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static double uniform(rng_t *r) { return (double)(splitmix64(r) >> 11) * (1.0 / 9007199254740992.0); }

typedef struct {
    double cell;
    int side, half;
    int *head; /* side^3 cells, -1 = empty */
    int *next; /* per atom */
} grid_t;

static int grid_index(const grid_t *g, const double p[3], int c[3]) {
    for (int a = 0; a < 3; a++) {
        c[a] = (int)floor(p[a] / g->cell) + g->half;
        if (c[a] < 1 || c[a] >= g->side - 1) return 0;
    }
    return 1;
}

static int grid_build(grid_t *g, double radius, const double *pos, int count, int cap) {
    free(g->head);
    g->half = (int)ceil(1.5 * radius / g->cell) + 4;
    g->side = 2 * g->half;
    size_t n = (size_t)g->side * g->side * g->side;
    g->head = (int *)malloc(n * sizeof(int));
    if (!g->head) return 0;
    for (size_t q = 0; q < n; q++) g->head[q] = -1;
    if (!g->next) g->next = (int *)malloc((size_t)cap * sizeof(int));
    for (int q = 0; q < count; q++) {
        int c[3];
        if (!grid_index(g, pos + 3 * q, c)) return 0;
        size_t id = ((size_t)c[2] * g->side + c[1]) * g->side + c[0];
        g->next[q] = g->head[id];
        g->head[id] = q;
    }
    return 1;
}

/* Returns 0 on success, -1 on bad arguments or allocation failure. */
int globule_generate(int n, uint64_t seed, double density, double step, double min_sep,
                     int tries, int restarts_before_grow, double grow, const double *table,
                     const double *prob, int ntable, double *pos, double *radii) {
    if (n < 1 || !(density > 0) || !(step > 0) || !(min_sep > 0) || tries < 1 || ntable < 1)
        return -1;
    rng_t r = {seed * 0x2545F4914F6CDD1Dull + 0x1234567ull};
    double radius = cbrt(3.0 * n / (4.0 * M_PI * density));
    grid_t g = {min_sep, 0, 0, NULL, NULL};
    memset(pos, 0, sizeof(double) * 3 * (size_t)n);
    if (!grid_build(&g, radius, pos, 1, n)) return -1;
    double sep2 = min_sep * min_sep;
    int cur = 0, failed = 0;
    for (int m = 1; m < n; m++) {
        for (;;) {
            int placed = 0;
            double cand[3];
            for (int t = 0; t < tries && !placed; t++) {
                double z = 2.0 * uniform(&r) - 1.0;
                double phi = 2.0 * M_PI * uniform(&r);
                double rr = sqrt(fmax(0.0, 1.0 - z * z));
                cand[0] = pos[3 * cur] + step * rr * cos(phi);
                cand[1] = pos[3 * cur + 1] + step * rr * sin(phi);
                cand[2] = pos[3 * cur + 2] + step * z;
                if (cand[0] * cand[0] + cand[1] * cand[1] + cand[2] * cand[2] > radius * radius)
                    continue;
                int c[3];
                if (!grid_index(&g, cand, c)) continue;
                int ok = 1;
                for (int dz = -1; dz <= 1 && ok; dz++)
                    for (int dy = -1; dy <= 1 && ok; dy++)
                        for (int dx = -1; dx <= 1 && ok; dx++) {
                            size_t id = ((size_t)(c[2] + dz) * g.side + (c[1] + dy)) * g.side +
                                        (c[0] + dx);
                            for (int q = g.head[id]; q >= 0; q = g.next[q]) {
                                if (q == cur) continue;
                                double ex = cand[0] - pos[3 * q], ey = cand[1] - pos[3 * q + 1],
                                       ez = cand[2] - pos[3 * q + 2];
                                if (ex * ex + ey * ey + ez * ez < sep2) {
                                    ok = 0;
                                    break;
                                }
                            }
                        }
                if (ok) placed = 1;
            }
            if (placed) {
                memcpy(pos + 3 * m, cand, sizeof(cand));
                int c[3];
                grid_index(&g, cand, c);
                size_t id = ((size_t)c[2] * g.side + c[1]) * g.side + c[0];
                g.next[m] = g.head[id];
                g.head[id] = m;
                cur = m;
                failed = 0;
                break;
            }
            cur = (int)(uniform(&r) * m);
            if (cur >= m) cur = m - 1;
            if (++failed >= restarts_before_grow) {
                radius *= grow;
                failed = 0;
                if (1.5 * radius / g.cell + 4 > g.half - 2)
                    if (!grid_build(&g, radius, pos, m, n)) return -1;
            }
        }
    }
    for (int i = 0; i < n; i++) {
        double u = uniform(&r), acc = 0.0;
        int k = ntable - 1;
        for (int q = 0; q < ntable; q++) {
            acc += prob[q];
            if (u < acc) {
                k = q;
                break;
            }
        }
        radii[i] = table[k];
    }
    free(g.head);
    free(g.next);
    return 0;
}

/* Log-uniform integers in [lo, hi]. */
void globule_log_uniform(int count, uint64_t seed, double lo, double hi, int *out) {
    rng_t r = {seed * 0x2545F4914F6CDD1Dull + 0x7654321ull};
    for (int q = 0; q < count; q++) out[q] = (int)llround(exp(log(lo) + uniform(&r) * (log(hi) - log(lo))));
}
