/* Drives every entry point of the oracle on a small cluster of atoms, for a
 * build under AddressSanitizer and UndefinedBehaviorSanitizer (test aid). */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void *orc_create(int n, const double *centres, const double *radii, double rho);
void orc_destroy(void *h);
int orc_num_vertices(void *h);
void orc_get_vertices(void *h, double *p, int *atoms, int *sign);
void orc_labels_grid(void *h, const double lo[3], double hs, const int dims[3], int k0, int k1,
                     uint8_t *out);
void orc_labels_grid_cert(void *h, const double lo[3], double hs, const int dims[3], int k0,
                          int k1, uint8_t *out);
void orc_labels_points(void *h, long count, const double *x, uint8_t *out);
void orc_dist_points(void *h, long count, const double *x, double cap, double *out, int *type);
void orc_edges(void *h, const double lo[3], double hs, const int dims[3], long count,
               const long *keys, const int *ends, int *status, double *lambda, double *normal,
               int *type, int *atoms);

int main(void) {
    /* a 3 x 3 x 2 block of atoms 2.9 A apart, shifted off the lattice by a
     * fixed pattern so that no two distances coincide */
    enum { N = 18 };
    double c[3 * N], r[N];
    for (int q = 0; q < N; q++) {
        const int i = q % 3, j = (q / 3) % 3, k = q / 9;
        c[3 * q + 0] = 2.9 * i + 0.07 * ((q * 5) % 7);
        c[3 * q + 1] = 2.9 * j + 0.05 * ((q * 3) % 5);
        c[3 * q + 2] = 2.9 * k + 0.03 * ((q * 7) % 11);
        r[q] = 1.5 + 0.05 * (q % 4);
    }
    void *h = orc_create(N, c, r, 1.4);
    if (!h) return 2;
    const int nv = orc_num_vertices(h);
    double *vp = malloc(sizeof(double) * 3 * (nv + 1));
    int *va = malloc(sizeof(int) * 3 * (nv + 1)), *vs = malloc(sizeof(int) * (nv + 1));
    orc_get_vertices(h, vp, va, vs);
    const double lo[3] = {-4.0, -4.0, -4.0}, hs = 0.5;
    const int dims[3] = {26, 26, 24};
    const long np = (long)dims[0] * dims[1] * dims[2];
    uint8_t *lab = malloc(np), *labc = malloc(np);
    orc_labels_grid(h, lo, hs, dims, 0, dims[2], lab);
    orc_labels_grid_cert(h, lo, hs, dims, 0, dims[2], labc);
    long nin = 0, ndiff = 0;
    for (long q = 0; q < np; q++) {
        nin += lab[q];
        ndiff += labc[q] != 2 && labc[q] != lab[q];
    }
    /* crossing edges along +x, +y, +z */
    long ne = 0;
    long *keys = malloc(sizeof(long) * 3 * np);
    for (long q = 0; q < np; q++) {
        const long i = q % dims[0], j = (q / dims[0]) % dims[1], k = q / ((long)dims[0] * dims[1]);
        const long step[3] = {1, dims[0], (long)dims[0] * dims[1]};
        const long idx[3] = {i, j, k};
        for (int a = 0; a < 3; a++)
            if (idx[a] + 1 < dims[a] && lab[q] != lab[q + step[a]]) keys[ne++] = 3 * q + a;
    }
    int *st = malloc(sizeof(int) * (ne + 1)), *ty = malloc(sizeof(int) * (ne + 1));
    int *at = malloc(sizeof(int) * 3 * (ne + 1));
    double *la = malloc(sizeof(double) * (ne + 1)), *nr = malloc(sizeof(double) * 3 * (ne + 1));
    orc_edges(h, lo, hs, dims, ne, keys, NULL, st, la, nr, ty, at);
    long nok = 0;
    for (long q = 0; q < ne; q++) nok += st[q] == 1;
    double x[12] = {0.1, 0.2, 0.3, 1.5, 1.4, 1.3, -3.0, 0.0, 0.0, 2.9, 2.9, 1.45};
    uint8_t pl[4];
    double d[4];
    int dt[4];
    orc_labels_points(h, 4, x, pl);
    orc_dist_points(h, 4, x, 10.0, d, dt);
    orc_destroy(h);
    printf("OK vertices %d inside %ld cert_mismatch %ld edges %ld records %ld\n", nv, nin, ndiff,
           ne, nok);
    free(vp), free(va), free(vs), free(lab), free(labc), free(keys), free(st), free(ty), free(at);
    free(la), free(nr);
    return ndiff == 0 && nok == ne && nv > 0 ? 0 : 1;
}
