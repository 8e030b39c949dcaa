// Cavity-filled labels: the exterior-only reading of the probe set.
//
// The paper defines the SES through probe balls that overlap no atom
// (section 1) without saying whether probe positions in enclosed cavities
// count; the labels of eq. 2 count them (their surfaces bound the cavities).
// This variant fills the cavities: every outside grid point (label 0) that no
// path of axis-adjacent outside points joins to the boundary of the grid
// becomes inside.  In place, on the labels of eses_classify:
//   seed:   outside points on the grid's boundary faces become 2 (reached);
//   passes: each workgroup loads one 8^3 tile with a one-point halo into LDS
//           and spreads "reached" to axis-adjacent outside points until the
//           tile settles, writes the points it reached and raises a flag;
//           the host repeats passes until no tile changes (values only go
//           0 -> 2, so a stale halo only delays a step to the next pass);
//   finish: 0 -> 1 (filled, counted), 2 -> 0.
#include "eses_device.h"
#include "launch.h"

namespace eses {

constexpr int FT = 8;                 // tile edge (points)
constexpr int FH = FT + 2;            // with halo
constexpr int FILL_THREADS = 256;

__global__ void k_fill_seed(uint8_t *L, int nx, int ny, int nz) {
    const long long n = (long long)nx * ny * nz;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n;
         q += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(q % nx), j = (int)((q / nx) % ny), k = (int)(q / ((long long)nx * ny));
        const bool edge = i == 0 || j == 0 || k == 0 || i == nx - 1 || j == ny - 1 || k == nz - 1;
        if (edge && L[q] == 0) L[q] = 2;
    }
}

// One pass over tiles t = blockIdx.x (+ gridDim.x ...) of one molecule.
__device__ void fill_tile(uint8_t *L, int nx, int ny, int nz, int tx, int ty, int tz, int *changed,
                          uint8_t (*s)[FH][FH], int &dirty) {
    const int i0 = tx * FT - 1, j0 = ty * FT - 1, k0 = tz * FT - 1;
    for (int q = threadIdx.x; q < FH * FH * FH; q += FILL_THREADS) {
        const int a = q % FH, b = (q / FH) % FH, c = q / (FH * FH);
        const int i = i0 + a, j = j0 + b, k = k0 + c;
        uint8_t v = 1;  // outside the grid: a wall
        if (i >= 0 && j >= 0 && k >= 0 && i < nx && j < ny && k < nz)
            v = L[(long long)i + (long long)nx * ((long long)j + (long long)ny * k)];
        s[c][b][a] = v;
    }
    if (threadIdx.x == 0) dirty = 0;
    __syncthreads();
    bool mine = false;  // this thread reached one of its points in this tile
    for (;;) {
        int grew = 0;
        for (int q = threadIdx.x; q < FT * FT * FT; q += FILL_THREADS) {
            const int a = 1 + q % FT, b = 1 + (q / FT) % FT, c = 1 + q / (FT * FT);
            if (s[c][b][a] != 0) continue;
            if (s[c][b][a - 1] == 2 || s[c][b][a + 1] == 2 || s[c][b - 1][a] == 2 ||
                s[c][b + 1][a] == 2 || s[c - 1][b][a] == 2 || s[c + 1][b][a] == 2) {
                s[c][b][a] = 2;
                grew = 1;
                mine = true;
            }
        }
        // every thread leaves the loop on the same round: the round's growth
        // is combined across the workgroup before anyone tests it
        const int any = __syncthreads_or(grew);
        if (!any) break;
    }
    if (mine) {
        for (int q = threadIdx.x; q < FT * FT * FT; q += FILL_THREADS) {
            const int a = 1 + q % FT, b = 1 + (q / FT) % FT, c = 1 + q / (FT * FT);
            const int i = i0 + a, j = j0 + b, k = k0 + c;
            if (i >= nx || j >= ny || k >= nz) continue;
            const long long g = (long long)i + (long long)nx * ((long long)j + (long long)ny * k);
            if (s[c][b][a] == 2 && L[g] == 0) {
                L[g] = 2;
                dirty = 1;
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0 && dirty) atomicOr(changed, 1);
    __syncthreads();
}

// Every tile of every molecule of a batch (units as the classification's:
// (molecule, tile) pairs; tiles of edge `tile` points of the molecule).
__global__ void __launch_bounds__(FILL_THREADS) k_fill_pass(const Mol *mols,
                                                           uint8_t *const *labels,
                                                           const int2 *units, int nunits,
                                                           int *changed) {
    __shared__ uint8_t s[FH][FH][FH];
    __shared__ int dirty;
    for (int u = blockIdx.x; u < nunits; u += gridDim.x) {
        const int2 w = units[u];
        const Mol &m = mols[w.x];
        const int tiles_x = (m.dims[0] + FT - 1) / FT, tiles_y = (m.dims[1] + FT - 1) / FT;
        const int t = w.y;
        fill_tile(labels[w.x], m.dims[0], m.dims[1], m.dims[2], t % tiles_x, (t / tiles_x) % tiles_y,
                  t / (tiles_x * tiles_y), changed, s, dirty);
    }
}

// One molecule: tiles by block index.
__global__ void __launch_bounds__(FILL_THREADS) k_fill_pass1(uint8_t *L, int nx, int ny, int nz,
                                                            int *changed) {
    __shared__ uint8_t s[FH][FH][FH];
    __shared__ int dirty;
    const int tiles_x = (nx + FT - 1) / FT, tiles_y = (ny + FT - 1) / FT,
              tiles_z = (nz + FT - 1) / FT;
    const long long nt = (long long)tiles_x * tiles_y * tiles_z;
    for (long long t = blockIdx.x; t < nt; t += gridDim.x)
        fill_tile(L, nx, ny, nz, (int)(t % tiles_x), (int)((t / tiles_x) % tiles_y),
                  (int)(t / ((long long)tiles_x * tiles_y)), changed, s, dirty);
}

__global__ void k_fill_finish(uint8_t *L, long long n, unsigned long long *filled) {
    unsigned long long c = 0;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n;
         q += (long long)gridDim.x * blockDim.x) {
        const uint8_t v = L[q];
        if (v == 0) {
            L[q] = 1;
            ++c;
        } else if (v == 2) {
            L[q] = 0;
        }
    }
    for (int d = WAVE / 2; d > 0; d >>= 1) c += __shfl_down(c, d, WAVE);
    if (lane_id() == 0 && c) atomicAdd(filled, c);
}

static unsigned grid_for(long long n, int bs, long long cap) {
    long long b = (n + bs - 1) / bs;
    if (b > cap) b = cap;
    return (unsigned)(b < 1 ? 1 : b);
}

hipError_t launch_fill_seed(uint8_t *L, const int dims[3], hipStream_t st) {
    const long long n = (long long)dims[0] * dims[1] * dims[2];
    hipLaunchKernelGGL(k_fill_seed, dim3(grid_for(n, 256, 8192)), dim3(256), 0, st, L, dims[0],
                       dims[1], dims[2]);
    return hipGetLastError();
}

hipError_t launch_fill_pass(const Mol *mols_dev, uint8_t *const *labels_dev, const int2 *units,
                            int nunits, int *changed, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_pass, dim3(grid_for(nunits, 1, 8192)), dim3(FILL_THREADS), 0, st,
                       mols_dev, labels_dev, units, nunits, changed);
    return hipGetLastError();
}

hipError_t launch_fill_pass1(uint8_t *L, const int dims[3], int *changed, hipStream_t st) {
    const long long nt = (long long)((dims[0] + FT - 1) / FT) * ((dims[1] + FT - 1) / FT) *
                         ((dims[2] + FT - 1) / FT);
    hipLaunchKernelGGL(k_fill_pass1, dim3(grid_for(nt, 1, 8192)), dim3(FILL_THREADS), 0, st, L,
                       dims[0], dims[1], dims[2], changed);
    return hipGetLastError();
}

hipError_t launch_fill_finish(uint8_t *L, long long n, unsigned long long *filled,
                              hipStream_t st) {
    hipLaunchKernelGGL(k_fill_finish, dim3(grid_for(n, 256, 4096)), dim3(256), 0, st, L, n, filled);
    return hipGetLastError();
}

}  // namespace eses
