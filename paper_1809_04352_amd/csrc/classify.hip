// Stage 2: inside/outside label of every grid point (eq. 2).
//
// One workgroup per tile of TILE^3 points.  Each lane owns one point; the
// tile's candidate lists (shared by all its points) are read through the
// cache, and the label is written as one byte per point (x fastest).
#include "eses_device.h"
#include "launch.h"

namespace eses {

constexpr int CLS_BLOCK = 512;

__global__ void __launch_bounds__(CLS_BLOCK) k_classify_fp64(Mol m, uint8_t *labels) {
    const int T = m.tile;
    const int per = T * T * T;
    const int tiles_per_block = CLS_BLOCK / per;
    int tile = blockIdx.x * tiles_per_block + threadIdx.x / per;
    if (tile >= m.ntiles) return;
    int local = threadIdx.x % per;
    int t3[3] = {tile % m.tdims[0], (tile / m.tdims[0]) % m.tdims[1],
                 tile / (m.tdims[0] * m.tdims[1])};
    int i = t3[0] * T + local % T;
    int j = t3[1] * T + (local / T) % T;
    int k = t3[2] * T + local / (T * T);
    if (i >= m.dims[0] || j >= m.dims[1] || k >= m.dims[2]) return;
    double x = grid_coord(m.lo[0], m.h, i);
    double y = grid_coord(m.lo[1], m.h, j);
    double z = grid_coord(m.lo[2], m.h, k);
    int lab = label_fp64(m, tile, x, y, z);
    labels[(long long)i + (long long)m.dims[0] * ((long long)j + (long long)m.dims[1] * k)] =
        (uint8_t)lab;
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
            label_fp64_t<true>(m, tile, grid_coord(m.lo[0], m.h, i), grid_coord(m.lo[1], m.h, j),
                               grid_coord(m.lo[2], m.h, k), cnt);
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

hipError_t launch_classify_fp64(const Mol &m, uint8_t *labels, hipStream_t st) {
    const int per = m.tile * m.tile * m.tile;
    const int tpb = CLS_BLOCK / per;
    unsigned nb = (unsigned)((m.ntiles + tpb - 1) / tpb);
    hipLaunchKernelGGL(k_classify_fp64, dim3(nb < 1 ? 1 : nb), dim3(CLS_BLOCK), 0, st, m, labels);
    return hipGetLastError();
}

}  // namespace eses
