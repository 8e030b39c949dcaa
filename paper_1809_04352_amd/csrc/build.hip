// Stage 1 kernels: cell binning, SAS neighbours and pair circles, concave
// probe positions, exposure flags, exposed-feature cut lists and per-tile
// candidate lists.  Every list is built in two passes (count, scan, fill) so
// its order is deterministic.
#include "eses_device.h"
#include "launch.h"

namespace eses {

// Molecule of block b of a segmented launch: the largest q with start[q] <= b.
__device__ inline int seg_mol(const Seg &s, int b) {
    int lo = 0, hi = s.nm - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s.start[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// The molecule view m, its temporaries tmp and the block's index bid within
// the molecule, for a kernel launched over a Seg.
#define SEG_BEGIN(s)                                   \
    const int seg_q_ = seg_mol(s, (int)blockIdx.x);     \
    const Mol &m = (s).mols[seg_q_];                    \
    const BuildTmp &tmp = (s).tmp[seg_q_];              \
    const int bid = (int)blockIdx.x - (s).start[seg_q_]

// ----------------------------------------------------------------- utilities

__global__ void k_fill_i32(int *p, long long n, int v) { fill_i32(p, n, v); }

__global__ void k_copy_i32(int *dst, const int *src, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// Scalars the host reads back, gathered into host memory by one thread.
__global__ void k_collect(ReadBack rb, long long *host) {
    for (int q = 0; q < rb.n; ++q)
        host[q] = rb.is64[q] ? *(const long long *)rb.p[q] : (long long)*(const int *)rb.p[q];
}

hipError_t launch_collect(const ReadBack &rb, long long *host, hipStream_t st) {
    hipLaunchKernelGGL(k_collect, dim3(1), dim3(1), 0, st, rb, host);
    return hipGetLastError();
}

__global__ void k_fill_u32(uint32_t *p, long long n, uint32_t v) {
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n;
         q += (long long)gridDim.x * blockDim.x)
        p[q] = v;
}

// Exclusive scan, three passes: per-block sums, one-block scan of the sums,
// per-block scan plus offset.  out has n + 1 entries (out[n] = total).
constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;

template <typename T>
__global__ void __launch_bounds__(SCAN_BLOCK) k_scan_reduce(const int *in, long long n, T *bsum) {
    __shared__ T lds[SCAN_BLOCK / WAVE + 1];
    long long base = (long long)blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
    T v = 0;
#pragma unroll
    for (int q = 0; q < SCAN_ITEMS; ++q)
        if (base + q < n) v += (T)in[base + q];
    T tot;
    block_excl_scan<T, SCAN_BLOCK>(v, lds, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

template <typename T>
__global__ void __launch_bounds__(SCAN_BLOCK) k_scan_blocks(T *bsum, long long nb) {
    __shared__ T lds[SCAN_BLOCK / WAVE + 1];
    T carry = 0;
    for (long long b0 = 0; b0 < nb; b0 += SCAN_BLOCK) {
        long long q = b0 + threadIdx.x;
        T v = q < nb ? bsum[q] : T(0);
        T tot;
        T ex = block_excl_scan<T, SCAN_BLOCK>(v, lds, &tot);
        if (q < nb) bsum[q] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) bsum[nb] = carry;
}

template <typename T>
__global__ void __launch_bounds__(SCAN_BLOCK) k_scan_apply(const int *in, long long n,
                                                           const T *bsum, T *out) {
    __shared__ T lds[SCAN_BLOCK / WAVE + 1];
    long long base = (long long)blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
    T vals[SCAN_ITEMS];
    T v = 0;
#pragma unroll
    for (int q = 0; q < SCAN_ITEMS; ++q) {
        vals[q] = base + q < n ? (T)in[base + q] : T(0);
        v += vals[q];
    }
    T tot;
    T ex = block_excl_scan<T, SCAN_BLOCK>(v, lds, &tot) + bsum[blockIdx.x];
#pragma unroll
    for (int q = 0; q < SCAN_ITEMS; ++q) {
        if (base + q < n) out[base + q] = ex;
        ex += vals[q];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = bsum[gridDim.x];
}

// Inputs up to SCAN1_MAX: one workgroup walks the input in coalesced tiles
// of SCAN1_BLOCK x 4 elements, carrying the running total, so the scan is a
// single launch; blockIdx.x selects one of several arrays of equal length.
constexpr int SCAN1_BLOCK = 1024;
constexpr long long SCAN1_MAX = 1 << 15;

struct ScanArrays {
    const int *in[4];
    void *out[4];
};

template <typename T>
__global__ void __launch_bounds__(SCAN1_BLOCK) k_scan_small(ScanArrays a, long long n) {
    __shared__ T lds[SCAN1_BLOCK / WAVE + 1];
    const int *in = a.in[blockIdx.x];
    T *out = (T *)a.out[blockIdx.x];
    T carry = 0;
    for (long long b0 = 0; b0 < n; b0 += 4 * SCAN1_BLOCK) {
        const long long b = b0 + 4 * threadIdx.x;
        T v[4];
        T sum = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            v[q] = b + q < n ? (T)in[b + q] : T(0);
            sum += v[q];
        }
        T tot;
        T ex = block_excl_scan<T, SCAN1_BLOCK>(sum, lds, &tot) + carry;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (b + q < n) out[b + q] = ex;
            ex += v[q];
        }
        carry += tot;
    }
    if (threadIdx.x == 0) out[n] = carry;
}

template <typename T>
static hipError_t scan_impl(const int *in, long long n, T *out, T *tmp, hipStream_t st) {
    if (n <= SCAN1_MAX) {
        ScanArrays a{};
        a.in[0] = in;
        a.out[0] = out;
        hipLaunchKernelGGL(k_scan_small<T>, dim3(1), dim3(SCAN1_BLOCK), 0, st, a, n);
        return hipGetLastError();
    }
    long long nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_scan_reduce<T>, dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, st, in, n, tmp);
    hipLaunchKernelGGL(k_scan_blocks<T>, dim3(1), dim3(SCAN_BLOCK), 0, st, tmp, nb);
    hipLaunchKernelGGL(k_scan_apply<T>, dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, st, in, n, tmp,
                       out);
    return hipGetLastError();
}

long long scan_tmp_elems(long long n) { return (n + SCAN_TILE - 1) / SCAN_TILE + 2; }

hipError_t scan_i32(const int *in, long long n, int *out, int *tmp, hipStream_t st) {
    return scan_impl<int>(in, n, out, tmp, st);
}

hipError_t scan_i64(const int *in, long long n, long long *out, long long *tmp, hipStream_t st) {
    return scan_impl<long long>(in, n, out, tmp, st);
}

hipError_t scan_i32_multi(const int *const *in, long long n, int *const *out, int k, int *tmp,
                          hipStream_t st) {
    if (k < 1 || k > 4) return hipErrorInvalidValue;
    if (n <= SCAN1_MAX) {
        ScanArrays a{};
        for (int q = 0; q < k; ++q) {
            a.in[q] = in[q];
            a.out[q] = out[q];
        }
        hipLaunchKernelGGL(k_scan_small<int>, dim3(k), dim3(SCAN1_BLOCK), 0, st, a, n);
        return hipGetLastError();
    }
    for (int q = 0; q < k; ++q) {
        hipError_t e = scan_impl<int>(in[q], n, out[q], tmp, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t fill_i32(int *p, long long n, int v, hipStream_t st) {
    long long nb = (n + 255) / 256;
    if (nb > 4096) nb = 4096;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)nb), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t copy_i32(int *dst, const int *src, long long n, hipStream_t st) {
    long long nb = (n + 255) / 256;
    if (nb > 4096) nb = 4096;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_copy_i32, dim3((unsigned)nb), dim3(256), 0, st, dst, src, n);
    return hipGetLastError();
}

hipError_t fill_u32(uint32_t *p, long long n, uint32_t v, hipStream_t st) {
    long long nb = (n + 255) / 256;
    if (nb > 4096) nb = 4096;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)nb), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

// Segmented scans (see launch.h): block b of the chunk passes finds its array
// by binary search over the arrays' first chunks.
__device__ inline int sseg_of(const ScanSeg *segs, int nseg, long long b) {
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (segs[mid].chunk0 <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ void __launch_bounds__(SCAN_BLOCK) k_sseg_reduce(const ScanSeg *segs, int nseg,
                                                            int *sums) {
    __shared__ int lds[SCAN_BLOCK / WAVE + 1];
    const int g = sseg_of(segs, nseg, blockIdx.x);
    const ScanSeg sg = segs[g];
    const long long base = (blockIdx.x - sg.chunk0) * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
    int v = 0;
#pragma unroll
    for (int q = 0; q < SCAN_ITEMS; ++q)
        if (base + q < sg.n) v += sg.in[base + q];
    int tot;
    block_excl_scan<int, SCAN_BLOCK>(v, lds, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(SCAN_BLOCK) k_sseg_blocks(const ScanSeg *segs, int nseg,
                                                            int *sums) {
    __shared__ int lds[SCAN_BLOCK / WAVE + 1];
    const ScanSeg sg = segs[blockIdx.x];
    const long long nb = (sg.n + SCAN_TILE - 1) / SCAN_TILE;
    int carry = 0;
    for (long long b0 = 0; b0 < nb; b0 += SCAN_BLOCK) {
        const long long q = b0 + threadIdx.x;
        const int v = q < nb ? sums[sg.chunk0 + q] : 0;
        int tot;
        const int ex = block_excl_scan<int, SCAN_BLOCK>(v, lds, &tot);
        if (q < nb) sums[sg.chunk0 + q] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) sg.out[sg.n] = carry;
}

__global__ void __launch_bounds__(SCAN_BLOCK) k_sseg_apply(const ScanSeg *segs, int nseg,
                                                           const int *sums) {
    __shared__ int lds[SCAN_BLOCK / WAVE + 1];
    const int g = sseg_of(segs, nseg, blockIdx.x);
    const ScanSeg sg = segs[g];
    const long long base = (blockIdx.x - sg.chunk0) * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
    int vals[SCAN_ITEMS];
    int v = 0;
#pragma unroll
    for (int q = 0; q < SCAN_ITEMS; ++q) {
        vals[q] = base + q < sg.n ? sg.in[base + q] : 0;
        v += vals[q];
    }
    int tot;
    int ex = block_excl_scan<int, SCAN_BLOCK>(v, lds, &tot) + sums[blockIdx.x];
#pragma unroll
    for (int q = 0; q < SCAN_ITEMS; ++q) {
        if (base + q < sg.n) sg.out[base + q] = ex;
        ex += vals[q];
    }
}

long long scan_seg_chunk() { return SCAN_TILE; }

hipError_t scan_seg(const ScanSeg *segs, int nseg, long long nchunks, int *sums, hipStream_t st) {
    if (nseg <= 0) return hipSuccess;
    if (nchunks > 0)
        hipLaunchKernelGGL(k_sseg_reduce, dim3((unsigned)nchunks), dim3(SCAN_BLOCK), 0, st, segs,
                           nseg, sums);
    hipLaunchKernelGGL(k_sseg_blocks, dim3((unsigned)nseg), dim3(SCAN_BLOCK), 0, st, segs, nseg,
                       sums);
    if (nchunks > 0)
        hipLaunchKernelGGL(k_sseg_apply, dim3((unsigned)nchunks), dim3(SCAN_BLOCK), 0, st, segs,
                           nseg, sums);
    return hipGetLastError();
}

__global__ void k_gather_ints(const int *const *addr, int n, int *out) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) out[q] = *addr[q];
}

hipError_t launch_gather_ints(const int *const *addr, int n, int *out, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_ints, dim3((n + 255) / 256), dim3(256), 0, st, addr, n, out);
    return hipGetLastError();
}

// ----------------------------------------------------------- atom binning

// Bounds of the centres and the largest radius; flags non-finite or
// non-positive input.  One block.
__global__ void __launch_bounds__(256) k_bounds(Seg sg) {
    SEG_BEGIN(sg);
    (void)bid;
    const double *c = m.in_c, *r = m.in_r;
    const long long n = m.n;
    double *out = tmp.bounds;
    int *bad = tmp.bad;
    __shared__ double sh[7][256];
    __shared__ int shbad[256];
    double v[7] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY, 0.0};
    int b = 0;
    for (long long i = threadIdx.x; i < n; i += blockDim.x) {
        double x = c[3 * i], y = c[3 * i + 1], z = c[3 * i + 2], rr = r[i];
        if (!isfinite(x) || !isfinite(y) || !isfinite(z) || !isfinite(rr) || !(rr > 0.0)) b = 1;
        v[0] = fmin(v[0], x);
        v[1] = fmin(v[1], y);
        v[2] = fmin(v[2], z);
        v[3] = fmax(v[3], x);
        v[4] = fmax(v[4], y);
        v[5] = fmax(v[5], z);
        v[6] = fmax(v[6], rr);
    }
    for (int q = 0; q < 7; ++q) sh[q][threadIdx.x] = v[q];
    shbad[threadIdx.x] = b;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            for (int q = 0; q < 3; ++q) sh[q][threadIdx.x] = fmin(sh[q][threadIdx.x], sh[q][threadIdx.x + s]);
            for (int q = 3; q < 7; ++q) sh[q][threadIdx.x] = fmax(sh[q][threadIdx.x], sh[q][threadIdx.x + s]);
            shbad[threadIdx.x] |= shbad[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        for (int q = 0; q < 7; ++q) out[q] = sh[q][0];
        *bad = shbad[0];
    }
}

__device__ inline int cell_axis(const Mol &m, double x, int a) {
    int c = (int)floor((x - m.clo[a]) / m.cell);
    return c < 0 ? 0 : (c >= m.nc[a] ? m.nc[a] - 1 : c);
}

__global__ void k_cell_count(Seg sg) {
    SEG_BEGIN(sg);
    int *cell_id = tmp.cell_id, *count = tmp.cnt;
    int i = bid * blockDim.x + threadIdx.x;
    if (i >= m.n) return;
    int c = cell_axis(m, m.in_c[3 * i], 0) +
            m.nc[0] * (cell_axis(m, m.in_c[3 * i + 1], 1) + m.nc[1] * cell_axis(m, m.in_c[3 * i + 2], 2));
    cell_id[i] = c;
    atomicAdd(&count[c], 1);
}

// Cursor per cell: its first slot (cell_start after the scan).
__global__ void k_cell_fill_init(Seg sg) {
    SEG_BEGIN(sg);
    const int c = bid * blockDim.x + threadIdx.x;
    if (c <= m.ncell) tmp.fillb[c] = m.cell_start[c];
}

__global__ void k_cell_scatter(Seg sg) {
    SEG_BEGIN(sg);
    const int *cell_id = tmp.cell_id;
    int *fill = tmp.fillb, *slot_orig = tmp.slot;
    int i = bid * blockDim.x + threadIdx.x;
    if (i >= m.n) return;
    int pos = atomicAdd(&fill[cell_id[i]], 1);
    slot_orig[pos] = i;
}

// Sort each cell's caller ids ascending, then gather the atoms into internal
// order.  One wavefront per cell ranks its ids in LDS (the ids are distinct);
// a cell larger than the LDS slice is sorted by one lane.
constexpr int CS_WAVES = 4, CS_MAX = 256;

__global__ void __launch_bounds__(CS_WAVES *WAVE) k_cell_sort(Seg sg) {
    __shared__ int ids[CS_WAVES][CS_MAX];
    SEG_BEGIN(sg);
    int *slot_orig = tmp.slot;
    const int w = threadIdx.x / WAVE, lane = lane_id();
    const int c = bid * CS_WAVES + w;
    if (c >= m.ncell) return;  // uniform across the wavefront; no workgroup barrier below
    const int b = m.cell_start[c], n = m.cell_start[c + 1] - b;
    if (n <= 1) return;
    if (n > CS_MAX) {
        if (lane == 0)
            for (int q = b + 1; q < b + n; ++q) {
                int v = slot_orig[q];
                int p = q - 1;
                while (p >= b && slot_orig[p] > v) {
                    slot_orig[p + 1] = slot_orig[p];
                    --p;
                }
                slot_orig[p + 1] = v;
            }
        return;
    }
    for (int q = lane; q < n; q += WAVE) ids[w][q] = slot_orig[b + q];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int q = lane; q < n; q += WAVE) {
        const int v = ids[w][q];
        int rank = 0;
        for (int p = 0; p < n; ++p) rank += ids[w][p] < v ? 1 : 0;
        slot_orig[b + rank] = v;
    }
}

__global__ void k_gather_atoms(Seg sg) {
    SEG_BEGIN(sg);
    const int *slot_orig = tmp.slot;
    int q = bid * blockDim.x + threadIdx.x;
    if (q >= m.n) return;
    int i = slot_orig[q];
    m.orig[q] = i;
    m.atom[q] = make_double4(m.in_c[3 * i], m.in_c[3 * i + 1], m.in_c[3 * i + 2], m.in_r[i]);
}

// A fill pass writes slot `at` of a range sized by its count pass.  Both
// passes take the same decisions, but a write past the range is dropped and
// counted rather than trusted.
__device__ inline bool fill_ok(const Mol &m, long long at, long long end) {
    if (at < end) return true;
    atomicAdd(&m.diag[0], 1);
    return false;
}

// ------------------------------------------------ SAS neighbours and circles

// Cover-order key of neighbour k of atom i (s_i = r_i + rho): the cosine of
// the half-angle of the cap S_k cuts from S_i, tau_ik / d_ik.
__device__ inline double cover_key(double4 ai, double si, double4 ak, double rho) {
    const double sk = ak.w + rho;
    const double d2 = sq(ak.x - ai.x) + sq(ak.y - ai.y) + sq(ak.z - ai.z);
    return (si * si + d2 - sk * sk) / (2.0 * si * sqrt(d2));
}

// One wavefront per internal atom i; the atoms of the 5x5x5 stencil of cells
// (edge at least s_max plus the list slack, so that every candidate lies
// within two cells along each axis), row by row, are spread over the lanes
// and ballots compact the hits.  Stencil
// cells are visited in increasing cell index and internal ids increase with
// the cell index, so each neighbour list comes out ascending.
constexpr int NB_WAVES = 4;

template <bool FILL>
__global__ void __launch_bounds__(NB_WAVES *WAVE) k_nbr(Seg sg) {
    // per wavefront: the first atom and inclusive end offset of each of the
    // stencil's (y, z) cell rows (at most 25)
    __shared__ int rbeg[NB_WAVES][25], rend[NB_WAVES][25];
    // fill pass, pooled atoms: the cover-order keys of the atom's neighbours
    __shared__ double ckey[FILL ? NB_WAVES : 1][FILL ? NBR_POOL : 1];
    SEG_BEGIN(sg);
    int *nbr_cnt = tmp.nbr_cnt, *circ_cnt = tmp.circ_cnt;
    const int wv = threadIdx.x / WAVE;
    int i = bid * NB_WAVES + wv;
    if (i >= m.n) return;  // uniform across the wavefront (no block barriers)
    const int lane = lane_id();
    double4 ai = m.atom[i];
    double si = ai.w + m.rho;
    if (FILL && m.nbr_off[i + 1] - m.nbr_off[i] <= NBR_POOL) {
        const auto pool = tmp.nbr_pool + (long long)i * NBR_POOL;
        // the count pass kept this atom's neighbours (ascending): the same
        // lists from them, with the same arithmetic per neighbour
        const int wn = m.nbr_off[i], nlist = m.nbr_off[i + 1] - wn;
        const int wc = m.circ_off[i], ecc = m.circ_off[i + 1];
        int nc = 0;
        for (int base = 0; base < nlist; base += WAVE) {
            const int t = base + lane;
            bool circ = false;
            int k = -1;
            double4 oR = make_double4(0, 0, 0, 0), n = make_double4(0, 0, 0, 0);
            if (t < nlist) {
                k = pool[t];
                m.nbr[wn + t] = k;
                const double4 ak = m.atom[k];
                ckey[wv][t] = cover_key(ai, si, ak, m.rho);
                if (k > i) circ = pair_circle(ai, ak, m.rho, oR, n);
            }
            const unsigned long long bc = __ballot(circ);
            const int pc = wc + nc + mask_prefix(bc);
            if (circ && fill_ok(m, pc, ecc)) {
                m.circ_i[pc] = i;
                m.circ_j[pc] = k;
                m.circ_oR[pc] = oR;
                m.circ_n[pc] = n;
                m.cflag[pc] = 0u;
            }
            nc += __popcll(bc);
        }
        // the same list in cover order (as k_nbr_sort ranks longer lists)
        wave_sync();
        for (int q = lane; q < nlist; q += WAVE) {
            const double kq = ckey[wv][q];
            int rank = 0;
            for (int p = 0; p < nlist; ++p) {
                const double kp = ckey[wv][p];
                rank += (kp < kq || (kp == kq && p < q)) ? 1 : 0;
            }
            m.nbr_cov[wn + rank] = pool[q];
        }
        return;
    }
    int cx = cell_axis(m, ai.x, 0), cy = cell_axis(m, ai.y, 1), cz = cell_axis(m, ai.z, 2);
    const int x0 = max(cx - 2, 0), x1 = min(cx + 2, m.nc[0] - 1);
    const int y0 = max(cy - 2, 0), y1 = min(cy + 2, m.nc[1] - 1);
    const int z0 = max(cz - 2, 0), z1 = min(cz + 2, m.nc[2] - 1);
    const int ny = y1 - y0 + 1, nr = ny * (z1 - z0 + 1);
    // the cells of one row are consecutive, and so are their atoms: lane r
    // reads row r's range, then the rows' atoms are taken 64 at a time
    // across the lanes (row-major, ascending within a row: ascending ids)
    int kb = 0, ke = 0;
    if (lane < nr) {
        const int c = m.nc[0] * (y0 + lane % ny + m.nc[1] * (z0 + lane / ny));
        kb = m.cell_start[c + x0];
        ke = m.cell_start[c + x1 + 1];
    }
    const int incl = wave_incl_scan(ke - kb);
    if (lane < nr) {
        rbeg[wv][lane] = kb;
        rend[wv][lane] = incl;
    }
    wave_sync();
    const int total = __shfl(incl, WAVE - 1, WAVE);
    int nn = 0, nc = 0, nany = 0;
    bool contained = false;
    int wn = FILL ? m.nbr_off[i] : 0, en = FILL ? m.nbr_off[i + 1] : 0;
    int wc = FILL ? m.circ_off[i] : 0, ecc = FILL ? m.circ_off[i + 1] : 0;
    auto pool = tmp.nbr_pool + (long long)i * NBR_POOL;
    for (int base = 0; base < total; base += WAVE) {
        const int t = base + lane;
        int k = -1;
        if (t < total) {
            int r = 0;
            while (rend[wv][r] <= t) ++r;
            k = rbeg[wv][r] + t - (r > 0 ? rend[wv][r - 1] : 0);
        }
        bool nb = false, circ = false, any = false;
        double4 oR = make_double4(0, 0, 0, 0), n = make_double4(0, 0, 0, 0);
        if (k >= 0 && k != i) {
            double4 ak = m.atom[k];
            double sk = ak.w + m.rho;
            double dx = ak.x - ai.x, dy = ak.y - ai.y, dz = ak.z - ai.z;
            double d2 = dx * dx + dy * dy + dz * dz;
            nb = d2 < sq(si + sk + LIST_SLACK);
            if (!FILL && d2 == 0.0) atomicAdd(&m.diag[2], 1);  // coincident centres: rejected
            if (nb) {
                if (sqrt(d2) + si < sk) contained = true;
                if (pair_circle(ai, ak, m.rho, oR, n)) {
                    any = true;
                    circ = k > i;
                }
            }
        }
        unsigned long long bn = __ballot(nb), bc = __ballot(circ), ba = __ballot(any);
        if (!FILL) {
            const int pn = nn + mask_prefix(bn);
            if (nb && pn < NBR_POOL) pool[pn] = k;
        }
        if (FILL) {
            int pn = wn + nn + mask_prefix(bn);
            if (nb && fill_ok(m, pn, en)) m.nbr[pn] = k;
            int pc = wc + nc + mask_prefix(bc);
            if (circ && fill_ok(m, pc, ecc)) {
                m.circ_i[pc] = i;
                m.circ_j[pc] = k;
                m.circ_oR[pc] = oR;
                m.circ_n[pc] = n;
                m.cflag[pc] = 0u;
            }
        }
        nn += __popcll(bn);
        nc += __popcll(bc);
        nany += __popcll(ba);
    }
    unsigned long long bcont = __ballot(contained);
    if (!FILL && lane == 0) {
        if (nn > NBR_POOL) atomicAdd(tmp.nbr_big, 1);
        nbr_cnt[i] = nn;
        circ_cnt[i] = nc;
        m.circ_any[i] = nany;
        m.aflag[i] = bcont ? AF_CONTAINED : 0u;
    }
}

// Neighbour lists re-ordered by the cap each neighbour cuts from S_i,
// largest first (ascending cos of the cap's half-angle, tau_ik / d_ik), so
// loops that stop at the first covering ball find it early.  One wavefront
// per atom ranks its list in LDS; a list longer than NS_MAX keeps the
// ascending order.
constexpr int NS_WAVES = 4;
constexpr int NS_MAX = 256;

__global__ void __launch_bounds__(NS_WAVES *WAVE) k_nbr_sort(Seg sg) {
    __shared__ double keys[NS_WAVES][NS_MAX];
    SEG_BEGIN(sg);
    (void)tmp;
    const int w = threadIdx.x / WAVE;
    const int lane = lane_id();
    const int i = bid * NS_WAVES + w;
    // every wavefront reaches the barrier below; `mode` says what it does
    int b = 0, n = 0, mode = 0;  // 0 idle, 1 copy unsorted, 2 rank
    if (i < m.n) {
        b = m.nbr_off[i];
        n = m.nbr_off[i + 1] - b;
        // lists within the neighbour pool were ranked by the fill pass
        mode = n <= NBR_POOL ? 0 : n > NS_MAX ? 1 : 2;
    }
    if (mode == 1)
        for (int q = lane; q < n; q += WAVE) m.nbr_cov[b + q] = m.nbr[b + q];
    if (mode == 2) {
        double4 ai = m.atom[i];
        double si = ai.w + m.rho;
        for (int q = lane; q < n; q += WAVE) keys[w][q] = cover_key(ai, si, m.atom[m.nbr[b + q]], m.rho);
    }
    __syncthreads();
    if (mode == 2) {
        for (int q = lane; q < n; q += WAVE) {
            double kq = keys[w][q];
            int rank = 0;
            for (int p = 0; p < n; ++p) {
                double kp = keys[w][p];
                rank += (kp < kq || (kp == kq && p < q)) ? 1 : 0;
            }
            m.nbr_cov[b + rank] = m.nbr[b + q];
        }
    }
}

// ------------------------------------------------- concave probe positions

// Circle id of the pair (a, b), a < b, or -1.
__device__ inline int find_circle(const Mol &m, int a, int b) {
    int lo = m.circ_off[a], hi = m.circ_off[a + 1] - 1;
    while (lo <= hi) {
        int mid = (lo + hi) >> 1;
        int v = m.circ_j[mid];
        if (v == b) return mid;
        if (v < b) lo = mid + 1;
        else hi = mid - 1;
    }
    return -1;
}

// One wavefront per circle (i, j); lanes take the neighbours k > j of i.
// The circle meets S_k where the in-plane angle phi to the direction of c_k
// satisfies
//   cos(phi) = (|c_k - o|^2 + R^2 - s_k^2) / (2 R b_k),
// b_k = distance of c_k from the circle's axis.  The two points are
// o + R (cos(phi) e +- sin(phi) n x e), e = in-plane unit vector towards c_k;
// the "+" point has (p - c_i) . ((c_j - c_i) x (c_k - c_i)) > 0.  A point is
// kept iff no neighbour other than j, k holds it strictly inside its SAS ball
// (points on S_i can only be inside balls of i's neighbours).  Output order:
// k ascending, "+" before "-".
constexpr int VX_WAVES = 4;
constexpr int VX_NBR = 128;  // neighbours (and circles) of atom i staged in LDS

// Atom i's neighbours (cover order with (r + rho)^2, ascending order with the
// atom records) and i's circles, staged for the wavefronts of its workgroup.
// Admissibility of a three-sphere point p (section 1): kept when every other
// atom has |p - c_l|^2 >= s_l^2 (1 - VERTEX_TOL).  A probe that touches four
// or more atoms exactly is then reported by every triple of them, whatever the
// rounding of p.
constexpr double VERTEX_TOL = 1e-9;

struct VxLds {
    double4 nat[VX_NBR];
    double4 natasc[VX_NBR];
    double4 coR[VX_NBR];
    double4 cn[VX_NBR];
    int nid[VX_NBR];
    int nasc[VX_NBR];
    int cj[VX_NBR];
};

// The concave probe positions on circle c = (i, j): for each neighbour k of
// i above j, the two points of the circle at distance s_k from c_k, kept if
// no other neighbour's SAS ball holds them (i's neighbours 0..nst-1 from
// LDS, the rest from global memory).
// Geometry of c_k against circle (o, R, n): w = c_k - o, its axial part t,
// in-plane part p (|p|^2 = b2), |w|^2 = ww and num = |w|^2 + R^2 - s_k^2.
// One code path (and no contraction) for every caller, so the values are
// bitwise the same wherever they are computed.
struct VxAxis {
    double px, py, pz, t, b2, ww, num, sk;
};

__device__ inline VxAxis vx_axis(const Mol &m, double4 oR, double4 n, double4 ak) {
#pragma clang fp contract(off)
    VxAxis g;
    g.sk = ak.w + m.rho;
    const double wx = ak.x - oR.x, wy = ak.y - oR.y, wz = ak.z - oR.z;
    g.t = wx * n.x + wy * n.y + wz * n.z;
    g.px = wx - g.t * n.x;
    g.py = wy - g.t * n.y;
    g.pz = wz - g.t * n.z;
    g.b2 = g.px * g.px + g.py * g.py + g.pz * g.pz;
    g.ww = wx * wx + wy * wy + wz * wz;
    g.num = g.ww + oR.w * oR.w - g.sk * g.sk;
    return g;
}

// False only when S_k certainly misses the circle: num^2 > 4 R^2 b2 (1 +
// 1e-10) puts |cos(phi)| = |num| / (2 R sqrt(b2)) above 1 by far more than
// the few roundings of its computed value, which is then outside [-1, 1] too.
__device__ inline bool vx_maybe_live(const VxAxis &g, double R) {
    return g.num * g.num <= 4.0 * R * R * g.b2 * (1.0 + 1e-10);
}

// The two points of circle (o, R, n) at distance s_k from c_k (isolated
// points when c_k is off the axis); `live` when they exist, `crossed` when
// they are two distinct points (S_k cuts the circle).  b and cos/sin(phi)
// are kept for the error bound.
struct VxPts {
    double v0[3], v1[3];
    double b, cphi, sphi;
    bool live, crossed;
};

__device__ inline VxPts vertex_points(double4 oR, double4 n, const VxAxis &g) {
#pragma clang fp contract(off)
    VxPts r;
    const double R = oR.w;
    r.live = false;
    r.crossed = false;
    r.b = r.cphi = r.sphi = 0.0;
    for (int a = 0; a < 3; ++a) r.v0[a] = r.v1[a] = 0.0;
    const double b = sqrt(g.b2);
    if (b > 1e-12 * (sqrt(g.ww) + R)) {  // c_k off the axis: isolated points
        const double cphi = g.num / (2.0 * R * b);
        if (cphi >= -1.0 && cphi <= 1.0) {
            r.live = true;
            r.crossed = cphi > -1.0 && cphi < 1.0;
            const double sphi = sqrt(fmax(0.0, 1.0 - cphi * cphi));
            const double ex = g.px / b, ey = g.py / b, ez = g.pz / b;
            const double fx = n.y * ez - n.z * ey, fy = n.z * ex - n.x * ez,
                         fz = n.x * ey - n.y * ex;
            r.v0[0] = oR.x + R * (cphi * ex + sphi * fx);
            r.v0[1] = oR.y + R * (cphi * ey + sphi * fy);
            r.v0[2] = oR.z + R * (cphi * ez + sphi * fz);
            r.v1[0] = oR.x + R * (cphi * ex - sphi * fx);
            r.v1[1] = oR.y + R * (cphi * ey - sphi * fy);
            r.v1[2] = oR.z + R * (cphi * ez - sphi * fz);
            r.b = b;
            r.cphi = cphi;
            r.sphi = sphi;
        }
    }
    return r;
}

// A bound on the rounding error of the two positions (first order, safety
// 4), propagated from the circle's bound n.w = e: w = c_k - o within e +
// u|w|, its axial part t within 3 (e + 7u|w|), the in-plane part within
// those plus 6u|t|, so its length b and direction e' = w_perp / b within
// that over b; cos(phi) = (|w|^2 + R^2 - s_k^2) / (2 R b) within the
// numerator's error (2|w| e + 2R e + 4u (|w|^2 + R^2 + s_k^2)) over 2 R b plus
// |cos(phi)| (e / R + db / b + 2u), sin(phi) within min(sqrt(2 dc), |cos| dc /
// sin); the position o + R (cos e' + sin f) adds R times the errors of the
// unit vectors and of the two factors.
__device__ inline double vertex_eps(double4 oR, double4 n, const VxAxis &g, const VxPts &r) {
    const double R = oR.w, b = r.b, cphi = r.cphi, sphi = r.sphi;
    const double ec = n.w, wl = sqrt(g.ww), at = fabs(g.t);
    const double dw = ec + U64 * wl;
    const double dp = dw + 3.0 * (dw + 7.0 * U64 * wl) + 6.0 * U64 * at;
    const double de = 2.0 * dp / b + 4.0 * U64;
    const double df = 2.0 * (de + 6.0 * U64);
    const double dc = (2.0 * wl * dw + 2.0 * R * ec + 4.0 * U64 * (g.ww + R * R + g.sk * g.sk)) /
                          (2.0 * R * b) +
                      fabs(cphi) * (ec / R + dp / b + 2.0 * U64);
    const double ds =
        (sphi > 0.0 ? fmin(sqrt(2.0 * dc), fabs(cphi) * dc / sphi) : sqrt(2.0 * dc)) + U64;
    const double cm = fmax(fabs(oR.x), fmax(fabs(oR.y), fabs(oR.z)));
    return 4.0 * (ec + ec + R * (dc + ds + de + df) + 4.0 * U64 * (cm + R));
}

// Exposure of the points v0 (while ok0) and v1 (while ok1) against i's
// neighbours at cover positions [q0, q1) (0..nst-1 from LDS, the rest from
// global memory), j and k skipped.  The loop is uniform across the wavefront
// and ends when no lane has a live point left.
__device__ inline void vertex_expose(const Mol &m, const VxLds &L, int nb, int nst, int q0, int q1,
                                     int j, int k, const double *v0, const double *v1, bool &ok0,
                                     bool &ok1) {
#pragma clang fp contract(off)
    for (int q2 = q0; q2 < q1; ++q2) {
        if (!__any(ok0 || ok1)) break;
        int l;
        double4 al;
        if (q2 < nst) {
            l = L.nid[q2];
            al = L.nat[q2];
        } else {
            l = m.nbr_cov[nb + q2];
            double4 a = m.atom[l];
            al = make_double4(a.x, a.y, a.z, sq(a.w + m.rho) * (1.0 - VERTEX_TOL));
        }
        if (l == j || l == k) continue;
        double d0 = sq(v0[0] - al.x) + sq(v0[1] - al.y) + sq(v0[2] - al.z);
        double d1 = sq(v1[0] - al.x) + sq(v1[1] - al.y) + sq(v1[2] - al.z);
        ok0 = ok0 && !(d0 < al.w);
        ok1 = ok1 && !(d1 < al.w);
    }
}


// The two points of circle (o, R, n) at distance s_k from c_k and whether
// each is exposed: in no other neighbour's open SAS ball.  `eps` (their
// error bound) only when `want_eps`.
__device__ inline void vertex_pair(const Mol &m, bool act, double4 oR, double4 n, int j, int k,
                                   double4 ak, const VxLds &L, int nb, int ne, int nst,
                                   bool want_eps, bool &crossed, double *v0, double *v1, bool &ok0,
                                   bool &ok1, double &eps) {
    VxPts r;
    VxAxis g;
    if (act) {
        g = vx_axis(m, oR, n, ak);
        r = vertex_points(oR, n, g);
    } else {
        r.live = r.crossed = false;
        for (int a = 0; a < 3; ++a) r.v0[a] = r.v1[a] = 0.0;
    }
    crossed = r.crossed;
    for (int a = 0; a < 3; ++a) {
        v0[a] = r.v0[a];
        v1[a] = r.v1[a];
    }
    ok0 = r.live;
    ok1 = r.live;
    vertex_expose(m, L, nb, nst, 0, ne - nb, j, k, v0, v1, ok0, ok1);
    eps = (want_eps && (ok0 || ok1)) ? vertex_eps(oR, n, g, r) : 0.0;
}

template <bool FILL>
__device__ void vertex_circle(const Mol &m, int c, int c0, int i, int nb, int ne, int nst,
                              const VxLds &L, int ncl, int lane, int *vcnt) {
    // i's neighbour lists and circles come from LDS when they fit (all
    // ne - nb neighbours; ncl >= 0 circles), else from global memory
    const bool asc_lds = ne - nb <= VX_NBR;
    const bool circ_lds = ncl >= 0;
    const int j = circ_lds ? L.cj[c - c0] : m.circ_j[c];
    const double4 oR = circ_lds ? L.coR[c - c0] : m.circ_oR[c];
    const double4 n = circ_lds ? L.cn[c - c0] : m.circ_n[c];
    int count = 0;
    int wv = FILL ? m.vert_off[c] : 0, ev = FILL ? m.vert_off[c + 1] : 0;
    uint32_t lflag = 0;
    // first neighbour above j (the list is ascending and holds j)
    int lo = nb, hi = ne;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if ((asc_lds ? L.nasc[mid - nb] : m.nbr[mid]) <= j) lo = mid + 1;
        else hi = mid;
    }
    for (int base = lo; base < ne; base += WAVE) {
        int q = base + lane;
        const bool act = q < ne;
        const int k = act ? (asc_lds ? L.nasc[q - nb] : m.nbr[q]) : -1;
        const double4 ak = act ? (asc_lds ? L.natasc[q - nb] : m.atom[k])
                               : make_double4(0.0, 0.0, 0.0, 0.0);
        bool crossed, ok0, ok1;
        double v0[3], v1[3], veps;
        vertex_pair(m, act, oR, n, j, k, ak, L, nb, ne, nst, FILL, crossed, v0, v1, ok0, ok1,
                    veps);
        const double v0x = v0[0], v0y = v0[1], v0z = v0[2], v1x = v1[0], v1y = v1[1], v1z = v1[2];
        unsigned long long b0 = __ballot(ok0), b1 = __ballot(ok1);
        if (FILL) {
            // lane order, "+" before "-" within a lane
            int before = __popcll(b0 & ((1ull << lane) - 1ull)) + __popcll(b1 & ((1ull << lane) - 1ull));
            int p0 = wv + count + before;
            int p1 = p0 + (ok0 ? 1 : 0);
            if (ok0 && fill_ok(m, p0, ev)) {
                m.vert_p[p0] = make_double4(v0x, v0y, v0z, veps);
                m.vert_ijks[p0] = make_int4(i, j, k, 1);
            }
            if (ok1 && fill_ok(m, p1, ev)) {
                m.vert_p[p1] = make_double4(v1x, v1y, v1z, veps);
                m.vert_ijks[p1] = make_int4(i, j, k, -1);
            }
        } else {
            bool anyx = ok0 || ok1;
            uint32_t f = (crossed ? CF_CROSSED : 0u) | (anyx ? CF_EXPOSED_VERTEX : 0u);
            if (f) {
                lflag |= f;
                int cik = -1;
                if (circ_lds) {
                    int a = 0, b = ncl - 1;
                    while (a <= b) {
                        int mid = (a + b) >> 1;
                        int v = L.cj[mid];
                        if (v == k) {
                            cik = m.circ_off[i] + mid;
                            break;
                        }
                        if (v < k) a = mid + 1;
                        else b = mid - 1;
                    }
                } else {
                    cik = find_circle(m, i, k);
                }
                int cjk = find_circle(m, j, k);
                if (cik >= 0) atomicOr(&m.cflag[cik], f);
                if (cjk >= 0) atomicOr(&m.cflag[cjk], f);
            }
            if (anyx) atomicOr(&m.aflag[k], AF_EXPOSED_VERTEX);
        }
        count += __popcll(b0) + __popcll(b1);
    }
    if (!FILL) {
        // reduce the circle's own flags over the wavefront
        uint32_t f = 0;
        if (__any(lflag & CF_CROSSED)) f |= CF_CROSSED;
        if (__any(lflag & CF_EXPOSED_VERTEX)) f |= CF_EXPOSED_VERTEX;
        if (lane == 0) {
            vcnt[c] = count;
            if (f) atomicOr(&m.cflag[c], f);
            if (f & CF_EXPOSED_VERTEX) {
                atomicOr(&m.aflag[i], AF_EXPOSED_VERTEX);
                atomicOr(&m.aflag[j], AF_EXPOSED_VERTEX);
            }
        }
    }
}

// Pair t of the flattened (circle, k) list of the count pass: circle cc (its
// partner at ascending position pj[cc]) and k's ascending position p.
__device__ inline void vx_pair_of(int t, int ncl, const int *poff, const int *pj, int &cc, int &p) {
    int lo = 0, hi = ncl;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (poff[mid + 1] <= t) lo = mid + 1;
        else hi = mid;
    }
    cc = lo;
    p = pj[cc] + 1 + (t - poff[cc]);
}

// Flags f on the three circles of triple (i, j, k): (i, j) and (i, k) are
// i's own circles (flags gathered in LDS), (j, k) is looked up globally.
__device__ inline void vx_flag_pair(const Mol &m, const VxLds &L, int ncl, uint32_t *fl, int cc,
                                    int j, int k, uint32_t f) {
    atomicOr(&fl[cc], f);
    int a = 0, b = ncl - 1;
    while (a <= b) {
        int mid = (a + b) >> 1;
        int v = L.cj[mid];
        if (v == k) {
            atomicOr(&fl[mid], f);
            break;
        }
        if (v < k) a = mid + 1;
        else b = mid - 1;
    }
    const int cjk = find_circle(m, j, k);
    if (cjk >= 0) atomicOr(&m.cflag[cjk], f);
}

// One workgroup per atom i, one wavefront per circle (i, j) of i; i's
// neighbours (cover order) are staged in LDS for the exposure tests.
// Seven waves per SIMD (72 VGPRs, a few spilled; the LDS of seven workgroups
// fits): the kernel waits mostly on dependent loads (29.5 vs 31.1 ms of batch
// build at six waves).
template <bool FILL>
__global__ void __launch_bounds__(VX_WAVES *WAVE) __attribute__((amdgpu_waves_per_eu(7)))
    k_vertex(Seg sg) {
    __shared__ VxLds L;
    __shared__ int pj[VX_NBR], poff[VX_NBR + 1], vc[VX_NBR], scan_lds[VX_WAVES + 1];
    __shared__ uint32_t fl[VX_NBR];
    __shared__ int qitem[2 * VX_WAVES * WAVE], qn;
    SEG_BEGIN(sg);
    int *vcnt = tmp.vcnt;
    const VertexPool &pool = tmp.pool;
    const int i = bid;
    const int c0 = m.circ_off[i], c1 = m.circ_off[i + 1];
    const int nb = m.nbr_off[i], ne = m.nbr_off[i + 1];
    if (c0 == c1) return;  // uniform across the workgroup
    if (FILL && m.vert_off[c0] == m.vert_off[c1]) return;  // no probe position on i's circles
    const int nst = min(VX_NBR, ne - nb);
    // the count pass pooled the positions of an atom whose lists fit in LDS
    if (FILL && pool.use && c1 - c0 <= VX_NBR && ne - nb <= VX_NBR) return;
    const int ncl = c1 - c0 <= VX_NBR ? c1 - c0 : -1;
    // one thread per staged neighbour and circle: every load is issued
    // before the first LDS store, so that their latencies overlap
    static_assert(VX_NBR <= VX_WAVES * WAVE, "one staging round");
    {
        const int q = threadIdx.x;
        const bool qa = q < nst, qc = q < ncl;
        int l = 0, k = 0, cj = 0;
        double4 coR{}, cn{};
        if (qa) {
            l = m.nbr_cov[nb + q];
            k = m.nbr[nb + q];
        }
        if (qc) {
            cj = m.circ_j[c0 + q];
            coR = m.circ_oR[c0 + q];
            cn = m.circ_n[c0 + q];
        }
        double4 al{}, ak{};
        if (qa) {
            al = m.atom[l];
            ak = m.atom[k];
        }
        if (qa) {
            L.nat[q] = make_double4(al.x, al.y, al.z, sq(al.w + m.rho) * (1.0 - VERTEX_TOL));
            L.nid[q] = l;
            L.nasc[q] = k;
            L.natasc[q] = ak;
        }
        if (qc) {
            L.cj[q] = cj;
            L.coR[q] = coR;
            L.cn[q] = cn;
        }
    }
    __syncthreads();
    const int lane = lane_id();
    const int d = ne - nb;
    if (!FILL && ncl >= 0 && d <= VX_NBR) {
        // count pass over the flattened (circle, k) pairs of atom i: circle cc
        // with partner j at ascending position pj[cc] takes the neighbours
        // above it, pairs poff[cc] .. poff[cc + 1]
        int np = 0;
        if ((int)threadIdx.x < ncl) {
            const int j = L.cj[threadIdx.x];
            int lo = 0, hi = d;
            while (lo < hi) {
                int mid = (lo + hi) >> 1;
                if (L.nasc[mid] <= j) lo = mid + 1;
                else hi = mid;
            }
            pj[threadIdx.x] = lo - 1;  // the list holds j
            np = d - lo;
            vc[threadIdx.x] = 0;
            fl[threadIdx.x] = 0;
        }
        int total;
        const int off = block_excl_scan<int, VX_WAVES * WAVE>(np, scan_lds, &total);
        if ((int)threadIdx.x < ncl) poff[threadIdx.x] = off;
        if (threadIdx.x == 0) poff[ncl] = total;
        __syncthreads();
        // Two phases: a cheap test drops the pairs whose sphere certainly
        // misses the circle (about two in three) and queues the rest in
        // LDS; the queue, once it holds a workgroup's worth (or the pairs
        // are done), gets the positions, the exposure tests and, for exposed
        // points only, the error bound, with every lane busy.  A dropped pair
        // has no point, so it flags nothing.
        if (threadIdx.x == 0) qn = 0;
        __syncthreads();
        for (int t0 = 0; t0 < total; t0 += VX_WAVES * WAVE) {
            const int t = t0 + (int)threadIdx.x;
            if (t < total) {
                int cc, p;
                vx_pair_of(t, ncl, poff, pj, cc, p);
                const VxAxis g = vx_axis(m, L.coR[cc], L.cn[cc], L.natasc[p]);
                // queued as (circle, k's position), both below VX_NBR
                if (vx_maybe_live(g, L.coR[cc].w)) qitem[atomicAdd(&qn, 1)] = cc | (p << 16);
            }
            __syncthreads();
            const int nq = qn;
            if (nq < VX_WAVES * WAVE && t0 + VX_WAVES * WAVE < total) continue;  // uniform
            for (int q0 = 0; q0 < nq; q0 += VX_WAVES * WAVE) {
                const int q = q0 + (int)threadIdx.x;
                const bool act = q < nq;
                int cc = 0, p = 0;
                if (act) {
                    const int it = qitem[q];
                    cc = it & 0xFFFF;
                    p = it >> 16;
                }
                const int j = L.cj[cc], k = act ? L.nasc[p] : -1;
                const double4 oR = L.coR[cc], n = L.cn[cc];
                const VxAxis g = vx_axis(m, oR, n, L.natasc[p]);
                VxPts r = vertex_points(oR, n, g);
                bool ok0 = act && r.live, ok1 = ok0;
                vertex_expose(m, L, nb, nst, 0, d, j, k, r.v0, r.v1, ok0, ok1);
                if (!act) continue;
                const int nx = (ok0 ? 1 : 0) + (ok1 ? 1 : 0);
                // the positions go to the pool (placed and ordered on their
                // circle after the scan)
                if (nx) {
                    const double veps = vertex_eps(oR, n, g, r);
                    const int w = atomicAdd(pool.count, nx), w1 = w + (ok0 ? 1 : 0);
                    if (ok0 && w < pool.cap) {
                        pool.p[w] = make_double4(r.v0[0], r.v0[1], r.v0[2], veps);
                        pool.id[w] = make_int4(c0 + cc, 0, k, 1);
                    }
                    if (ok1 && w1 < pool.cap) {
                        pool.p[w1] = make_double4(r.v1[0], r.v1[1], r.v1[2], veps);
                        pool.id[w1] = make_int4(c0 + cc, 0, k, -1);
                    }
                    atomicAdd(&vc[cc], nx);
                    atomicOr(&m.aflag[k], AF_EXPOSED_VERTEX);
                }
                const uint32_t f =
                    (r.crossed ? CF_CROSSED : 0u) | (nx ? CF_EXPOSED_VERTEX : 0u);
                if (f) vx_flag_pair(m, L, ncl, fl, cc, j, k, f);
            }
            __syncthreads();
            if (threadIdx.x == 0) qn = 0;
            __syncthreads();
        }
        __syncthreads();
        if ((int)threadIdx.x < ncl) {
            const int c = c0 + threadIdx.x;
            const uint32_t f = fl[threadIdx.x];
            vcnt[c] = vc[threadIdx.x];
            if (f) atomicOr(&m.cflag[c], f);
            if (f & CF_EXPOSED_VERTEX) {
                atomicOr(&m.aflag[i], AF_EXPOSED_VERTEX);
                atomicOr(&m.aflag[L.cj[threadIdx.x]], AF_EXPOSED_VERTEX);
            }
        }
        return;
    }
    // (the count pass leaves this atom's positions to the fill pass)
    if (!FILL && threadIdx.x == 0) atomicAdd(tmp.vx_big, 1);
    for (int c = c0 + threadIdx.x / WAVE; c < c1; c += VX_WAVES) {
        if (FILL && m.vert_off[c + 1] == m.vert_off[c]) continue;  // no probe position here
        vertex_circle<FILL>(m, c, c0, i, nb, ne, nst, L, ncl, lane, vcnt);
    }
}

// A circle that no other sphere cuts is wholly inside or wholly outside each
// other SAS ball, so one test point decides whether it is admissible.
__global__ void k_circle_free(Seg sg) {
    SEG_BEGIN(sg);
    (void)tmp;
    int c = bid * blockDim.x + threadIdx.x;
    if (c >= m.ncirc) return;
    if (m.cflag[c] & CF_CROSSED) return;
    int i = m.circ_i[c], j = m.circ_j[c];
    double4 oR = m.circ_oR[c];
    double4 n = m.circ_n[c];
    double ux, uy, uz;
    perp_unit(n.x, n.y, n.z, ux, uy, uz);
    double qx = oR.x + oR.w * ux, qy = oR.y + oR.w * uy, qz = oR.z + oR.w * uz;
    for (int q = m.nbr_off[i]; q < m.nbr_off[i + 1]; ++q) {
        int l = m.nbr_cov[q];
        if (l == j) continue;
        double4 al = m.atom[l];
        double sl = al.w + m.rho;
        double dx = qx - al.x, dy = qy - al.y, dz = qz - al.z;
        if (dx * dx + dy * dy + dz * dz < sl * sl) return;
    }
    atomicOr(&m.cflag[c], CF_EXPOSED_FREE);
    atomicOr(&m.aflag[i], AF_EXPOSED_CIRCLE);
    atomicOr(&m.aflag[j], AF_EXPOSED_CIRCLE);
}

// Per atom: the face flag.
//   A face has an admissible point iff it carries an admissible
//   three-sphere point or admissible crossing-free circle, or it has no
//   circle at all and lies in no other ball (an isolated sphere).
__global__ void k_atom_features(Seg sg) {
    SEG_BEGIN(sg);
    int *face_cnt = tmp.face_cnt;
    int i = bid * blockDim.x + threadIdx.x;
    if (i >= m.n) return;
    uint32_t f = m.aflag[i];
    bool face = (f & (AF_EXPOSED_VERTEX | AF_EXPOSED_CIRCLE)) ||
                (m.circ_any[i] == 0 && !(f & AF_CONTAINED));
    if (face) m.aflag[i] = f | AF_FACE;
    face_cnt[i] = face ? 1 : 0;
}

// ------------------------------------------------------ exposed feature lists

__global__ void k_face_list(Seg sg) {
    SEG_BEGIN(sg);
    (void)tmp;
    int i = bid * blockDim.x + threadIdx.x;
    if (i >= m.n) return;
    if (!(m.aflag[i] & AF_FACE)) return;
    int f = m.face_off_atom[i];
    m.face_atom[f] = i;
}

constexpr int FC_WAVES = 4;
constexpr int CUT_CAPS = 128;  // cuts of one face tested for containment in LDS
constexpr int EC_CAPS = 64;    // cuts of one circle tested for containment in LDS

// The set of directions a cut (v, tau) rejects, {u : u . v > tau} on the unit
// sphere of directions (faces) or circle of in-plane directions (circles),
// is the open cap (arc) around v / |v| of angular radius theta, cos theta =
// tau / |v|.  A cut whose cap lies inside another cut's cap rejects nothing
// that the other does not, so it can be dropped without changing any
// admissibility test: cap k lies inside cap l when the angle alpha between
// their axes satisfies alpha + theta_k < theta_l, i.e. theta_l > theta_k and
// cos alpha > cos(theta_l - theta_k) = c_l c_k + s_l s_k.  It is dropped only
// with a margin of 1e-9 on that cosine (an angle gap of at least 1e-9 rad, far
// above the rounding of the cosines, about 1e-15), so a direction near cap
// k's rim lies inside cap l by that gap and its test against l is decided
// with certainty.  Equal caps are both kept.
struct Cap {
    double ax, ay, az, c, s;
};

__device__ inline Cap cut_cap(double4 v) {
    Cap k;
    const double d = sqrt(v.x * v.x + v.y * v.y + v.z * v.z);
    k.ax = v.x / d;
    k.ay = v.y / d;
    k.az = v.z / d;
    k.c = fmin(1.0, fmax(-1.0, v.w / d));
    k.s = sqrt(fmax(0.0, 1.0 - k.c * k.c));
    return k;
}

__device__ inline bool cap_inside(const Cap &k, const Cap &l) {
    if (!(l.c < k.c)) return false;  // theta_l > theta_k
    const double ca = k.ax * l.ax + k.ay * l.ay + k.az * l.az;
    return ca - (l.c * k.c + l.s * k.s) > 1e-9;
}

// Per wavefront: the caps of one surface's candidate cuts in LDS; lane q of a
// pass asks whether cut q is inside another one.
template <int N>
struct CapLds {
    double ax[N], ay[N], az[N], c[N], s[N];
};

template <int N>
__device__ inline void cap_put(CapLds<N> &L, int q, const Cap &k) {
    L.ax[q] = k.ax;
    L.ay[q] = k.ay;
    L.az[q] = k.az;
    L.c[q] = k.c;
    L.s[q] = k.s;
}

// Whether cut q (of n staged, lane-varying q) lies inside another staged cut;
// the loop over the others is uniform across the wavefront.
template <int N>
__device__ inline bool cap_redundant(const CapLds<N> &L, int n, int q, bool act) {
    bool red = false;
    Cap k;
    if (act) {
        k.ax = L.ax[q];
        k.ay = L.ay[q];
        k.az = L.az[q];
        k.c = L.c[q];
        k.s = L.s[q];
    }
    for (int l = 0; l < n; ++l) {
        if (!__any(act && !red)) break;
        const Cap o = {L.ax[l], L.ay[l], L.az[l], L.c[l], L.s[l]};
        if (act && !red && l != q && cap_inside(k, o)) red = true;
    }
    return red;
}

// Face cut lists: one wavefront per exposed face, the cuts of its atom's
// neighbours (cover order) without those inside another one (faces with more
// than CUT_CAPS neighbours keep every cut).  Count pass (cut_cnt) and fill
// pass, with the same decisions.
template <bool FILL>
__global__ void __launch_bounds__(FC_WAVES *WAVE) k_face_cuts(Seg sg) {
    __shared__ CapLds<CUT_CAPS> caps[FC_WAVES];
    SEG_BEGIN(sg);
    int *cut_cnt = tmp.fcut_cnt;
    const int wv = threadIdx.x / WAVE;
    int f = bid * FC_WAVES + wv;
    if (f >= m.nface) return;  // uniform across the wavefront
    const int lane = lane_id();
    int i = m.face_atom[f];
    double4 ai = m.atom[i];
    double si = ai.w + m.rho;
    int nb = m.nbr_off[i], ne = m.nbr_off[i + 1];
    const int n = ne - nb;
    const bool filt = n <= CUT_CAPS;
    CapLds<CUT_CAPS> &L = caps[wv];
    auto cut_of = [&](int q) {
        double4 ak = m.atom[m.nbr_cov[nb + q]];
        double sk = ak.w + m.rho;
        double vx = ak.x - ai.x, vy = ak.y - ai.y, vz = ak.z - ai.z;
        double d2 = vx * vx + vy * vy + vz * vz;
        return make_double4(vx, vy, vz, (si * si + d2 - sk * sk) / (2.0 * si));
    };
    if (filt && !FILL) {  // (the fill pass reads the count pass's decisions)
        for (int q = lane; q < n; q += WAVE) cap_put(L, q, cut_cap(cut_of(q)));
        wave_sync();
    }
    int w = FILL ? m.face_cut_off[f] : 0, we = FILL ? m.face_cut_off[f + 1] : 0;
    int cnt = 0;
    static_assert(CUT_CAPS <= 2 * WAVE, "two keep words per face");
    for (int base = 0; base < n; base += WAVE) {
        const int q = base + lane;
        const bool act = q < n;
        bool keep;
        if (FILL && filt)  // as the count pass found
            keep = act && ((tmp.fcut_keep[2LL * f + base / WAVE] >> lane) & 1ull);
        else
            keep = act && !(filt && cap_redundant(L, n, q, act));
        const unsigned long long bm = __ballot(keep);
        if (!FILL && filt && lane == 0) tmp.fcut_keep[2LL * f + base / WAVE] = bm;
        if (FILL && keep) {
            const int p = w + cnt + mask_prefix(bm);
            if (fill_ok(m, p, we)) m.face_cut[p] = cut_of(q);
        }
        cnt += __popcll(bm);
    }
    if (!FILL && lane == 0) cut_cnt[f] = cnt;
}

// Exposed circles: a 0/1 flag per circle (scanned into positions), the id
// list, then per exposed circle the neighbours of its owner that reach the
// circle (distance from c_k to the circle below s_k), one wavefront per circle.
__global__ void k_ec_flag(Seg sg) {
    SEG_BEGIN(sg);
    int *ecf = tmp.ecf;
    int c = bid * blockDim.x + threadIdx.x;
    if (c >= m.ncirc) return;
    ecf[c] = (m.cflag[c] & CF_EXPOSED) ? 1 : 0;
}

__global__ void k_ec_ids(Seg sg) {
    SEG_BEGIN(sg);
    const int *ec_pos = tmp.ec_pos;
    int c = bid * blockDim.x + threadIdx.x;
    if (c >= m.ncirc) return;
    if (m.cflag[c] & CF_EXPOSED) m.ec_circ[ec_pos[c]] = c;
}

constexpr int EC_WAVES = 4;

// Exposed-circle cut lists: one wavefront per exposed circle, the in-plane
// cuts of its owner's neighbours that reach the circle, without those whose
// arc lies inside another one's (the cap test above on in-plane directions;
// circles with more than EC_CAPS reaching neighbours keep every cut).
template <bool FILL>
__global__ void __launch_bounds__(EC_WAVES *WAVE) k_ec_cuts(Seg sg) {
    __shared__ CapLds<EC_CAPS> caps[EC_WAVES];
    __shared__ double4 cuts[EC_WAVES][EC_CAPS];
    SEG_BEGIN(sg);
    int *cut_cnt = tmp.eccut_cnt;
    const int wv = threadIdx.x / WAVE;
    int e = bid * EC_WAVES + wv;
    if (e >= m.nec) return;  // uniform across the wavefront
    const int lane = lane_id();
    int c = m.ec_circ[e];
    int i = m.circ_i[c], j = m.circ_j[c];
    double4 oR = m.circ_oR[c];
    double4 n = m.circ_n[c];
    double R = oR.w;
    CapLds<EC_CAPS> &L = caps[wv];
    // the reaching neighbours' cuts, in cover order (staged while they fit)
    int nin = 0;
    for (int base = m.nbr_off[i]; base < m.nbr_off[i + 1]; base += WAVE) {
        int q = base + lane;
        bool in = false;
        double4 cut = make_double4(0, 0, 0, 0);
        if (q < m.nbr_off[i + 1]) {
            int k = m.nbr_cov[q];
            if (k != j) {
                double4 ak = m.atom[k];
                double sk = ak.w + m.rho;
                double wx = ak.x - oR.x, wy = ak.y - oR.y, wz = ak.z - oR.z;
                double t = wx * n.x + wy * n.y + wz * n.z;
                double ux = wx - t * n.x, uy = wy - t * n.y, uz = wz - t * n.z;
                double b = sqrt(ux * ux + uy * uy + uz * uz);
                in = t * t + sq(b - R) < sq(sk + LIST_SLACK);
                double ww = wx * wx + wy * wy + wz * wz;
                cut = make_double4(ux, uy, uz, (R * R + ww - sk * sk) / (2.0 * R));
            }
        }
        unsigned long long bm = __ballot(in);
        const int p = nin + mask_prefix(bm);
        if (in && p < EC_CAPS) {
            cuts[wv][p] = cut;
            if (!FILL) cap_put(L, p, cut_cap(cut));
        }
        nin += __popcll(bm);
    }
    wave_sync();
    int w = FILL ? m.ec_cut_off[e] : 0, we = FILL ? m.ec_cut_off[e + 1] : 0;
    int cnt = 0;
    static_assert(EC_CAPS <= WAVE, "one keep word per circle");
    if (nin <= EC_CAPS) {
        for (int base = 0; base < nin; base += WAVE) {
            const int q = base + lane;
            const bool act = q < nin;
            const bool keep = act && (FILL ? ((tmp.eccut_keep[e] >> lane) & 1ull)  // as counted
                                           : !cap_redundant(L, nin, q, act));
            const unsigned long long bm = __ballot(keep);
            if (!FILL && lane == 0) tmp.eccut_keep[e] = bm;
            if (FILL && keep) {
                const int p = w + cnt + mask_prefix(bm);
                if (fill_ok(m, p, we)) m.ec_cut[p] = cuts[wv][q];
            }
            cnt += __popcll(bm);
        }
    } else {
        // too many to stage: every reaching cut, as found
        for (int base = m.nbr_off[i]; base < m.nbr_off[i + 1]; base += WAVE) {
            int q = base + lane;
            bool in = false;
            double4 cut = make_double4(0, 0, 0, 0);
            if (q < m.nbr_off[i + 1]) {
                int k = m.nbr_cov[q];
                if (k != j) {
                    double4 ak = m.atom[k];
                    double sk = ak.w + m.rho;
                    double wx = ak.x - oR.x, wy = ak.y - oR.y, wz = ak.z - oR.z;
                    double t = wx * n.x + wy * n.y + wz * n.z;
                    double ux = wx - t * n.x, uy = wy - t * n.y, uz = wz - t * n.z;
                    double b = sqrt(ux * ux + uy * uy + uz * uz);
                    in = t * t + sq(b - R) < sq(sk + LIST_SLACK);
                    double ww = wx * wx + wy * wy + wz * wz;
                    cut = make_double4(ux, uy, uz, (R * R + ww - sk * sk) / (2.0 * R));
                }
            }
            unsigned long long bm = __ballot(in);
            if (FILL) {
                int p = w + cnt + mask_prefix(bm);
                if (in && fill_ok(m, p, we)) m.ec_cut[p] = cut;
            }
            cnt += __popcll(bm);
        }
    }
    if (!FILL && lane == 0) cut_cnt[e] = cnt;
}

// Per-atom offsets of the circle-ordered exposed-circle and vertex lists.
__global__ void k_feature_off_atom(Seg sg) {
    SEG_BEGIN(sg);
    const int *ec_pos = tmp.ec_pos;
    int i = bid * blockDim.x + threadIdx.x;
    if (i > m.n) return;
    m.vert_off_atom[i] = m.vert_off[m.circ_off[i]];
    m.ec_off_atom[i] = ec_pos[m.circ_off[i]];
}

// ---------------------------------------------------------------- tile lists

// One wavefront per tile.  The tile box spans grid points [T t, T t + T] on
// each axis (one point past the tile, so the box also holds the far ends of
// the edges the tile owns).  Candidates are gathered from the cells that
// overlap the box grown by s_max + rho: the cells of one (y, z) row are
// consecutive, and so are their atoms and features, so each row is one range
// per kind.  Lane r reads row r's ranges; the rows' candidates are then
// taken 64 at a time across the lanes (row-major, ascending within a row)
// and compacted with ballots.
constexpr int TILE_WAVES = 4;

// Row of candidate t: the first row whose inclusive end exceeds t.
__device__ inline int tile_row(const int *incl, int nrow, int t) {
    int lo = 0, hi = nrow - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (incl[mid] <= t) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

constexpr int TILE_KEEP = 192;  // entries of each of a tile's lists the count pass keeps (LDS)
constexpr int TILE_SLOT = 256;  // entries of a tile's pool slot (its four lists together)

template <bool FILL>
__global__ void __launch_bounds__(TILE_WAVES *WAVE) k_tiles(Seg sg) {
    // per wavefront and kind (atoms, exposed circles, vertices): each row's
    // first candidate and inclusive end offset
    __shared__ int rbeg[TILE_WAVES][3][WAVE], rend[TILE_WAVES][3][WAVE];
    // count pass: the first TILE_KEEP entries of the tile's four lists
    __shared__ int keep[FILL ? 1 : TILE_WAVES][4][FILL ? 1 : TILE_KEEP];
    SEG_BEGIN(sg);
    int *cntA = tmp.cA, *cntF = tmp.cF, *cntC = tmp.cC, *cntV = tmp.cV;
    const TilePool &tp = tmp.tp;
    const int wv = threadIdx.x / WAVE;
    int tile = bid * TILE_WAVES + wv;
    if (tile >= m.ntiles) return;  // uniform across the wavefront (no block barriers)
    // the fill pass skips tiles whose lists the count pass pooled and those
    // whose four lists are empty (most of a grid's tiles lie away from the
    // molecule)
    if (FILL && (tp.off[tile] >= 0 ||
                 (m.tA_off[tile] == m.tA_off[tile + 1] && m.tF_off[tile] == m.tF_off[tile + 1] &&
                  m.tC_off[tile] == m.tC_off[tile + 1] && m.tV_off[tile] == m.tV_off[tile + 1])))
        return;
    const int lane = lane_id();
    int t3[3] = {tile % m.tdims[0], (tile / m.tdims[0]) % m.tdims[1],
                 tile / (m.tdims[0] * m.tdims[1])};
    double blo[3], bhi[3];
    int c0[3], c1[3];
    const double grow = m.smax + m.rho + LIST_SLACK;
    for (int a = 0; a < 3; ++a) {
        blo[a] = m.lo[a] + (double)(t3[a] * m.tile) * m.h;
        bhi[a] = m.lo[a] + (double)(t3[a] * m.tile + m.tile) * m.h;
        c0[a] = cell_axis(m, blo[a] - grow, a);
        c1[a] = cell_axis(m, bhi[a] + grow, a);
    }
    int nA = 0, nF = 0, nC = 0, nV = 0;
    int oA = FILL ? m.tA_off[tile] : 0, oF = FILL ? m.tF_off[tile] : 0;
    int oC = FILL ? m.tC_off[tile] : 0, oV = FILL ? m.tV_off[tile] : 0;
    const double rho = m.rho;
    const int ny = c1[1] - c0[1] + 1, nrows = ny * (c1[2] - c0[2] + 1);
    int *ab = rbeg[wv][0], *eb = rbeg[wv][1], *vb = rbeg[wv][2];
    int *ai = rend[wv][0], *ei = rend[wv][1], *vi = rend[wv][2];
    for (int r0 = 0; r0 < nrows; r0 += WAVE) {
        const int nr = min(WAVE, nrows - r0);
        int a0 = 0, a1 = 0, e0 = 0, e1 = 0, v0 = 0, v1 = 0;
        if (lane < nr) {
            const int r = r0 + lane;
            const int crow = m.nc[0] * (c0[1] + r % ny + m.nc[1] * (c0[2] + r / ny));
            a0 = m.cell_start[crow + c0[0]];
            a1 = m.cell_start[crow + c1[0] + 1];
            e0 = m.ec_off_atom[a0];
            e1 = m.ec_off_atom[a1];
            v0 = m.vert_off_atom[a0];
            v1 = m.vert_off_atom[a1];
        }
        const int ia = wave_incl_scan(a1 - a0), ie = wave_incl_scan(e1 - e0),
                  iv = wave_incl_scan(v1 - v0);
        ab[lane] = a0;
        eb[lane] = e0;
        vb[lane] = v0;
        ai[lane] = ia;
        ei[lane] = ie;
        vi[lane] = iv;
        wave_sync();
        const int tA = __shfl(ia, WAVE - 1, WAVE), tE = __shfl(ie, WAVE - 1, WAVE),
                  tV = __shfl(iv, WAVE - 1, WAVE);
        for (int base = 0; base < tA; base += WAVE) {
            const int t = base + lane;
            bool inA = false, inF = false;
            int i = 0;
            if (t < tA) {
                const int r = tile_row(ai, nr, t);
                i = ab[r] + t - (r > 0 ? ai[r - 1] : 0);
                double4 a = m.atom[i];
                double s = a.w + rho;
                double d2 = box_dist2(blo, bhi, a.x, a.y, a.z);
                inA = d2 < sq(s + LIST_SLACK);
                inF = (m.aflag[i] & AF_FACE) && d2 < sq(s + rho + LIST_SLACK);
            }
            unsigned long long bA = __ballot(inA), bF = __ballot(inF);
            if (FILL) {
                int pa = oA + nA + mask_prefix(bA), pf = oF + nF + mask_prefix(bF);
                if (inA && fill_ok(m, pa, m.tA_off[tile + 1])) m.tA[pa] = i;
                if (inF && fill_ok(m, pf, m.tF_off[tile + 1])) m.tF[pf] = m.face_off_atom[i];
            } else {
                const int pa = nA + mask_prefix(bA), pf = nF + mask_prefix(bF);
                if (inA && pa < TILE_KEEP) keep[wv][0][pa] = i;
                if (inF && pf < TILE_KEEP) keep[wv][1][pf] = m.face_off_atom[i];
            }
            nA += __popcll(bA);
            nF += __popcll(bF);
        }
        for (int base = 0; base < tE; base += WAVE) {
            const int t = base + lane;
            bool in = false;
            int e = 0;
            if (t < tE) {
                const int r = tile_row(ei, nr, t);
                e = eb[r] + t - (r > 0 ? ei[r - 1] : 0);
                int ci = m.ec_circ[e];
                double4 oR = m.circ_oR[ci];
                double4 n = m.circ_n[ci];
                double d2 = box_dist2(blo, bhi, oR.x, oR.y, oR.z);
                // signed distance of the box from the circle's plane
                double tmin = 0.0, tmax = 0.0;
                double nv[3] = {n.x, n.y, n.z}, ov[3] = {oR.x, oR.y, oR.z};
                for (int a = 0; a < 3; ++a) {
                    double u0 = nv[a] * (blo[a] - ov[a]), u1 = nv[a] * (bhi[a] - ov[a]);
                    tmin += fmin(u0, u1);
                    tmax += fmax(u0, u1);
                }
                in = d2 < sq(oR.w + rho + LIST_SLACK) && tmin < rho + LIST_SLACK &&
                     tmax > -rho - LIST_SLACK;
            }
            unsigned long long bC = __ballot(in);
            int pc = oC + nC + mask_prefix(bC);
            if (FILL && in && fill_ok(m, pc, m.tC_off[tile + 1])) m.tC[pc] = e;
            if (!FILL && in && pc < TILE_KEEP) keep[wv][2][pc] = e;
            nC += __popcll(bC);
        }
        for (int base = 0; base < tV; base += WAVE) {
            const int t = base + lane;
            bool in = false;
            int v = 0;
            if (t < tV) {
                const int r = tile_row(vi, nr, t);
                v = vb[r] + t - (r > 0 ? vi[r - 1] : 0);
                double4 p = m.vert_p[v];
                in = box_dist2(blo, bhi, p.x, p.y, p.z) < sq(rho + LIST_SLACK);
            }
            unsigned long long bV = __ballot(in);
            int pv = oV + nV + mask_prefix(bV);
            if (FILL && in && fill_ok(m, pv, m.tV_off[tile + 1])) m.tV[pv] = v;
            if (!FILL && in && pv < TILE_KEEP) keep[wv][3][pv] = v;
            nV += __popcll(bV);
        }
        wave_sync();  // the next batch of rows overwrites the offsets
    }
    if (!FILL) {
        if (lane == 0) {
            cntA[tile] = nA;
            cntF[tile] = nF;
            cntC[tile] = nC;
            cntV[tile] = nV;
        }
        // the kept lists go to the tile's slot of the pool (tp.cap entries
        // per tile), or the fill pass rebuilds them
        const int tot = nA + nF + nC + nV;
        const bool kept = nA <= TILE_KEEP && nF <= TILE_KEEP && nC <= TILE_KEEP && nV <= TILE_KEEP;
        const int base = kept && tot <= tp.cap ? tile * tp.cap : -1;
        if (lane == 0) {
            tp.off[tile] = base;
            if (base < 0) atomicOr(tp.unpooled, 1);
        }
        if (base >= 0) {
            wave_sync();
            const int n4[4] = {nA, nF, nC, nV};
            int w = base;
            for (int k = 0; k < 4; ++k) {
                for (int q = lane; q < n4[k]; q += WAVE) tp.pool[w + q] = keep[wv][k][q];
                w += n4[k];
            }
        }
    }
}

// Pooled tile lists to their places: one wavefront per tile.
__global__ void __launch_bounds__(TILE_WAVES *WAVE) k_tiles_place(Seg sg) {
    SEG_BEGIN(sg);
    const TilePool &tp = tmp.tp;
    const int *cA = tmp.cA, *cF = tmp.cF, *cC = tmp.cC, *cV = tmp.cV;
    const int tile = bid * TILE_WAVES + threadIdx.x / WAVE;
    if (tile >= m.ntiles) return;
    const int b = tp.off[tile];
    if (b < 0) return;
    const int lane = lane_id();
    const int n4[4] = {cA[tile], cF[tile], cC[tile], cV[tile]};
    int *dst[4] = {m.tA + m.tA_off[tile], m.tF + m.tF_off[tile], m.tC + m.tC_off[tile],
                   m.tV + m.tV_off[tile]};
    int w = b;
    for (int k = 0; k < 4; ++k) {
        for (int q = lane; q < n4[k]; q += WAVE) dst[k][q] = tp.pool[w + q];
        w += n4[k];
    }
}

// --------------------------------------------------------- vertex export

// Caller ids in ascending order; the side flips with the parity of the sort,
// since (p - c_a) . ((c_b - c_a) x (c_c - c_a)) is antisymmetric in (a, b, c).
__global__ void k_export_vertices(Mol m, double *p, int *atoms, int8_t *sign, long long count) {
    long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (v >= count) return;
    double4 q = m.vert_p[v];
    int4 t = m.vert_ijks[v];
    int a[3] = {m.orig[t.x], m.orig[t.y], m.orig[t.z]};
    int sg = t.w;
    for (int x = 0; x < 2; ++x)
        for (int y = 0; y < 2 - x; ++y)
            if (a[y] > a[y + 1]) {
                int tmp = a[y];
                a[y] = a[y + 1];
                a[y + 1] = tmp;
                sg = -sg;
            }
    p[3 * v] = q.x;
    p[3 * v + 1] = q.y;
    p[3 * v + 2] = q.z;
    atoms[3 * v] = a[0];
    atoms[3 * v + 1] = a[1];
    atoms[3 * v + 2] = a[2];
    sign[v] = (int8_t)sg;
}

// ------------------------------------------------------------------ launchers

hipError_t launch_export_vertices(const Mol &m, double *p, int *atoms, int8_t *sign,
                                  long long count, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_export_vertices, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st,
                       m, p, atoms, sign, count);
    return hipGetLastError();
}

static inline unsigned blocks_for(long long n, int bs) {
    long long b = (n + bs - 1) / bs;
    return (unsigned)(b < 1 ? 1 : b);
}

// Pooled probe positions into their circles' ranges (vcnt[c], the circle's
// count, is consumed as a cursor), then every circle's range ordered as the
// fill pass writes it: ascending k, "+" before "-".
__global__ void k_vertex_place(Seg sg) {
    SEG_BEGIN(sg);
    const VertexPool &pool = tmp.pool;
    int *vcnt = tmp.vcnt;
    const int n = tmp.npool;
    const int q = bid * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const int4 id = pool.id[q];
    const int w = m.vert_off[id.x] + atomicSub(&vcnt[id.x], 1) - 1;
    if (!fill_ok(m, w, m.vert_off[id.x + 1]) || w < m.vert_off[id.x]) return;
    m.vert_p[w] = pool.p[q];
    m.vert_ijks[w] = make_int4(m.circ_i[id.x], m.circ_j[id.x], id.z, id.w);
}

__global__ void k_vertex_order(Seg sg) {
    SEG_BEGIN(sg);
    (void)tmp;
    const int c = bid * blockDim.x + threadIdx.x;
    if (c >= m.ncirc) return;
    const int b = m.vert_off[c], e = m.vert_off[c + 1];
    for (int a = b + 1; a < e; ++a) {
        const double4 p = m.vert_p[a];
        const int4 v = m.vert_ijks[a];
        int q = a - 1;
        while (q >= b) {
            const int4 u = m.vert_ijks[q];
            if (u.z < v.z || (u.z == v.z && u.w > v.w)) break;
            m.vert_p[q + 1] = m.vert_p[q];
            m.vert_ijks[q + 1] = u;
            --q;
        }
        m.vert_p[q + 1] = p;
        m.vert_ijks[q + 1] = v;
    }
}

// ------------------------------------------------------ segmented launches

// Block counts of one molecule for each build kernel (the launchers of a
// build stage add these up over the molecules of a batch).
long long build_blocks(BuildKernel k, const Mol &m, const BuildTmp &t) {
    switch (k) {
    case BK_BOUNDS: return 1;
    case BK_CELL_COUNT: return blocks_for(m.n, 256);
    case BK_CELL_FILL: return blocks_for(m.ncell + 1, 256);
    case BK_CELL_SCATTER: return blocks_for(m.n, 256);
    case BK_CELL_SORT: return blocks_for(m.ncell, CS_WAVES);
    case BK_GATHER: return blocks_for(m.n, 256);
    case BK_NBR: return blocks_for(m.n, NB_WAVES);
    case BK_NBR_SORT: return blocks_for(m.n, NS_WAVES);
    case BK_VERTEX: return m.ncirc > 0 ? m.n : 0;
    case BK_VERTEX_PLACE: return t.pool.use && t.npool > 0 ? blocks_for(t.npool, 256) : 0;
    case BK_VERTEX_ORDER: return m.ncirc > 0 && m.nvert > 0 ? blocks_for(m.ncirc, 256) : 0;
    case BK_CIRCLE_FREE: return m.ncirc > 0 ? blocks_for(m.ncirc, 128) : 0;
    case BK_ATOM_FEATURES: return blocks_for(m.n, 256);
    case BK_EC_FLAG: return m.ncirc > 0 ? blocks_for(m.ncirc, 256) : 0;
    case BK_EC_IDS: return m.ncirc > 0 ? blocks_for(m.ncirc, 256) : 0;
    case BK_FEATURE_OFF: return blocks_for(m.n + 1, 256);
    case BK_FACE_LIST: return blocks_for(m.n, 256);
    case BK_FACE_CUTS: return m.nface > 0 ? blocks_for(m.nface, FC_WAVES) : 0;
    case BK_EC_CUTS: return m.nec > 0 ? blocks_for(m.nec, EC_WAVES) : 0;
    case BK_TILES: return blocks_for(m.ntiles, TILE_WAVES);
    case BK_TILES_FILL: return t.tp_unpooled ? blocks_for(m.ntiles, TILE_WAVES) : 0;
    case BK_TILES_PLACE: return blocks_for(m.ntiles, TILE_WAVES);
    }
    return 0;
}

hipError_t launch_build(BuildKernel k, const Seg &s, long long nblocks, hipStream_t st) {
    if (nblocks <= 0) return hipSuccess;
    const dim3 g((unsigned)nblocks);
    switch (k) {
    case BK_BOUNDS: hipLaunchKernelGGL(k_bounds, g, dim3(256), 0, st, s); break;
    case BK_CELL_COUNT: hipLaunchKernelGGL(k_cell_count, g, dim3(256), 0, st, s); break;
    case BK_CELL_FILL: hipLaunchKernelGGL(k_cell_fill_init, g, dim3(256), 0, st, s); break;
    case BK_CELL_SCATTER: hipLaunchKernelGGL(k_cell_scatter, g, dim3(256), 0, st, s); break;
    case BK_CELL_SORT: hipLaunchKernelGGL(k_cell_sort, g, dim3(CS_WAVES * WAVE), 0, st, s); break;
    case BK_GATHER: hipLaunchKernelGGL(k_gather_atoms, g, dim3(256), 0, st, s); break;
    case BK_NBR: hipLaunchKernelGGL(k_nbr<false>, g, dim3(NB_WAVES * WAVE), 0, st, s); break;
    case BK_NBR_SORT: hipLaunchKernelGGL(k_nbr_sort, g, dim3(NS_WAVES * WAVE), 0, st, s); break;
    case BK_VERTEX: hipLaunchKernelGGL(k_vertex<false>, g, dim3(VX_WAVES * WAVE), 0, st, s); break;
    case BK_VERTEX_PLACE: hipLaunchKernelGGL(k_vertex_place, g, dim3(256), 0, st, s); break;
    case BK_VERTEX_ORDER: hipLaunchKernelGGL(k_vertex_order, g, dim3(256), 0, st, s); break;
    case BK_CIRCLE_FREE: hipLaunchKernelGGL(k_circle_free, g, dim3(128), 0, st, s); break;
    case BK_ATOM_FEATURES: hipLaunchKernelGGL(k_atom_features, g, dim3(256), 0, st, s); break;
    case BK_EC_FLAG: hipLaunchKernelGGL(k_ec_flag, g, dim3(256), 0, st, s); break;
    case BK_EC_IDS: hipLaunchKernelGGL(k_ec_ids, g, dim3(256), 0, st, s); break;
    case BK_FEATURE_OFF: hipLaunchKernelGGL(k_feature_off_atom, g, dim3(256), 0, st, s); break;
    case BK_FACE_LIST: hipLaunchKernelGGL(k_face_list, g, dim3(256), 0, st, s); break;
    case BK_FACE_CUTS: hipLaunchKernelGGL(k_face_cuts<false>, g, dim3(FC_WAVES * WAVE), 0, st, s); break;
    case BK_EC_CUTS: hipLaunchKernelGGL(k_ec_cuts<false>, g, dim3(EC_WAVES * WAVE), 0, st, s); break;
    case BK_TILES: hipLaunchKernelGGL(k_tiles<false>, g, dim3(TILE_WAVES * WAVE), 0, st, s); break;
    case BK_TILES_FILL: hipLaunchKernelGGL(k_tiles<true>, g, dim3(TILE_WAVES * WAVE), 0, st, s); break;
    case BK_TILES_PLACE: hipLaunchKernelGGL(k_tiles_place, g, dim3(TILE_WAVES * WAVE), 0, st, s); break;
    }
    return hipGetLastError();
}

// The fill passes (second pass of a count/fill pair).
hipError_t launch_build_fill(BuildKernel k, const Seg &s, long long nblocks, hipStream_t st) {
    if (nblocks <= 0) return hipSuccess;
    const dim3 g((unsigned)nblocks);
    switch (k) {
    case BK_NBR: hipLaunchKernelGGL(k_nbr<true>, g, dim3(NB_WAVES * WAVE), 0, st, s); break;
    case BK_VERTEX: hipLaunchKernelGGL(k_vertex<true>, g, dim3(VX_WAVES * WAVE), 0, st, s); break;
    case BK_FACE_CUTS: hipLaunchKernelGGL(k_face_cuts<true>, g, dim3(FC_WAVES * WAVE), 0, st, s); break;
    case BK_EC_CUTS: hipLaunchKernelGGL(k_ec_cuts<true>, g, dim3(EC_WAVES * WAVE), 0, st, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int tile_keep_max() { return TILE_SLOT; }

}  // namespace eses
