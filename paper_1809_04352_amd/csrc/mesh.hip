// Triangle mesh of the surface from the labels and the crossing records, and
// the surface's area and enclosed volume (section 2.2: the Eulerian output is
// turned into a triangle mesh by marching cubes; the appendix table reports
// each complex's surface area and volume).
//
// Every cube of eight axis-adjacent grid points with mixed labels is cut by
// the triangles of its configuration (mc_table.h); a triangle's corners are
// the crossing points of three of the cube's edges, p = s + (1 - lambda) h e
// for the edge's record (eq. 4), found by binary search of the edge key among
// the molecule's sorted records.  Area: the sum of the triangles' areas.
// Volume: the divergence theorem over the closed, outward-oriented mesh,
// sum of det(v0, v1, v2) / 6 with the vertices taken relative to the grid
// origin.
#include <algorithm>
#include <array>
#include <mutex>
#include <set>
#include <vector>

#include "eses_device.h"
#include "launch.h"
#include "mc_table.h"

namespace eses {

// ------------------------------------------------------------ case table

namespace {

void corner_xyz(int c, int xyz[3]) {
    xyz[0] = c & 1;
    xyz[1] = (c >> 1) & 1;
    xyz[2] = (c >> 2) & 1;
}

// The edge joining two corners that differ in one coordinate.
int edge_of(int c0, int c1) {
    int p[3], q[3];
    corner_xyz(c0, p);
    corner_xyz(c1, q);
    int a = 0;
    while (p[a] == q[a]) ++a;
    int r = 0, bit = 0;
    for (int b = 0; b < 3; ++b) {
        if (b == a) continue;
        r |= p[b] << bit;
        ++bit;
    }
    return 4 * a + r;
}

McTable build_table() {
    McTable t{};
    for (int cfg = 0; cfg < 256; ++cfg) {
        auto in = [&](int c) { return (cfg >> c) & 1; };
        // segments on the six faces (pairs of edges)
        std::vector<std::pair<int, int>> seg;
        for (int a = 0; a < 3; ++a)
            for (int side = 0; side < 2; ++side) {
                const int b = (a + 1) % 3, c = (a + 2) % 3;
                int cor[4];
                const int uv[4][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}};
                for (int q = 0; q < 4; ++q) {
                    int xyz[3];
                    xyz[a] = side;
                    xyz[b] = uv[q][0];
                    xyz[c] = uv[q][1];
                    cor[q] = xyz[0] + 2 * xyz[1] + 4 * xyz[2];
                }
                int cross[4], nc = 0;  // face edges q -> q+1 that cross
                for (int q = 0; q < 4; ++q)
                    if (in(cor[q]) != in(cor[(q + 1) % 4])) cross[nc++] = q;
                if (nc == 2) {
                    seg.push_back({edge_of(cor[cross[0]], cor[(cross[0] + 1) % 4]),
                                   edge_of(cor[cross[1]], cor[(cross[1] + 1) % 4])});
                } else if (nc == 4) {
                    // cut off each inside corner: its two face edges
                    for (int q = 0; q < 4; ++q)
                        if (in(cor[q]))
                            seg.push_back({edge_of(cor[(q + 3) % 4], cor[q]),
                                           edge_of(cor[q], cor[(q + 1) % 4])});
                }
            }
        // loops
        std::vector<std::vector<int>> adj(12);
        for (auto &s : seg) {
            adj[s.first].push_back(s.second);
            adj[s.second].push_back(s.first);
        }
        bool seen[12] = {false};
        int nt = 0;
        for (int e0 = 0; e0 < 12; ++e0) {
            if (seen[e0] || adj[e0].empty()) continue;
            std::vector<int> loop{e0};
            seen[e0] = true;
            int prev = -1, cur = e0;
            for (;;) {
                int nxt = -1;
                for (int v : adj[cur])
                    if (v != prev && (!seen[v] || (v == e0 && loop.size() > 2))) {
                        nxt = v;
                        break;
                    }
                if (nxt < 0 || nxt == e0) break;
                loop.push_back(nxt);
                seen[nxt] = true;
                prev = cur;
                cur = nxt;
            }
            // orientation: Newell normal of the edge midpoints against the
            // inside -> outside directions of the loop's edges
            double N[3] = {0, 0, 0}, D[3] = {0, 0, 0};
            const int L = (int)loop.size();
            std::vector<std::array<double, 3>> mid(L);
            for (int q = 0; q < L; ++q) {
                int p0[3], p1[3];
                corner_xyz(mc_edge_corner(loop[q], 0), p0);
                corner_xyz(mc_edge_corner(loop[q], 1), p1);
                const bool in0 = in(mc_edge_corner(loop[q], 0));
                for (int k = 0; k < 3; ++k) {
                    mid[q][k] = 0.5 * (p0[k] + p1[k]);
                    D[k] += in0 ? (p1[k] - p0[k]) : (p0[k] - p1[k]);
                }
            }
            for (int q = 0; q < L; ++q) {
                const auto &u = mid[q], &v = mid[(q + 1) % L];
                N[0] += (u[1] - v[1]) * (u[2] + v[2]);
                N[1] += (u[2] - v[2]) * (u[0] + v[0]);
                N[2] += (u[0] - v[0]) * (u[1] + v[1]);
            }
            if (N[0] * D[0] + N[1] * D[1] + N[2] * D[2] < 0) std::reverse(loop.begin(), loop.end());
            const int s = (int)(std::min_element(loop.begin(), loop.end()) - loop.begin());
            std::rotate(loop.begin(), loop.begin() + s, loop.end());
            for (int q = 1; q + 1 < L; ++q) {
                t.tri[cfg][nt][0] = (int8_t)loop[0];
                t.tri[cfg][nt][1] = (int8_t)loop[q];
                t.tri[cfg][nt][2] = (int8_t)loop[q + 1];
                ++nt;
            }
        }
        t.ntri[cfg] = (uint8_t)nt;
    }
    return t;
}

}  // namespace

const McTable &mc_table() {
    static const McTable t = build_table();
    return t;
}

__constant__ uint8_t c_ntri[256];
__constant__ int8_t c_tri[256][12][3];

// The table in each device's constant memory, uploaded once per device.
hipError_t mc_upload() {
    static std::mutex mu;
    static std::set<int> done;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(mu);
    if (done.count(dev)) return hipSuccess;
    const McTable &t = mc_table();
    e = hipMemcpyToSymbol(HIP_SYMBOL(c_ntri), t.ntri, sizeof(t.ntri));
    if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(c_tri), t.tri, sizeof(t.tri));
    if (e == hipSuccess) done.insert(dev);
    return e;
}

// ------------------------------------------------------------- kernels

constexpr int MESH_THREADS = 256;

struct MeshArgs {
    const uint8_t *L;
    const long long *key;
    const double *lam;
    long long nrec;
    int nx, ny, nz;
    double h;
    double lo[3];
};

// Record index of an edge key (-1 if absent).
__device__ inline long long find_key(const long long *key, long long n, long long k) {
    long long a = 0, b = n - 1;
    while (a <= b) {
        const long long m = (a + b) >> 1;
        const long long v = key[m];
        if (v == k) return m;
        if (v < k) a = m + 1;
        else b = m - 1;
    }
    return -1;
}

// Configuration of cube q (lower corner (i, j, k)); 0 for the last layer.
__device__ inline int cube_config(const MeshArgs &A, long long q, int &i, int &j, int &k) {
    const long long nxy = (long long)A.nx * A.ny;
    i = (int)(q % A.nx);
    j = (int)((q / A.nx) % A.ny);
    k = (int)(q / nxy);
    if (i + 1 >= A.nx || j + 1 >= A.ny || k + 1 >= A.nz) return 0;
    int cfg = 0;
    for (int c = 0; c < 8; ++c) {
        const long long g = (long long)(i + (c & 1)) + A.nx * ((long long)(j + ((c >> 1) & 1)) +
                                                               (long long)A.ny * (k + ((c >> 2) & 1)));
        cfg |= (A.L[g] & 1) << c;
    }
    return cfg;
}

// Record and position (relative to the grid origin) of cube edge e.
__device__ inline long long edge_point(const MeshArgs &A, int i, int j, int k, int e, double p[3]) {
    const int a = e >> 2, r = e & 3;
    int off[3] = {0, 0, 0};
    int bit = 0;
    for (int b = 0; b < 3; ++b) {
        if (b == a) continue;
        off[b] = (r >> bit) & 1;
        ++bit;
    }
    const int ii = i + off[0], jj = j + off[1], kk = k + off[2];
    const long long g = (long long)ii + A.nx * ((long long)jj + (long long)A.ny * kk);
    const long long rec = find_key(A.key, A.nrec, 3 * g + a);
    const int ijk[3] = {ii, jj, kk};
    for (int b = 0; b < 3; ++b) {
        // fl(lo + fl(i h)) - lo, then the offset along the edge
        const double x = grid_coord(A.lo[b], A.h, ijk[b]) - A.lo[b];
        p[b] = x;
    }
    if (rec >= 0) p[a] += (1.0 - A.lam[rec]) * A.h;
    return rec;
}

// Per cube: its triangles' area and volume terms (and count); per block the
// sums go to out[2 block .. 2 block + 1] (area, volume) and counts[block]
// (triangles).  Edges without
// a record (a configuration the records do not cover) are counted in bad.
__global__ void __launch_bounds__(MESH_THREADS) k_mesh_count(MeshArgs A, long long ncube,
                                                            double *out, int *counts, int *bad) {
    __shared__ double sa[MESH_THREADS / WAVE], sv[MESH_THREADS / WAVE];
    __shared__ int sc[MESH_THREADS / WAVE];
    const long long q = blockIdx.x * (long long)MESH_THREADS + threadIdx.x;
    double area = 0.0, vol = 0.0;
    int nt = 0;
    if (q < ncube) {
        int i, j, k;
        const int cfg = cube_config(A, q, i, j, k);
        nt = c_ntri[cfg];
        for (int t = 0; t < nt; ++t) {
            double v[3][3];
            for (int c = 0; c < 3; ++c)
                if (edge_point(A, i, j, k, c_tri[cfg][t][c], v[c]) < 0) atomicAdd(bad, 1);
            const double ux = v[1][0] - v[0][0], uy = v[1][1] - v[0][1], uz = v[1][2] - v[0][2];
            const double wx = v[2][0] - v[0][0], wy = v[2][1] - v[0][1], wz = v[2][2] - v[0][2];
            const double cx = uy * wz - uz * wy, cy = uz * wx - ux * wz, cz = ux * wy - uy * wx;
            area += 0.5 * sqrt(cx * cx + cy * cy + cz * cz);
            vol += (v[0][0] * (v[1][1] * v[2][2] - v[1][2] * v[2][1]) -
                    v[0][1] * (v[1][0] * v[2][2] - v[1][2] * v[2][0]) +
                    v[0][2] * (v[1][0] * v[2][1] - v[1][1] * v[2][0])) /
                   6.0;
        }
    }
    for (int d = WAVE / 2; d > 0; d >>= 1) {
        area += __shfl_down(area, d, WAVE);
        vol += __shfl_down(vol, d, WAVE);
        nt += __shfl_down(nt, d, WAVE);
    }
    const int w = threadIdx.x / WAVE;
    if (lane_id() == 0) {
        sa[w] = area;
        sv[w] = vol;
        sc[w] = nt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, v = 0.0;
        int c = 0;
        for (int x = 0; x < MESH_THREADS / WAVE; ++x) {
            a += sa[x];
            v += sv[x];
            c += sc[x];
        }
        out[2 * blockIdx.x] = a;  // block sums, reduced in a fixed order below
        out[2 * blockIdx.x + 1] = v;
        counts[blockIdx.x] = c;
    }
}

// The block sums of area and volume added in a fixed order (the result does
// not depend on the order blocks ran in): sum[0..1].
__global__ void __launch_bounds__(MESH_THREADS) k_mesh_reduce(const double *part, long long nb,
                                                             double *sum) {
    __shared__ double sa[MESH_THREADS], sv[MESH_THREADS];
    double a = 0.0, v = 0.0;
    for (long long b = threadIdx.x; b < nb; b += MESH_THREADS) {
        a += part[2 * b];
        v += part[2 * b + 1];
    }
    sa[threadIdx.x] = a;
    sv[threadIdx.x] = v;
    __syncthreads();
    for (int d = MESH_THREADS / 2; d > 0; d >>= 1) {
        if ((int)threadIdx.x < d) {
            sa[threadIdx.x] += sa[threadIdx.x + d];
            sv[threadIdx.x] += sv[threadIdx.x + d];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        sum[0] = sa[0];
        sum[1] = sv[0];
    }
}

// Triangles (record indices of their three corners), at the block offsets
// of the count pass; within a block in cube order.
__global__ void __launch_bounds__(MESH_THREADS) k_mesh_write(MeshArgs A, long long ncube,
                                                            const long long *boff, long long cap,
                                                            int *tri) {
    __shared__ int scan[MESH_THREADS / WAVE + 1];
    const long long q = blockIdx.x * (long long)MESH_THREADS + threadIdx.x;
    int i = 0, j = 0, k = 0, cfg = 0;
    if (q < ncube) cfg = cube_config(A, q, i, j, k);
    const int nt = c_ntri[cfg];
    int total;
    const int pre = block_excl_scan<int, MESH_THREADS>(nt, scan, &total);
    long long w = boff[blockIdx.x] + pre;
    for (int t = 0; t < nt; ++t, ++w) {
        if (w >= cap) break;
        for (int c = 0; c < 3; ++c) {
            double p[3];
            tri[3 * w + c] = (int)edge_point(A, i, j, k, c_tri[cfg][t][c], p);
        }
    }
}

hipError_t launch_mesh(const Mol &m, const uint8_t *L, const long long *key, const double *lam,
                       long long nrec, double *out, int *counts, int *bad, long long *nblocks,
                       hipStream_t st) {
    hipError_t e = mc_upload();
    if (e != hipSuccess) return e;
    MeshArgs A{L, key, lam, nrec, m.dims[0], m.dims[1], m.dims[2], m.h, {m.lo[0], m.lo[1], m.lo[2]}};
    const long long ncube = m.npts;
    *nblocks = (ncube + MESH_THREADS - 1) / MESH_THREADS;
    hipLaunchKernelGGL(k_mesh_count, dim3((unsigned)*nblocks), dim3(MESH_THREADS), 0, st, A, ncube,
                       out + 2, counts, bad);
    hipLaunchKernelGGL(k_mesh_reduce, dim3(1), dim3(MESH_THREADS), 0, st, out + 2, *nblocks, out);
    return hipGetLastError();
}

hipError_t launch_mesh_write(const Mol &m, const uint8_t *L, const long long *key,
                             const double *lam, long long nrec, const long long *boff,
                             long long cap, int *tri, hipStream_t st) {
    MeshArgs A{L, key, lam, nrec, m.dims[0], m.dims[1], m.dims[2], m.h, {m.lo[0], m.lo[1], m.lo[2]}};
    const long long ncube = m.npts;
    const long long nb = (ncube + MESH_THREADS - 1) / MESH_THREADS;
    hipLaunchKernelGGL(k_mesh_write, dim3((unsigned)nb), dim3(MESH_THREADS), 0, st, A, ncube, boff,
                       cap, tri);
    return hipGetLastError();
}

}  // namespace eses
