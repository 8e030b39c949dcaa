// Host-side launchers of the ESES kernels (one per kernel family).
#pragma once

#include "eses_internal.h"

namespace eses {

// utilities
long long scan_tmp_elems(long long n);
hipError_t scan_i32(const int *in, long long n, int *out, int *tmp, hipStream_t st);
hipError_t scan_i64(const int *in, long long n, long long *out, long long *tmp, hipStream_t st);
// k (<= 4) arrays of length n scanned together (one launch when n is small).
hipError_t scan_i32_multi(const int *const *in, long long n, int *const *out, int k, int *tmp,
                          hipStream_t st);
// Up to 16 device scalars (int, or long long where is64) copied by one kernel
// into host-visible memory `host` (long long each).
struct ReadBack {
    const void *p[16];
    int is64[16];
    int n;
};
hipError_t launch_collect(const ReadBack &rb, long long *host, hipStream_t st);

hipError_t fill_i32(int *p, long long n, int v, hipStream_t st);
hipError_t copy_i32(int *dst, const int *src, long long n, hipStream_t st);
hipError_t fill_u32(uint32_t *p, long long n, uint32_t v, hipStream_t st);

// stage 1
hipError_t launch_bounds(const double *c, const double *r, long long n, double *out, int *bad,
                         hipStream_t st);
hipError_t launch_cell_count(const Mol &m, int *cell_id, int *count, hipStream_t st);
hipError_t launch_cell_scatter(const Mol &m, const int *cell_id, int *fill, int *slot_orig,
                               hipStream_t st);
hipError_t launch_cell_sort_gather(const Mol &m, int *slot_orig, hipStream_t st);
hipError_t launch_nbr(const Mol &m, bool fill, int *nbr_cnt, int *circ_cnt, hipStream_t st);
hipError_t launch_nbr_sort(const Mol &m, hipStream_t st);
// Probe positions found by the count pass of the atoms whose neighbours and
// circles fit in LDS (p: x, y, z, -; id: circle, -, k, sign); count: one
// int, zeroed before the count pass.  When count <= cap after it,
// launch_vertex_place writes them (consuming the per-circle counts vcnt) and
// the fill pass (use = 1) skips those atoms; launch_vertex_order then puts
// every circle's positions in the fill pass's order.
struct VertexPool {
    double4 *p;
    int4 *id;
    int *count;
    int cap;
    int use;
};
hipError_t launch_vertex(const Mol &m, bool fill, int *vcnt, const VertexPool &pool,
                         hipStream_t st);
hipError_t launch_vertex_place(const Mol &m, const VertexPool &pool, int n, int *vcnt,
                               hipStream_t st);
hipError_t launch_vertex_order(const Mol &m, hipStream_t st);
hipError_t launch_circle_free(const Mol &m, hipStream_t st);
hipError_t launch_atom_features(const Mol &m, int *face_cnt, hipStream_t st);
hipError_t launch_ec_flag(const Mol &m, int *ecf, hipStream_t st);
hipError_t launch_ec_ids(const Mol &m, const int *ec_pos, hipStream_t st);
hipError_t launch_face_list(const Mol &m, int *cut_cnt, hipStream_t st);
hipError_t launch_face_cuts(const Mol &m, hipStream_t st);
hipError_t launch_ec_cuts(const Mol &m, bool fill, int *cut_cnt, hipStream_t st);
// Tile lists kept by the count pass: each tile's four lists (atoms, faces,
// circles, probes, in that order) copied into its slot of `pool` (cap ints
// per tile, cap <= tile_keep_max()) at off[t] = t * cap, or off[t] = -1 when
// they do not fit (then *unpooled, zeroed before, is set and the fill pass
// rebuilds that tile).
struct TilePool {
    int *pool, *off, *unpooled;
    int cap;
};
int tile_keep_max();
hipError_t launch_tiles_place(const Mol &m, const TilePool &tp, const int *cA, const int *cF,
                              const int *cC, const int *cV, hipStream_t st);
hipError_t launch_tiles(const Mol &m, bool fill, int *cA, int *cF, int *cC, int *cV,
                        const TilePool &tp, hipStream_t st);

// stage 2
hipError_t launch_classify(const Mol &m, bool fp32, uint8_t *labels, hipStream_t st);
hipError_t launch_units(const Mol *mols_dev, const int *tile_base_dev, int nmols, long long total,
                        int *cls_count, int *cls_fill, int2 *units, hipStream_t st);
int classify_batch_blocks_per_cu(bool fp32);
// (also zeroes every molecule's uncertain-point counter first)
hipError_t launch_classify_batch(const Mol *mols_dev, int nmols, uint8_t *const *labels_dev,
                                 const int2 *units, int nunits, int *head, int nblocks, bool fp32,
                                 hipStream_t st);
// Uncertain-point counters of a batch: zeroed, or gathered into out[nmols].
hipError_t launch_unc_zero(const Mol *mols_dev, int nmols, hipStream_t st);
hipError_t launch_unc_gather(const Mol *mols_dev, int nmols, int *out, hipStream_t st);
// Diagnostic word k (Mol::diag) of every molecule of a batch into out[nmols].
hipError_t launch_diag_gather(const Mol *mols_dev, int nmols, int k, int *out, hipStream_t st);
// labels[idx[q]] = val[q] for q < n.
hipError_t launch_scatter_labels(const long long *idx, const uint8_t *val, int n, uint8_t *labels,
                                 hipStream_t st);
hipError_t launch_classify_work(const Mol &m, unsigned long long *work, hipStream_t st);
hipError_t launch_count_inside(const uint8_t *labels, long long n, unsigned long long *out,
                               hipStream_t st);

// stage 3
// Blocks of the crossing-edge passes (one per EDGE_BLOCK points of a row).
long long edge_detect_blocks(const Mol &m);
hipError_t launch_edge_detect_count(const uint8_t *L, const Mol &m, int *bcount, long long *nblk,
                                    hipStream_t st);
// keys: the first cap crossing edges; tcount: per-tile counts of them; rank:
// each edge's rank within its tile (cap ints).
hipError_t launch_edge_detect_write(const uint8_t *L, const Mol &m, const long long *boff,
                                    long long cap, long long *keys, int *tcount, int *rank,
                                    hipStream_t st);
// Crossing edges grouped by tile (tcount, rank: from the key pass):
// order[] holds, per tile, its edges padded
// to a multiple of the chunk size (edge_order_capacity entries); coff[t] is
// the tile's first chunk and coff[ntiles] the number of chunks.  units
// (edge_units_capacity ints) receives the work list of the root kernel: the
// tile counts per chunk-count class and their fill cursors, the queue
// counter, the number of units and, from EU_LIST on, the tiles with edges,
// the ones with most chunks first.
constexpr int EU_CLASSES = 8;
constexpr int EU_CLASS = 0, EU_FILL = 8, EU_QUEUE = 16, EU_COUNT = 24, EU_LIST = 32;
long long edge_order_capacity(const Mol &m, long long count);
long long edge_units_capacity(const Mol &m);
hipError_t launch_edge_group(const Mol &m, const long long *keys, long long count, int *tcount,
                             int *ccount, int *coff, const int *rank, int *order, int *units,
                             int *tmp, hipStream_t st);
// fallback: count ints; nfallback, overflow: one int each (overflow is set,
// not cleared).
hipError_t launch_edge_roots(const Mol &m, const uint8_t *L, const long long *keys,
                             long long count, const int *order, const int *tcount,
                             const int *coff, int *units, double *lam, double *nrm,
                             uint8_t *ptype, int *patoms, int *fallback, int *nfallback,
                             int *overflow, hipStream_t st);

hipError_t launch_edge_work(const Mol &m, const uint8_t *L, const long long *keys,
                            long long count, const int *order, const int *tcount,
                            const int *coff, int *units, int *fallback, int *nfallback,
                            int *overflow, unsigned long long *work, hipStream_t st);

// One molecule's buffers for the fused root launch of a batch (after its
// crossing edges are grouped): mol indexes the device Mol array; units as
// written by launch_edge_group; nfallback zeroed.
struct EdgeJob {
    const uint8_t *L;
    const long long *keys;
    const int *order, *tcount, *coff, *units;
    double *lam, *nrm;
    uint8_t *ptype;
    int *patoms, *fallback, *nfallback;
    int mol, pad;
};
// Every job's tiles in one persistent launch (jobs in the given order, each
// one's tiles with most chunks first), then the jobs' fallback edges in one
// launch.  prefix: nj + 1 ints of workspace; queue: one int, zeroed;
// overflow: one int, set (not cleared) when an edge has more roots than the
// per-edge lists hold.
hipError_t launch_edge_roots_batch(const Mol *mols, const EdgeJob *jobs, int nj, int *prefix,
                                   int *queue, int *overflow, hipStream_t st);

constexpr int EDGE_WORK_COUNTERS = 16;

// marching-cubes mesh (mesh.hip): per block of cubes, the triangle counts
// (counts[*nblocks]); the area and volume sums into out[0..1] (out holds
// 2 + 2 * blocks doubles: the block sums follow, added in a fixed order);
// records missing for a cut edge counted in *bad.
// The write pass puts the triangles (record indices) at the scanned block
// offsets boff.
hipError_t launch_mesh(const Mol &m, const uint8_t *L, const long long *key, const double *lam,
                       long long nrec, double *out, int *counts, int *bad, long long *nblocks,
                       hipStream_t st);
hipError_t launch_mesh_write(const Mol &m, const uint8_t *L, const long long *key,
                             const double *lam, long long nrec, const long long *boff,
                             long long cap, int *tri, hipStream_t st);

// cavity filling (fill.hip): boundary seeds of one molecule's labels; passes
// over 8^3 tiles until *changed stays 0 (zeroed by the caller before each
// pass) -- for a batch over (molecule, 8^3 tile) units; then 0 -> 1 (counted
// in *filled) and 2 -> 0.
hipError_t launch_fill_seed(uint8_t *L, const int dims[3], hipStream_t st);
hipError_t launch_fill_pass(const Mol *mols_dev, uint8_t *const *labels_dev, const int2 *units,
                            int nunits, int *changed, hipStream_t st);
hipError_t launch_fill_pass1(uint8_t *L, const int dims[3], int *changed, hipStream_t st);
hipError_t launch_fill_finish(uint8_t *L, long long n, unsigned long long *filled,
                              hipStream_t st);

// vertex export
hipError_t launch_export_vertices(const Mol &m, double *p, int *atoms, int8_t *sign,
                                  long long count, hipStream_t st);

}  // namespace eses
