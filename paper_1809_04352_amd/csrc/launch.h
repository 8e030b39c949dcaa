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

// Probe positions found by the count pass of the atoms whose neighbours and
// circles fit in LDS (p: x, y, z, -; id: circle, -, k, sign); count: one
// int, zeroed before the count pass.  When count <= cap after it,
// launch_vertex_place writes them (consuming the per-circle counts vcnt) and
// the fill pass (use = 1) skips those atoms; launch_vertex_order then puts
// every circle's positions in the fill pass's order.
struct VertexPool {
    GMEM double4 *p;
    GMEM int4 *id;
    GMEM int *count;
    int cap;
    int use;
};

// Tile lists kept by the count pass: each tile's four lists (atoms, faces,
// circles, probes, in that order) copied into its slot of `pool` (cap ints
// per tile, cap <= tile_keep_max()) at off[t] = t * cap, or off[t] = -1 when
// they do not fit (then *unpooled, zeroed before, is set and the fill pass
// rebuilds that tile).
struct TilePool {
    GMEM int *pool, *off, *unpooled;
    int cap;
};
int tile_keep_max();

// Temporaries of one molecule's build (device pointers; the counts npool and
// tp_unpooled are set by the host from read-backs before the kernels that
// use them).
struct BuildTmp {
    GMEM double *bounds;       // [8]: centre bounds (lo, hi), largest radius
    GMEM int *bad;             // non-finite or non-positive input
    GMEM int *cell_id, *cnt, *fillb, *slot;
    GMEM int *nbr_cnt, *circ_cnt;
    GMEM int *nbr_pool;        // [n][NBR_POOL]: each atom's SAS neighbours as the count pass
                               // found them (ascending; complete when they fit)
    GMEM int *nbr_big;         // atoms with more neighbours than that (ranked by k_nbr_sort)
    int nnbr_big;         // (its value, read back)
    GMEM int *vcnt;            // [ncirc] probe positions per circle
    VertexPool pool;
    int npool;            // positions the count pass pooled
    GMEM int *vx_big;          // atoms whose lists exceed LDS (positions left to the fill pass)
    int nvx_big;          // (its value, read back)
    GMEM int *face_cnt, *ecf, *ec_pos;
    GMEM int *fcut_cnt, *eccut_cnt;
    // kept cuts found by the cut count passes, for their fill passes: bit q
    // of word (2 f + q / 64) for cut q of face f, bit q of word e for the
    // q-th reaching cut of exposed circle e (where the lists were staged)
    GMEM unsigned long long *fcut_keep, *eccut_keep;
    GMEM int *cA, *cF, *cC, *cV;  // per-tile list lengths
    TilePool tp;
    int tp_unpooled;      // some tile's lists did not fit its pool slot
    int pad;
};

// Neighbours per atom kept by the neighbour count pass for the fill pass.
constexpr int NBR_POOL = 128;

// One launch over the blocks of several molecules: block b works for
// molecule q with start[q] <= b < start[q + 1] (the largest such q, so
// molecules with no blocks are skipped), as that molecule's block
// b - start[q].  mols, tmp: device arrays of the molecules' views and
// temporaries.
struct Seg {
    const Mol *mols;
    const BuildTmp *tmp;
    const int *start;
    int nm;
};

enum BuildKernel {
    BK_BOUNDS, BK_CELL_COUNT, BK_CELL_FILL, BK_CELL_SCATTER, BK_CELL_SORT, BK_GATHER, BK_NBR,
    BK_NBR_SORT, BK_VERTEX, BK_VERTEX_PLACE, BK_VERTEX_ORDER, BK_CIRCLE_FREE, BK_ATOM_FEATURES,
    BK_EC_FLAG, BK_EC_IDS, BK_FEATURE_OFF, BK_FACE_LIST, BK_FACE_CUTS, BK_EC_CUTS, BK_TILES,
    BK_TILES_FILL, BK_TILES_PLACE
};
// Blocks of kernel k for one molecule, and the launch of k (count pass where
// k has two) or of its fill pass (BK_NBR, BK_VERTEX, BK_EC_CUTS) over a Seg.
long long build_blocks(BuildKernel k, const Mol &m, const BuildTmp &t);
hipError_t launch_build(BuildKernel k, const Seg &s, long long nblocks, hipStream_t st);
hipError_t launch_build_fill(BuildKernel k, const Seg &s, long long nblocks, hipStream_t st);

// Exclusive scans of many int arrays of their own lengths in three launches
// (chunk sums, one workgroup per array over its chunk sums, chunks): array g
// scans in[0..n) into out[0..n] (out[n] = total).  chunk0[g]: the array's
// first chunk (prefix of ceil(n / scan_seg_chunk()) over the arrays);
// sums: nchunks ints of workspace.  Arrays of length 0 get out[0] = 0.
struct ScanSeg {
    GMEM const int *in;
    GMEM int *out;
    long long n;
    long long chunk0;
};
long long scan_seg_chunk();
hipError_t scan_seg(const ScanSeg *segs, int nseg, long long nchunks, int *sums, hipStream_t st);

// Ints at device addresses addr[0..n) gathered into out[0..n).
hipError_t launch_gather_ints(const int *const *addr, int n, int *out, hipStream_t st);

// stage 2
hipError_t launch_classify(const Mol &m, bool fp32, uint8_t *labels, hipStream_t st);
// Classes of the batch's classification units (heaviest first).
constexpr int UNIT_CLASSES = 24;
hipError_t launch_units(const Mol *mols_dev, const int *tile_base_dev, int nmols, long long total,
                        int order, int *cls_count, int *cls_fill, int2 *units, hipStream_t st);
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
// Slab views: *n_own = the keys below limit (a prefix), which are shifted by
// `shift` into the whole grid's numbering.
hipError_t launch_slab_keys(long long *keys, long long count, long long limit, long long shift,
                            long long *n_own, hipStream_t st);
hipError_t launch_edge_group(const Mol &m, const long long *keys, long long count, int *tcount,
                             int *ccount, int *coff, const int *rank, int *order, int *units,
                             int *tmp, hipStream_t st);
// The crossing-edge passes over every molecule of a batch in one launch each.
// Per molecule: its labels; bcount/boff: per detection block (of
// edge_detect_blocks) counts and their exclusive scan (boff[nblk] = the
// total); nw: the edges written (the total, at most the output capacity);
// the rest as for launch_edge_detect_write and launch_edge_group, tcount and
// the units header zeroed before the write pass.
struct EdgeDetectJob {
    GMEM const uint8_t *L;
    GMEM int *bcount, *boff;
    GMEM long long *keys;
    GMEM int *tcount, *ccount, *coff, *rank, *order, *units;
    long long nw;
};
// Block starts (nm + 1 prefix sums, device and host copies) of the write
// pass (detection blocks of the molecules with nw > 0), the tile passes (256
// tiles a block) and the edge pass (256 edges a block).
struct EdgeBatchStarts {
    const int *write, *tile, *edge;
    const int *write_host, *tile_host, *edge_host;
};
// start: block starts of the count pass (every molecule's detection blocks).
hipError_t launch_edge_detect_count_batch(const Mol *mols, const EdgeDetectJob *jobs,
                                          const int *start, const int *start_host, int nm,
                                          hipStream_t st);
// (also zeroes every molecule's ownerless-record counter, Mol::diag[3])
hipError_t launch_edge_detect_write_batch(const Mol *mols, const EdgeDetectJob *jobs,
                                          const EdgeBatchStarts &s, int nm, hipStream_t st);
// coff_scan: the scans of ccount into coff of the molecules with nw > 0
// (scan_seg layout; sums: nchunks ints of workspace).
hipError_t launch_edge_group_batch(const Mol *mols, const EdgeDetectJob *jobs,
                                   const EdgeBatchStarts &s, const ScanSeg *coff_scan,
                                   int nscan, long long nchunks, int *sums, int nm,
                                   hipStream_t st);
// Diagnostic word k (Mol::diag) of every molecule of a batch set to v.
hipError_t launch_diag_set(const Mol *mols, int nm, int k, int v, hipStream_t st);
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
    GMEM const uint8_t *L;
    GMEM const long long *keys;
    GMEM const int *order, *tcount, *coff, *units;
    GMEM double *lam, *nrm;
    GMEM uint8_t *ptype;
    GMEM int *patoms, *fallback, *nfallback;
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
