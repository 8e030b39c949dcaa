/*
 * eses.h -- C-ABI of the MI355X (gfx950) Eulerian solvent-excluded surface
 * hot path.
 *
 * The method (Zhao, Wang, Tong, Wei, arXiv 1809.04352) takes a list of atoms
 * with centres c_i and van der Waals radii r_i (eq. 1), a probe radius rho, a
 * grid spacing h and a box, and produces
 *   - Inside[i,j,k] = 1 iff grid point (i,j,k) lies in M, the volume enclosed
 *     by the solvent-excluded surface (SES) (eq. 2), and
 *   - for each grid edge whose two ends carry different labels, the point
 *     where the surface crosses it, p = lambda s + (1 - lambda) t (eq. 3-4),
 *     with its outward normal and the patch it lies on.
 * The SES is the boundary of the union of the probe balls that overlap no atom
 * (section 1): with s_i = r_i + rho, U the union of the open balls B(c_i, s_i)
 * and A = R^3 \ U the admissible probe centres, M = { x : dist(x, A) >= rho }.
 * Its patches are convex (probe touching one atom), saddle (two) and concave
 * (three or more) (section 1).  The concave-patch probe positions -- points on
 * three SAS spheres that lie in A -- are produced on the way and exported.
 *
 * Conventions shared by every call:
 *   - Grid point (i,j,k) is x = lo + (i,j,k) h, each coordinate evaluated as
 *     fl(lo_a + fl(i h)) in FP64 (no fused multiply-add).  dims[a] =
 *     ceil((hi_a - lo_a) / h) + 1 (the padded bounding box of section 2.3).
 *   - Labels are uint8, 1 = inside M, laid out labels[i + nx (j + ny k)]
 *     (x fastest).  A point at distance exactly rho from A is inside (M is
 *     closed).  Probe-accessible interior cavities count as solvent.
 *   - Edge key = 3 * (i + nx (j + ny k)) + axis for the edge from s = (i,j,k)
 *     to t = s + e_axis; only the six-neighbour axis edges exist.  lambda is
 *     the weight of s in eq. 4 (1 at s, 0 at t) and marks the FIRST label
 *     change walking from s.  Records are sorted by key.
 *   - Normals are unit vectors pointing out of M into the solvent.
 *   - patch_type: 1 convex (atoms[0] = the atom), 2 saddle (atoms[0..1], the
 *     pair), 3 concave (atoms[0..2], the probe's three atoms); unused atom
 *     slots are -1.  Atom ids are the caller's indices, ascending.
 *   - Concave probe positions are reported once per atom triple (a<b<c) and
 *     side: sign = +1 iff (p - c_a) . ((c_b - c_a) x (c_c - c_a)) > 0.  A
 *     probe touching a fourth atom is admissible (|p - c| >= s non-strict,
 *     tested as |p - c|^2 >= s^2 (1 - 1e-9)), so a probe touching four or
 *     more atoms is reported by every triple of them.
 *
 * Memory and streams: every pointer inside eses_molecule, and every output
 * buffer, is DEVICE memory owned by the caller; it must stay valid until the
 * work queued on `stream` (a hipStream_t, NULL = the default stream) has
 * finished.  The candidates handle and its device workspace are owned by the
 * library and released by eses_free_candidates.  Calls that return counts to
 * the host synchronise `stream`.
 *
 * Errors: every call returns an eses_status; nothing throws across the ABI.
 * On failure eses_last_error() holds a message (thread-local, valid until the
 * next call on the same thread).
 */
#ifndef ESES_H
#define ESES_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ESES_OK = 0,
    ESES_EINVAL = -1,     /* bad argument: null, non-finite, n <= 0, dims < 2, shared centres ... */
    ESES_ENOMEM = -2,     /* device allocation failed; message holds the bytes */
    ESES_ECAPACITY = -3,  /* output capacity too small; required count returned */
    ESES_EDEVICE = -4,    /* a HIP runtime call failed */
    ESES_EINTERNAL = -5   /* an internal list overflowed or a kernel reported
                             an inconsistency */
} eses_status;

typedef enum {
    ESES_FP64 = 0,        /* every inside/outside test in FP64 */
    ESES_FP32_RECHECK = 1 /* FP32 tests with a rounding-error bound per test;
                             points whose margin is below the bound are
                             re-tested in FP64 */
} eses_precision;

/* One molecule: the paper's problem statement (eq. 1, probe radius, grid
 * spacing, box).  centres: device, [n_atoms][3] float64, angstrom, pairwise
 * distinct (atoms are distinct balls: two atoms with the same centre make
 * eses_build_candidates return ESES_EINVAL).
 * radii: device, [n_atoms] float64, finite and > 0.  probe_radius and spacing
 * finite and > 0.  bbox_lo/bbox_hi: host values; grid point (0,0,0) = bbox_lo
 * and dims = ceil((hi - lo) / h) + 1 >= 2 per axis. */
typedef struct {
    const double *centers;
    const double *radii;
    int64_t n_atoms;
    double probe_radius;
    double spacing;
    double bbox_lo[3];
    double bbox_hi[3];
} eses_molecule;

/* Tuning knobs; pass NULL for defaults.  Results never depend on them. */
typedef struct {
    int32_t tile;          /* tile edge in grid points: 4 or 8 (default 8) */
    int32_t force_recheck; /* test aid: with ESES_FP32_RECHECK, treat every FP32
                              decision as uncertain so each point is re-tested
                              in FP64 (0 = off) */
    int32_t blocks_per_cu; /* batches (n_mols > 1): persistent workgroups per
                              compute unit of the fused classification launch
                              (0 = as many as fit) */
    int32_t edge_fallback; /* test aid: send every crossing edge to the
                              one-wavefront-per-edge root kernel, the path
                              otherwise taken only by edges of a tile whose
                              root lists overflow (0 = off) */
    int32_t vertex_pool;   /* test aid: entries of the pool in which the
                              probe-position count pass keeps what it finds
                              (0 = default); when the pool overflows, the
                              positions are recomputed by a fill pass */
    int32_t tile_pool;     /* test aid: entries of a tile's candidate lists the
                              count pass keeps (0 = default; at most the
                              default); tiles with more are rebuilt by a fill
                              pass */
    int32_t unc_queue;     /* test aid: initial capacity of the queue of points
                              whose FP64 decision cannot be certified (0 =
                              default); a queue that overflows is grown and the
                              molecule classified again */
    int32_t unit_order;    /* batches: order in which the fused classification
                              takes its (molecule, tile) units: 0 = three
                              classes (tiles with probe, face or circle
                              candidates, then atom-only tiles, then empty
                              tiles; default), 1 = heaviest first by a cost
                              estimate from the tile's list sizes */
    int32_t edges_per_molecule; /* test aid, batches: find and group each
                              molecule's crossing edges with launches of its
                              own on worker streams, the path otherwise taken
                              only when a molecule's grid has 3 x points >=
                              2^31 - 1 (0 = off: one launch per pass over the
                              whole batch) */
} eses_config;

typedef struct eses_candidates eses_candidates; /* opaque, library-owned */

/* Counts describing one molecule's candidate set. */
typedef struct {
    int64_t n_atoms;
    int32_t dims[3];
    int64_t n_points;
    int64_t n_neighbour_pairs;   /* ordered pairs i != j with overlapping SAS balls */
    int64_t n_circles;           /* unordered pairs whose SAS spheres meet in a circle */
    int64_t n_vertices;          /* concave probe positions (exposed three-sphere points) */
    int64_t n_exposed_faces;     /* atoms whose SAS sphere has an admissible point */
    int64_t n_exposed_circles;   /* circles with an admissible point */
    int64_t n_tiles;
    int64_t tile_list_entries;   /* total per-tile candidate entries */
} eses_candidate_stats;

typedef struct {
    int64_t n_points;
    int64_t n_inside;
    int64_t n_rechecked;         /* FP32_RECHECK: points re-tested in FP64 */
    /* Work of the FP64 decision procedure, counted by a separate statistics
     * pass over the same points (run only when stats are requested): */
    int64_t n_shell;             /* points inside an SAS ball but in no van der Waals ball */
    int64_t tests_atom;          /* point-atom ball tests */
    int64_t tests_vertex;        /* point-probe (concave) tests */
    int64_t tests_face;          /* face reach tests */
    int64_t tests_face_cut;      /* face admissibility half-space tests */
    int64_t tests_circle;        /* circle reach tests */
    int64_t tests_circle_cut;    /* circle admissibility half-space tests */
    int64_t n_exact;             /* points whose FP64 decision could not be
                                    certified, re-decided exactly on the host */
} eses_classify_stats;

/* Structure-of-arrays output of eses_edge_intersections for one molecule.
 * All arrays are device memory of `capacity` records. */
typedef struct {
    int64_t *key;          /* [capacity] edge key, ascending */
    double *lambda;        /* [capacity] weight of s, eq. 4 */
    double *normal;        /* [capacity][3] outward unit normal */
    uint8_t *patch_type;   /* [capacity] 1 convex, 2 saddle, 3 concave */
    int32_t *atoms;        /* [capacity][3] atom ids, -1 unused */
    int64_t capacity;
} eses_isect_soa;

/* Host helper: the padded bounding box of the van der Waals spheres,
 * lo = min(c - r) - margin, hi = max(c + r) + margin (section 2.3).
 * centers_host [n][3] and radii_host [n] are HOST arrays. */
eses_status eses_bbox_from_atoms(const double *centers_host, const double *radii_host, int64_t n,
                                 double margin, double lo[3], double hi[3]);

/* Host helper: exact labels (eq. 2) of points, in exact arithmetic on the
 * given doubles -- the arbiter that eses_classify applies to the grid points
 * whose FP64 decision it cannot certify, exported for callers who need the
 * label of arbitrary points.  All arrays are HOST memory owned by the caller:
 * centers [n_atoms][3], radii [n_atoms] (finite, > 0), probe_atoms
 * [n_probes][3] (ascending atom indices of each concave probe position, as
 * eses_copy_vertices reports them) and probe_sign [n_probes] (its side),
 * points [n_points][3]; labels [n_points] receives 1 (inside) or 0.  Each
 * comparison of the label (ball membership, a candidate's distance against
 * rho, the admissibility of a radial projection or a circle point) is a
 * polynomial in the inputs up to square roots removed by squaring; its sign is
 * taken in FP64 when a running error bound decides it, else exactly in
 * dyadic big-integer arithmetic.  ESES_EINVAL for a null or non-finite
 * argument or a probe that names no atom. */
eses_status eses_exact_labels(const double *centers, const double *radii, int64_t n_atoms,
                              double probe_radius, const int32_t *probe_atoms,
                              const int8_t *probe_sign, int64_t n_probes, const double *points,
                              int64_t n_points, uint8_t *labels);

/* Host helper: dims[a] = ceil((hi_a - lo_a) / spacing) + 1 of a molecule. */
eses_status eses_grid_dims(const eses_molecule *mol, int32_t dims[3]);

/* Stage 1 of the method (section 2.2: the grid and the analytic patches).
 * Bins the atoms, finds overlapping SAS pairs and their circles, enumerates
 * the concave probe positions (three-sphere points in A), marks which faces
 * and circles have admissible points, and builds per-tile candidate lists
 * for tiles of `tile`^3 grid points (the blocks of section 2.3, with the
 * half-open ownership of section 2.5).  Synchronises `stream` to size its
 * workspace.  On success *out is a new handle. */
eses_status eses_build_candidates(const eses_molecule *mols, int32_t n_mols,
                                  const eses_config *cfg, void *stream, eses_candidates **out);

/* Counts of molecule `mol` of a built handle (host). */
eses_status eses_candidates_info(const eses_candidates *c, int32_t mol, eses_candidate_stats *st);

/* Copies the concave probe positions of molecule `mol` into device buffers:
 * p [capacity][3] float64, atoms [capacity][3] int32 (ascending caller ids),
 * sign [capacity] int8.  *count (host) receives the number of positions; if
 * it exceeds capacity the first `capacity` are written and ESES_ECAPACITY is
 * returned.  Order: deterministic, unspecified.  Synchronises `stream`. */
eses_status eses_copy_vertices(const eses_candidates *c, int32_t mol, double *p, int32_t *atoms,
                               int8_t *sign, int64_t capacity, int64_t *count, void *stream);

/* Stage 2 (eq. 2): labels every grid point of every molecule.
 * labels: host array of n_mols DEVICE pointers, each [nx*ny*nz] uint8.
 * stats: host array of n_mols entries or NULL (non-NULL synchronises).
 * A handle of several molecules runs one persistent fused launch over all
 * their tiles (heaviest tiles first, from an atomic work queue), recorded
 * once per precision as a HIP graph and replayed on later calls. */
eses_status eses_classify(eses_candidates *c, eses_precision prec, uint8_t *const *labels,
                          eses_classify_stats *stats, void *stream);

/* Stage 3 (eq. 3-4): records for every edge whose end labels differ.
 * labels: host array of n_mols DEVICE pointers (as written by eses_classify).
 * out: host array of n_mols SoA descriptors.  counts: host [n_mols], receives
 * the number of crossing edges per molecule; records beyond a molecule's
 * capacity are dropped and ESES_ECAPACITY is returned.  ESES_EINTERNAL if a
 * candidate list of the build met more entries than it had counted, or an
 * edge has more roots than the per-edge lists hold.  For a handle of several
 * molecules, each molecule's crossing edges are found and grouped on worker
 * streams and the roots of all molecules run in one persistent fused launch
 * (molecules with most crossing edges first).  Synchronises. */
eses_status eses_edge_intersections(eses_candidates *c, const uint8_t *const *labels,
                                    const eses_isect_soa *out, int64_t *counts, void *stream);

/* Surface mesh, area and volume of each molecule (section 2.2: the Eulerian
 * output is turned into a triangle mesh by marching cubes; the appendix table
 * reports each complex's SES area and volume).  Every cube of eight
 * axis-adjacent grid points with mixed labels is cut by the triangles of its
 * configuration; a triangle's corners are crossing points of the cube's edges
 * (the records of eses_edge_intersections).  The case table follows one rule
 * (on a face with four crossings, each inside corner is cut off), so
 * neighbouring cubes agree on their shared faces and the mesh is closed,
 * every edge shared by two triangles of opposite orientation; triangles are
 * oriented with normals out of M.  area = sum of triangle areas, volume =
 * divergence theorem over the mesh.
 * labels, isect, counts: as filled by eses_classify and
 * eses_edge_intersections (every crossing record present, else ESES_EINVAL).
 * triangles: NULL, or a host array of n_mols DEVICE pointers [cap][3] int32
 * that receive each triangle's corners as indices into the molecule's
 * records, with tri_capacity (host [n_mols]) their capacities; stats: host
 * [n_mols].  Triangles beyond a capacity are dropped with ESES_ECAPACITY
 * (n_triangles holds the required count).  Synchronises `stream`. */
typedef struct {
    double area;          /* angstrom^2 */
    double volume;        /* angstrom^3 */
    int64_t n_triangles;
} eses_mesh_stats;

eses_status eses_mesh(eses_candidates *c, const uint8_t *const *labels,
                      const eses_isect_soa *isect, const int64_t *counts,
                      int32_t *const *triangles, const int64_t *tri_capacity,
                      eses_mesh_stats *stats, void *stream);

/* Cavity-filled variant (the exterior-only reading of section 1's probe
 * balls "outside" the molecule, where the paper leaves open whether probes in
 * enclosed cavities count): in place on the labels of eses_classify, every
 * outside grid point (label 0) that no path of axis-adjacent outside points
 * joins to the grid's boundary faces becomes inside (1); the other labels are
 * unchanged.  Crossing records computed from the filled labels by
 * eses_edge_intersections then bound the molecule without its cavities.
 * labels: host array of n_mols DEVICE pointers (as for eses_classify);
 * n_filled: host [n_mols] or NULL, receives the points filled per molecule.
 * A flood fill from the boundary over 8^3 tiles in LDS, repeated until no
 * tile changes (one read-back per pass).  Synchronises `stream`. */
eses_status eses_fill_cavities(eses_candidates *c, uint8_t *const *labels, int64_t *n_filled,
                               void *stream);

/* Out-of-core form (the paper's block decomposition, sections 2.3-2.5 and
 * Alg. 1, in z-slabs): stages 2 and 3 of a handle of ONE molecule with the
 * grid's labels and records held in HOST memory and device memory bounded by
 * the candidates plus two slabs.  The grid is cut into slabs of slab_planes
 * z-planes (a positive multiple of the tile edge, 8 by default; the last slab
 * may be shorter).  Each slab is classified (with exact arbitration) and its
 * crossing edges solved on the GPU -- one extra plane is labelled so that the
 * z-edges leaving the slab's last plane are found -- and its own planes'
 * labels and the records of its points are copied to the host on a second
 * stream while the next slab runs.  Results are those of eses_classify and
 * eses_edge_intersections on the whole grid, bit for bit.
 * labels_host: HOST [nz][ny][nx] uint8 (pinned memory lets the copies
 * overlap the work); out_host: descriptor of HOST arrays (records appended in
 * key order); *count (host) receives the number of crossing edges (records
 * beyond out_host->capacity are dropped with ESES_ECAPACITY).  ESES_EINVAL
 * for a handle of several molecules or a slab size that is not a positive
 * multiple of the tile edge.  Synchronises `stream`. */
eses_status eses_stream_slabs(eses_candidates *c, eses_precision prec, int32_t slab_planes,
                              uint8_t *labels_host, const eses_isect_soa *out_host,
                              int64_t *count, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, hosts that forbid hipMalloc): stage 3 of a
 * handle of ONE molecule, as eses_edge_intersections, with every temporary of
 * its kernels (crossing-edge counts and offsets, the grouping by tile, the
 * work queue, fallback lists, counters) cut from a static device array of
 * 64 MiB that the library holds on each GPU it runs on until the process
 * ends; the call allocates nothing (no hipMalloc, hipHostMalloc, hipFree or
 * allocating library routine), and `labels` and `out` are the caller's as
 * before.  The scratch bounds the molecule: about 2 million crossing edges
 * at the batch's tile sizes; larger work returns ESES_ECAPACITY naming the
 * bytes it needs, before any record is written.  Every call on a GPU shares
 * that GPU's array and leaves its contents behind (what must start at zero is
 * cleared by the call): calls that overlap on one GPU -- from two threads, or
 * on two streams without ordering between them -- race and must not be made.
 * labels: DEVICE [nx*ny*nz] as written by eses_classify; out: host
 * descriptor of device arrays; *count (host) receives the number of crossing
 * edges (records beyond out->capacity are dropped with ESES_ECAPACITY).
 * ESES_EINVAL for a handle of several molecules.  Synchronises `stream`. */
eses_status eses_edge_intersections_noalloc(eses_candidates *c, const uint8_t *labels,
                                            const eses_isect_soa *out, int64_t *count,
                                            void *stream);

/* Work of the edge-root kernel for molecule-by-molecule statistics, counted
 * by a separate pass (not timed) over the same crossing edges. */
typedef struct {
    int64_t n_edges;          /* crossing edges */
    int64_t reach_sphere;     /* reach tests of van der Waals and probe spheres */
    int64_t reach_torus;      /* reach tests of tori */
    int64_t quad_solves;      /* sphere quadratics solved */
    int64_t quartic_solves;   /* torus quartics set up */
    int64_t horner_flops;     /* flops of polynomial evaluations in the quartic solver */
    int64_t cut_tests;        /* admissibility half-space tests of roots */
    int64_t label_evals;      /* labels evaluated between roots */
    int64_t label_tests[6];   /* their tests: atom, probe, face, face cut, circle, circle cut */
    int64_t cone_tests;       /* cut planes tested against an edge's direction cone */
} eses_edge_stats;

/* Runs the edge statistics pass for every molecule of `c` with the labels
 * of eses_classify.  stats: host [n_mols].  Synchronises. */
eses_status eses_edge_work(eses_candidates *c, const uint8_t *const *labels,
                           eses_edge_stats *stats, void *stream);

/* Kernel timing for diagnostics.  While enabled (process-wide), the library
 * records HIP events on the caller's stream around its classification kernel
 * and its edge kernels; eses_get_kernel_times returns the last durations of a
 * handle (waiting for the events).  For a handle of several molecules the
 * spans are those of the batched forms: the fused classification launch, the
 * crossing-edge passes and grouping of all molecules (one launch per pass, or
 * per molecule on worker streams for very large grids; from the first start
 * to the last end) and the fused root launch. */
typedef struct {
    double classify_ms;       /* classification launch of the last eses_classify */
    double edge_detect_ms;    /* crossing-edge pass and grouping of the last
                                 eses_edge_intersections */
    double edge_roots_ms;     /* root kernels of the last eses_edge_intersections */
} eses_kernel_times;

void eses_set_timing(int enable);
eses_status eses_get_kernel_times(const eses_candidates *c, eses_kernel_times *out);

/* Device workspace is taken on the caller's stream and, when released, kept
 * in a cache (per device, stream and power-of-two size class) for the next
 * call on that stream.  eses_trim_cache synchronises every device that holds
 * cached blocks and frees them; call it when no library work is in flight
 * (e.g. before handing the memory to other code).  Returns ESES_EDEVICE if a
 * HIP call failed. */
eses_status eses_trim_cache(void);

/* Device workspace from the caller (e.g. a framework's caching allocator).
 * With both functions set (process-wide), the library takes every workspace
 * block from alloc(bytes, stream, ctx) -- NULL means no memory
 * (ESES_ENOMEM) -- and hands it back with release(ptr, stream, ctx), instead
 * of using its own cache.  `stream` is the stream the block is used on (the
 * caller's stream; for a batch's per-molecule temporaries, one of the
 * library's worker streams, which follow the caller's stream); release is
 * stream-ordered: work already queued on `stream` may still use the block,
 * as with hipFreeAsync, so the allocator must not hand it to other work
 * before that stream's queued work completes.  Both may be called from the
 * library's worker threads.  NULL functions restore the cache; blocks taken
 * before a change go back where they came from.  Call it while no library
 * work is being set up on another thread. */
typedef void *(*eses_alloc_fn)(size_t bytes, void *stream, void *ctx);
typedef void (*eses_release_fn)(void *ptr, void *stream, void *ctx);
void eses_set_allocator(eses_alloc_fn alloc, eses_release_fn release, void *ctx);

/* Releases the handle; its device workspace returns to the cache of the
 * stream it was built on (eses_trim_cache frees it).  NULL is ignored. */
void eses_free_candidates(eses_candidates *c);

/* Message of the last failed call on this thread ("" if none). */
const char *eses_last_error(void);

/* Library version string. */
const char *eses_version(void);

#ifdef __cplusplus
}
#endif

#endif /* ESES_H */
