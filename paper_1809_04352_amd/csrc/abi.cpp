// C-ABI of the ESES hot path: argument checks, workspace, launch order and
// the count read-backs that size the lists (see include/eses.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <functional>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <initializer_list>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <utility>
#include <vector>

#include "../../include/eses.h"
#include "eses_device.h"
#include "exact.h"
#include "launch.h"
#include "worker_pool.h"

using namespace eses;

namespace {

thread_local std::string g_err;
std::atomic<int> g_timing{0};

void set_err(const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
}

struct Status {
    eses_status s;
};

#define CK(call)                                                                     \
    do {                                                                             \
        hipError_t e_ = (call);                                                      \
        if (e_ != hipSuccess) {                                                      \
            set_err("%s failed: %s", #call, hipGetErrorString(e_));                  \
            return ESES_EDEVICE;                                                     \
        }                                                                            \
    } while (0)

#define CKS(expr)                        \
    do {                                 \
        eses_status s_ = (expr);         \
        if (s_ != ESES_OK) return s_;    \
    } while (0)

// Device memory cache.  Released workspace blocks are kept per (device,
// stream, power-of-two size class) and handed to the next request of that
// class on the same stream: the stream orders the reuse after the work that
// used the block, so no synchronisation is needed.  Blocks stay cached until
// eses_trim_cache.
struct BlockCache {
    std::mutex mu;
    std::map<std::tuple<int, hipStream_t, int>, std::vector<void *>> free;
};

BlockCache &block_cache() {
    static BlockCache *c = new BlockCache();  // outlives static destruction
    return *c;
}

// The caller's allocator (eses_set_allocator), when set: workspace blocks come
// from it and go back to it instead of the cache.
struct ExtAlloc {
    std::mutex mu;
    eses_alloc_fn alloc = nullptr;
    eses_release_fn release = nullptr;
    void *ctx = nullptr;
};

ExtAlloc &ext_alloc() {
    static ExtAlloc *a = new ExtAlloc();
    return *a;
}

int size_class(size_t bytes) {
    int c = 8;  // 256 B
    while (((size_t)1 << c) < bytes) ++c;
    return c;
}

// Device workspace of one molecule: every buffer taken on the stream and
// returned to the cache together.  `key` names the stream whose cache the
// blocks come from and return to (st unless `keyed`): a batch builds on worker
// streams that wait for the caller's stream, so they may take blocks from its
// cache, and the blocks go back there when the handle is freed.
struct Arena {
    struct Block {
        void *p;
        int dev, cls;                 // cls < 0: from the caller's allocator
        eses_release_fn release;      // (with its context)
        void *ctx;
    };
    std::vector<Block> blocks;
    hipStream_t st = nullptr;   // stream the blocks are used on (new blocks allocated on it)
    hipStream_t key = nullptr;  // cache of the blocks when `keyed` (the null stream is a
    bool keyed = false;         // stream like any other), else st's
    // carve mode: blocks are cut in order from [carve, carve + carve_cap) (a
    // caller-provided region) and nothing is allocated or released
    char *carve = nullptr;
    size_t carve_cap = 0, carve_used = 0;

    hipStream_t cache() const { return keyed ? key : st; }

    template <typename T>
    eses_status alloc(T **p, long long count) {
        const size_t bytes = sizeof(T) * (size_t)(count > 0 ? count : 1);
        if (carve) {
            const size_t at = (carve_used + 255) & ~(size_t)255;
            if (at + bytes > carve_cap) {
                set_err("the work needs more than the %zu bytes of static scratch (at least %zu)",
                        carve_cap, at + bytes);
                return ESES_ECAPACITY;
            }
            carve_used = at + bytes;
            *p = (T *)(carve + at);
            return ESES_OK;
        }
        int dev = 0;
        (void)hipGetDevice(&dev);
        {
            eses_alloc_fn fa;
            eses_release_fn fr;
            void *ctx;
            {
                ExtAlloc &ea = ext_alloc();
                std::lock_guard<std::mutex> lock(ea.mu);
                fa = ea.alloc;
                fr = ea.release;
                ctx = ea.ctx;
            }
            if (fa) {
                void *q = fa(bytes, (void *)cache(), ctx);
                if (!q) {
                    set_err("the caller's allocator returned no memory for %zu bytes", bytes);
                    return ESES_ENOMEM;
                }
                blocks.push_back({q, dev, -1, fr, ctx});
                *p = (T *)q;
                return ESES_OK;
            }
        }
        const int cls = size_class(bytes);
        void *q = nullptr;
        {
            BlockCache &bc = block_cache();
            std::lock_guard<std::mutex> lock(bc.mu);
            auto it = bc.free.find(std::make_tuple(dev, cache(), cls));
            if (it != bc.free.end() && !it->second.empty()) {
                q = it->second.back();
                it->second.pop_back();
            }
        }
        if (!q) {
            hipError_t e = hipMallocAsync(&q, (size_t)1 << cls, st);
            if (e != hipSuccess || !q) {
                (void)hipGetLastError();
                set_err("device allocation of %zu bytes failed: %s", (size_t)1 << cls,
                        hipGetErrorString(e));
                return ESES_ENOMEM;
            }
        }
        blocks.push_back({q, dev, cls, nullptr, nullptr});
        *p = (T *)q;
        return ESES_OK;
    }

    void release() {
        carve_used = 0;
        if (blocks.empty()) return;
        for (const Block &b : blocks)
            if (b.cls < 0 && b.release) b.release(b.p, (void *)cache(), b.ctx);
        BlockCache &bc = block_cache();
        std::lock_guard<std::mutex> lock(bc.mu);
        for (const Block &b : blocks)
            if (b.cls >= 0) bc.free[std::make_tuple(b.dev, cache(), b.cls)].push_back(b.p);
        blocks.clear();
    }
};

struct MolState {
    Mol m{};
    Arena arena;    // per-molecule blocks allocated after the build (a grown
                    // uncertain-point queue); the build's arrays are the handle's
    eses_candidate_stats stats{};
    // host arbiter of uncertain labels (built on first need) and the number of
    // points it re-decided in the last classification
    std::unique_ptr<eses::ExactMolecule> exact;
    int64_t n_exact = 0;
};

}  // namespace

struct eses_candidates {
    std::vector<MolState *> mols;
    hipStream_t stream = nullptr;
    // batch structures (n_mols > 1)
    Arena batch;
    Mol *mols_dev = nullptr;
    int *tile_base_dev = nullptr;
    int2 *units = nullptr;
    int *cls = nullptr;        // unit class counts, then class fill positions
    int unit_order = 0;        // eses_config.unit_order
    int edges_per_molecule = 0;  // eses_config.edges_per_molecule
    int *head = nullptr;
    uint8_t **labels_dev = nullptr;
    int *unc_counts = nullptr;  // [n_mols] gathered uncertain-point counts
    int2 *fill_units = nullptr;  // (molecule, 8^3 tile) units of the cavity fill
    long long n_fill_units = 0;
    long long nunits = 0;
    int batch_blocks[2] = {0, 0};  // persistent classification grid: FP64, FP32
    int blocks_per_cu = 0;
    // recorded fused classification, per precision
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    // kernel timing (eses_set_timing)
    hipEvent_t ev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    bool cls_timed = false;
    double detect_ms = 0.0, roots_ms = 0.0;
};

namespace {

bool finite3(const double *v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

eses_status dims_of(const eses_molecule *m, int32_t dims[3]) {
    if (!m) {
        set_err("molecule is NULL");
        return ESES_EINVAL;
    }
    if (!(std::isfinite(m->spacing) && m->spacing > 0.0)) {
        set_err("spacing must be finite and > 0");
        return ESES_EINVAL;
    }
    if (!finite3(m->bbox_lo) || !finite3(m->bbox_hi)) {
        set_err("bounding box must be finite");
        return ESES_EINVAL;
    }
    for (int a = 0; a < 3; ++a) {
        double ext = (m->bbox_hi[a] - m->bbox_lo[a]) / m->spacing;
        if (!(ext > 0.0) || !(ext < 2.0e9)) {
            set_err("box extent along axis %d must be positive and below 2e9 spacings", a);
            return ESES_EINVAL;
        }
        dims[a] = (int32_t)std::ceil(ext) + 1;
        if (dims[a] < 2) {
            set_err("fewer than 2 grid points along axis %d", a);
            return ESES_EINVAL;
        }
    }
    return ESES_OK;
}

template <typename T>
eses_status d2h(T *host, const T *dev, size_t count, hipStream_t st) {
    CK(hipMemcpyAsync(host, dev, sizeof(T) * count, hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    return ESES_OK;
}

// Pinned host memory (per thread) that the read-back kernel writes into: one
// slot per host thread that ever reads back, allocated once.  The batch
// workers below are persistent threads, so the slots stay bounded by the
// number of threads (each worker keeps one for the process lifetime).
long long *readback_host() {
    thread_local long long *p = nullptr;
    if (!p && hipHostMalloc((void **)&p, 16 * sizeof(long long), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        p = nullptr;
    }
    return p;
}

// Worker streams for per-molecule work of a batch: created once per device
// (default priority, not blocking on the null stream) and kept for the
// process lifetime, so that workspace cached under them stays reusable.
constexpr int N_WORKERS = 8;

eses_status worker_streams(hipStream_t *ws) {
    static std::mutex mu;
    static std::map<int, std::vector<hipStream_t>> pool;
    int dev = 0;
    CK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(mu);
    std::vector<hipStream_t> &v = pool[dev];
    while ((int)v.size() < N_WORKERS) {
        hipStream_t s = nullptr;
        CK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        v.push_back(s);
    }
    for (int q = 0; q < N_WORKERS; ++q) ws[q] = v[q];
    return ESES_OK;
}

// Runs job(q, stream) for q in [0, n) on the worker streams from the pool's
// host threads, after the work already queued on `st`; `st` then waits for
// all of it.  Returns the status of the lowest failing q (its message in
// g_err, prefixed with the molecule index).
template <class Job>
eses_status run_on_workers(int n, hipStream_t st, Job job) {
    hipStream_t ws[N_WORKERS];
    CKS(worker_streams(ws));
    const int P = std::min(N_WORKERS, n);
    hipEvent_t ready = nullptr, done[N_WORKERS] = {};
    CK(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
    CK(hipEventRecord(ready, st));
    for (int p = 0; p < P; ++p) {
        CK(hipEventCreateWithFlags(&done[p], hipEventDisableTiming));
        CK(hipStreamWaitEvent(ws[p], ready, 0));
    }
    int dev = 0;
    CK(hipGetDevice(&dev));
    std::atomic<int> next{0};
    std::vector<eses_status> res(n, ESES_OK);
    std::vector<std::string> msg(n);
    const std::function<void(int)> work = [&](int p) {
        if (hipSetDevice(dev) != hipSuccess) {
            for (int q = next++; q < n; q = next++) {
                res[q] = ESES_EDEVICE;
                msg[q] = "hipSetDevice failed in a worker thread";
            }
            return;
        }
        for (int q = next++; q < n; q = next++) {
            g_err.clear();
            res[q] = job(q, ws[p]);
            if (res[q] != ESES_OK) msg[q] = g_err;
        }
    };
    {
        eses::WorkerPool &pool = eses::WorkerPool::get();
        std::lock_guard<std::mutex> one_call(pool.call);
        pool.run(P, work);
    }
    eses_status out = ESES_OK;
    for (int p = 0; p < P; ++p) {
        if (hipEventRecord(done[p], ws[p]) != hipSuccess ||
            hipStreamWaitEvent(st, done[p], 0) != hipSuccess)
            out = ESES_EDEVICE;
    }
    (void)hipEventDestroy(ready);
    for (int p = 0; p < P; ++p) (void)hipEventDestroy(done[p]);
    for (int q = 0; q < n; ++q)
        if (res[q] != ESES_OK) {
            char pre[64];
            snprintf(pre, sizeof pre, "molecule %d: ", q);
            g_err = pre + msg[q];
            return res[q];
        }
    if (out != ESES_OK) set_err("ordering the worker streams failed");
    return out;
}

// Device scalars read back with one kernel and one synchronisation: each
// item's value (an int, or a long long where is64) lands in *out.
struct Scalar {
    const void *dev;
    bool is64;
    long long *out;
};

// Set while an allocation-free entry point runs on this thread: read-backs
// then copy each scalar into host stack memory instead of the pinned slot
// (whose first use on a thread allocates it).
thread_local bool g_noalloc = false;

eses_status read_scalars(std::initializer_list<Scalar> items, hipStream_t st) {
    if (g_noalloc) {
        long long v[16];
        int q = 0;
        for (const Scalar &it : items) {
            if (q == 16) {
                set_err("internal: more than 16 read-backs");
                return ESES_EINTERNAL;
            }
            v[q] = 0;
            if (it.is64) CK(hipMemcpyAsync(&v[q], it.dev, sizeof(long long), hipMemcpyDeviceToHost, st));
            else CK(hipMemcpyAsync(&v[q], it.dev, sizeof(int), hipMemcpyDeviceToHost, st));
            ++q;
        }
        CK(hipStreamSynchronize(st));
        q = 0;
        for (const Scalar &it : items) {
            *it.out = it.is64 ? v[q] : (long long)(int)(v[q] & 0xffffffffLL);
            ++q;
        }
        return ESES_OK;
    }
    long long *h = readback_host();
    if (!h) {
        set_err("pinned host allocation for read-backs failed");
        return ESES_ENOMEM;
    }
    ReadBack rb{};
    for (const Scalar &it : items) {
        if (rb.n == 16) {
            set_err("internal: more than 16 read-backs");
            return ESES_EINTERNAL;
        }
        rb.p[rb.n] = it.dev;
        rb.is64[rb.n] = it.is64 ? 1 : 0;
        ++rb.n;
    }
    CK(launch_collect(rb, h, st));
    CK(hipStreamSynchronize(st));
    int q = 0;
    for (const Scalar &it : items) *it.out = h[q++];
    return ESES_OK;
}


// ------------------------------------------------------- staged build

// Device blocks requested by size, allocated as one block and cut in order
// (each piece 256-byte aligned): a build stage allocates all molecules'
// arrays of one kind of memory at once.
struct Planner {
    struct Req {
        void **p;
        size_t bytes;
    };
    std::vector<Req> reqs;
    template <typename T>
    void add(T **p, long long count) {
        reqs.push_back({(void **)p, sizeof(T) * (size_t)std::max<long long>(count, 1)});
    }
    static size_t up(size_t b) { return (b + 255) & ~(size_t)255; }
    // allocates, assigns the pointers and, with `zero`, clears the block
    eses_status commit(Arena &A, hipStream_t st, bool zero) {
        if (reqs.empty()) return ESES_OK;
        size_t total = 0;
        for (const Req &r : reqs) total += up(r.bytes);
        char *base = nullptr;
        CKS(A.alloc(&base, (long long)total));
        size_t off = 0;
        for (const Req &r : reqs) {
            *r.p = base + off;
            off += up(r.bytes);
        }
        reqs.clear();
        if (zero) CK(fill_u32((uint32_t *)base, (long long)(total / 4), 0u, st));
        return ESES_OK;
    }
};

// A stage's control data -- the molecules' views and temporaries, the block
// offsets of its launches, its scan and read-back lists -- laid out in one
// host image and copied to the device in one transfer.
struct StageCtl {
    std::vector<char> host;
    char *dev = nullptr;
    template <typename T>
    size_t put(const T *p, size_t count) {
        size_t off = (host.size() + 15) & ~(size_t)15;
        host.resize(off + sizeof(T) * std::max<size_t>(count, 1));
        if (count) memcpy(host.data() + off, p, sizeof(T) * count);
        return off;
    }
    template <typename T>
    T *at(size_t off) const { return (T *)(dev + off); }
    eses_status upload(Arena &T, hipStream_t st) {
        CKS(T.alloc(&dev, (long long)host.size()));
        CK(hipMemcpyAsync(dev, host.data(), host.size(), hipMemcpyHostToDevice, st));
        return ESES_OK;
    }
};

// Builds every molecule of a handle: each stage is one launch per kernel over
// all molecules (a molecule per range of blocks), with one read-back per
// stage for the sizes the next stage allocates (four in all).
class Builder {
  public:
    Builder(eses_candidates *c, const eses_molecule *in, int nm, hipStream_t st)
        : c_(c), in_(in), nm_(nm), st_(st), M(nm), B(nm) {
        T_.st = st;
        c_->batch.st = st;
    }
    ~Builder() { T_.release(); }

    eses_status run(int tile, int force_recheck, int edge_fallback, int vertex_pool,
                    int tile_pool, int unc_queue) {
        CKS(stage_bounds(tile, force_recheck, edge_fallback, unc_queue));
        CKS(stage_nbr());
        CKS(stage_vertex(vertex_pool));
        CKS(stage_tiles(tile_pool));
        CKS(stage_fill());
        for (int q = 0; q < nm_; ++q) c_->mols[q]->m = M[q];
        // the stages' host images are released with the builder
        CK(hipStreamSynchronize(st_));
        return ESES_OK;
    }

  private:
    eses_candidates *c_;
    const eses_molecule *in_;
    int nm_;
    hipStream_t st_;
    std::vector<Mol> M;
    std::vector<BuildTmp> B;
    Arena T_;                 // temporaries, released when the build ends
    std::vector<StageCtl> ctl_;  // kept until the build ends (host images of copies)

    eses_status fail(int q, eses_status s, const char *msg) {
        set_err("molecule %d: %s", q, msg);
        return s;
    }

    // Seg of kernel k over all molecules (offsets into the stage's control
    // image); the block total in *nb.
    size_t starts(StageCtl &C, BuildKernel k, long long *nb) {
        std::vector<int> st((size_t)nm_ + 1, 0);
        long long t = 0;
        for (int q = 0; q < nm_; ++q) {
            st[(size_t)q] = (int)t;
            t += build_blocks(k, M[q], B[q]);
        }
        st[(size_t)nm_] = (int)t;
        *nb = t;
        return C.put(st.data(), st.size());
    }

    struct Launch {
        BuildKernel k;
        bool fill;
        size_t off;
        long long nb;
    };

    // The molecules' views and temporaries into a new stage control image.
    StageCtl &begin(size_t *mols_off, size_t *tmp_off) {
        ctl_.emplace_back();
        StageCtl &C = ctl_.back();
        *mols_off = C.put(M.data(), M.size());
        *tmp_off = C.put(B.data(), B.size());
        return C;
    }

    Seg seg(const StageCtl &C, size_t mo, size_t to, size_t so) const {
        Seg s;
        s.mols = C.at<Mol>(mo);
        s.tmp = C.at<BuildTmp>(to);
        s.start = C.at<int>(so);
        s.nm = nm_;
        return s;
    }

    // Scan list: (in, out, n) per array; the chunk sums are cut from T_.
    struct ScanList {
        std::vector<ScanSeg> segs;
        long long chunks = 0;
        size_t off = 0;
        int *sums = nullptr;
        void add(const int *in, int *out, long long n) {
            segs.push_back({dev(in), dev(out), n, chunks});
            chunks += (n + scan_seg_chunk() - 1) / scan_seg_chunk();
        }
    };

    eses_status scan(const StageCtl &C, ScanList &L) {
        return scan_seg(C.at<ScanSeg>(L.off), (int)L.segs.size(), L.chunks, L.sums, st_) ==
                       hipSuccess
                   ? ESES_OK
                   : (set_err("build scan launch failed"), ESES_EDEVICE);
    }

    // Read-back of ints at device addresses (one transfer and one
    // synchronisation for the whole stage).
    eses_status read_ints(StageCtl &C, size_t addr_off, int n, int *dst_dev,
                          std::vector<int> &out) {
        CK(launch_gather_ints(C.at<const int *>(addr_off), n, dst_dev, st_));
        out.resize((size_t)n);
        CK(hipMemcpyAsync(out.data(), dst_dev, sizeof(int) * n, hipMemcpyDeviceToHost, st_));
        CK(hipStreamSynchronize(st_));
        return ESES_OK;
    }

    // -- stage 0: arguments, bounds of the centres
    eses_status stage_bounds(int tile, int force_recheck, int edge_fallback, int unc_queue) {
        for (int q = 0; q < nm_; ++q) {
            const eses_molecule *in = &in_[q];
            Mol &m = M[q];
            m = Mol{};
            if (!in->centers || !in->radii)
                return fail(q, ESES_EINVAL, "centers and radii must be device pointers");
            if (in->n_atoms < 1 || in->n_atoms > (1LL << 27))
                return fail(q, ESES_EINVAL, "n_atoms must be in [1, 2^27]");
            if (!(std::isfinite(in->probe_radius) && in->probe_radius > 0.0))
                return fail(q, ESES_EINVAL, "probe_radius must be finite and > 0");
            int32_t dims[3];
            eses_status ds = dims_of(in, dims);
            if (ds != ESES_OK) {
                std::string msg = g_err;
                return fail(q, ds, msg.c_str());
            }
            m.n = (int)in->n_atoms;
            m.rho = in->probe_radius;
            m.h = in->spacing;
            for (int a = 0; a < 3; ++a) {
                m.lo[a] = in->bbox_lo[a];
                m.dims[a] = dims[a];
            }
            m.npts = (long long)dims[0] * dims[1] * dims[2];
            m.in_c = dev(in->centers);
            m.in_r = dev(in->radii);
            m.tile = tile;
            m.force_recheck = force_recheck ? 1 : 0;
            m.edge_fallback = edge_fallback ? 1 : 0;
            for (int a = 0; a < 3; ++a) m.tdims[a] = (dims[a] + tile - 1) / tile;
            const long long ntiles = (long long)m.tdims[0] * m.tdims[1] * m.tdims[2];
            if (ntiles > (1LL << 30)) return fail(q, ESES_EINVAL, "grid too large (tiles)");
            m.ntiles = (int)ntiles;
            m.unc_cap = unc_queue > 0 ? unc_queue
                                      : (int)std::min<long long>(
                                            std::max<long long>(4096, m.npts / 512), 1LL << 22);
        }
        double *bnd = nullptr;
        int *bad = nullptr;
        CKS(T_.alloc(&bnd, 8LL * nm_));
        CKS(T_.alloc(&bad, nm_));
        Planner Z;  // persistent, zeroed
        for (int q = 0; q < nm_; ++q) {
            B[q] = BuildTmp{};
            B[q].bounds = dev(bnd + 8 * q);
            B[q].bad = dev(bad + q);
            Z.add(&M[q].diag, 4);
            Z.add(&M[q].unc_n, 1);
        }
        CKS(Z.commit(c_->batch, st_, true));
        size_t mo, to;
        StageCtl &C = begin(&mo, &to);
        long long nb;
        const size_t so = starts(C, BK_BOUNDS, &nb);
        CKS(C.upload(T_, st_));
        CK(launch_build(BK_BOUNDS, seg(C, mo, to, so), nb, st_));
        std::vector<double> hb((size_t)8 * nm_);
        std::vector<int> hbad((size_t)nm_);
        CK(hipMemcpyAsync(hb.data(), bnd, sizeof(double) * hb.size(), hipMemcpyDeviceToHost, st_));
        CK(hipMemcpyAsync(hbad.data(), bad, sizeof(int) * nm_, hipMemcpyDeviceToHost, st_));
        CK(hipStreamSynchronize(st_));
        for (int q = 0; q < nm_; ++q) {
            if (hbad[(size_t)q])
                return fail(q, ESES_EINVAL, "centres must be finite and radii finite and > 0");
            Mol &m = M[q];
            const double *b = &hb[(size_t)8 * q];
            m.smax = b[6] + m.rho;
            // cells of edge s_max (slightly more): SAS neighbours, within 2 s_max plus the list
            // slack, lie within two cells along each axis
            m.cell = (m.smax + LIST_SLACK) * (1.0 + 1e-9);
            m.cmag = m.smax;
            for (int a = 0; a < 6; ++a) m.cmag = std::max(m.cmag, std::fabs(b[a]) + m.smax);
            for (;;) {
                long long ncell = 1;
                for (int a = 0; a < 3; ++a) {
                    m.clo[a] = b[a];
                    m.nc[a] = (int)std::floor((b[3 + a] - b[a]) / m.cell) + 1;
                    ncell *= m.nc[a];
                }
                if (ncell <= 4LL * m.n + 64) {
                    m.ncell = (int)ncell;
                    break;
                }
                m.cell *= 1.5;  // sparse input: coarser cells keep the table small
            }
        }
        return ESES_OK;
    }

    // -- stage 1: cell binning, neighbour and circle counts
    eses_status stage_nbr() {
        Planner P, Z, TT, TZ;
        for (int q = 0; q < nm_; ++q) {
            Mol &m = M[q];
            BuildTmp &t = B[q];
            P.add(&m.cell_start, m.ncell + 1);
            P.add(&m.atom, m.n);
            P.add(&m.orig, m.n);
            P.add(&m.nbr_off, m.n + 1);
            P.add(&m.circ_off, m.n + 1);
            P.add(&m.circ_any, m.n);
            P.add(&m.aflag, m.n);
            P.add(&m.unc_idx, m.unc_cap);
            TT.add(&t.cell_id, m.n);
            TZ.add(&t.cnt, m.ncell + 1);
            TT.add(&t.fillb, m.ncell + 1);
            TT.add(&t.slot, m.n);
            TT.add(&t.nbr_cnt, m.n);
            TT.add(&t.circ_cnt, m.n);
            TT.add(&t.nbr_pool, (long long)m.n * NBR_POOL);
            TZ.add(&t.nbr_big, 1);
        }
        CKS(P.commit(c_->batch, st_, false));
        CKS(TT.commit(T_, st_, false));
        CKS(TZ.commit(T_, st_, true));
        size_t mo, to;
        StageCtl &C = begin(&mo, &to);
        const BuildKernel ks[] = {BK_CELL_COUNT, BK_CELL_FILL, BK_CELL_SCATTER, BK_CELL_SORT,
                                  BK_GATHER, BK_NBR};
        std::vector<Launch> L;
        for (BuildKernel k : ks) {
            Launch l{k, false, 0, 0};
            l.off = starts(C, k, &l.nb);
            L.push_back(l);
        }
        ScanList S1, S2;
        for (int q = 0; q < nm_; ++q) S1.add(B[q].cnt, M[q].cell_start, M[q].ncell);
        for (int q = 0; q < nm_; ++q) {
            S2.add(B[q].nbr_cnt, M[q].nbr_off, M[q].n);
            S2.add(B[q].circ_cnt, M[q].circ_off, M[q].n);
        }
        S1.off = C.put(S1.segs.data(), S1.segs.size());
        S2.off = C.put(S2.segs.data(), S2.segs.size());
        CKS(T_.alloc(&S1.sums, S1.chunks + 1));
        CKS(T_.alloc(&S2.sums, S2.chunks + 1));
        std::vector<const int *> addr;
        for (int q = 0; q < nm_; ++q) {
            addr.push_back(M[q].nbr_off + M[q].n);
            addr.push_back(M[q].circ_off + M[q].n);
            addr.push_back(M[q].diag + 2);
            addr.push_back(B[q].nbr_big);
        }
        const size_t ao = C.put(addr.data(), addr.size());
        int *rb;
        CKS(T_.alloc(&rb, (long long)addr.size()));
        CKS(C.upload(T_, st_));
        CK(launch_build(BK_CELL_COUNT, seg(C, mo, to, L[0].off), L[0].nb, st_));
        CKS(scan(C, S1));
        for (size_t k = 1; k < L.size(); ++k)
            CK(launch_build(L[k].k, seg(C, mo, to, L[k].off), L[k].nb, st_));
        CKS(scan(C, S2));
        std::vector<int> h;
        CKS(read_ints(C, ao, (int)addr.size(), rb, h));
        for (int q = 0; q < nm_; ++q) {
            if (h[(size_t)4 * q + 2])
                return fail(q, ESES_EINVAL,
                            "atom centres must be pairwise distinct (two atoms share a centre)");
            nbr_total_.push_back(h[(size_t)4 * q]);
            M[q].ncirc = h[(size_t)4 * q + 1];
            B[q].nnbr_big = h[(size_t)4 * q + 3];
        }
        return ESES_OK;
    }
    std::vector<int> nbr_total_;

    // -- stage 2: neighbour lists, circles, probe-position counts, flags
    eses_status stage_vertex(int vertex_pool) {
        Planner P, TT, TZ;
        for (int q = 0; q < nm_; ++q) {
            Mol &m = M[q];
            BuildTmp &t = B[q];
            const int tot = nbr_total_[(size_t)q];
            P.add(&m.nbr, tot);
            P.add(&m.nbr_cov, tot);
            P.add(&m.circ_i, m.ncirc);
            P.add(&m.circ_j, m.ncirc);
            P.add(&m.circ_oR, m.ncirc);
            P.add(&m.circ_n, m.ncirc);
            P.add(&m.cflag, m.ncirc);
            P.add(&m.vert_off, m.ncirc + 1);
            P.add(&m.face_off_atom, m.n + 1);
            P.add(&m.ec_off_atom, m.n + 1);
            P.add(&m.vert_off_atom, m.n + 1);
            t.pool.cap = vertex_pool > 0 ? vertex_pool : std::max(4096, m.ncirc / 4);
            TT.add(&t.vcnt, m.ncirc);
            TT.add(&t.pool.p, t.pool.cap);
            TT.add(&t.pool.id, t.pool.cap);
            TZ.add(&t.pool.count, 1);
            TZ.add(&t.vx_big, 1);
            TT.add(&t.face_cnt, m.n);
            TT.add(&t.ecf, m.ncirc);
            TT.add(&t.ec_pos, m.ncirc + 1);
        }
        CKS(P.commit(c_->batch, st_, false));
        CKS(TT.commit(T_, st_, false));
        CKS(TZ.commit(T_, st_, true));
        size_t mo, to;
        StageCtl &C = begin(&mo, &to);
        Launch nf{BK_NBR, true, 0, 0}, ns{BK_NBR_SORT, false, 0, 0}, vx{BK_VERTEX, false, 0, 0},
            cf{BK_CIRCLE_FREE, false, 0, 0}, af{BK_ATOM_FEATURES, false, 0, 0},
            ef{BK_EC_FLAG, false, 0, 0};
        for (Launch *l : {&nf, &ns, &vx, &cf, &af, &ef}) l->off = starts(C, l->k, &l->nb);
        // the cover-order sort only where some atom's neighbours exceeded the
        // pool (the fill pass ranks the others)
        {
            std::vector<int> st((size_t)nm_ + 1, 0);
            long long t = 0;
            for (int q = 0; q < nm_; ++q) {
                st[(size_t)q] = (int)t;
                if (B[q].nnbr_big > 0) t += build_blocks(BK_NBR_SORT, M[q], B[q]);
            }
            st[(size_t)nm_] = (int)t;
            ns.nb = t;
            ns.off = C.put(st.data(), st.size());
        }
        ScanList S1, S2, S3;
        for (int q = 0; q < nm_; ++q) {
            S1.add(B[q].vcnt, M[q].vert_off, M[q].ncirc);
            S2.add(B[q].face_cnt, M[q].face_off_atom, M[q].n);
            S3.add(B[q].ecf, B[q].ec_pos, M[q].ncirc);
        }
        for (ScanList *S : {&S1, &S2, &S3}) {
            S->off = C.put(S->segs.data(), S->segs.size());
            CKS(T_.alloc(&S->sums, S->chunks + 1));
        }
        std::vector<const int *> addr;
        for (int q = 0; q < nm_; ++q) {
            addr.push_back(M[q].vert_off + M[q].ncirc);
            addr.push_back(M[q].face_off_atom + M[q].n);
            addr.push_back(B[q].ec_pos + M[q].ncirc);
            addr.push_back(B[q].pool.count);
            addr.push_back(B[q].vx_big);
        }
        const size_t ao = C.put(addr.data(), addr.size());
        int *rb;
        CKS(T_.alloc(&rb, (long long)addr.size()));
        CKS(C.upload(T_, st_));
        CK(launch_build_fill(BK_NBR, seg(C, mo, to, nf.off), nf.nb, st_));
        CK(launch_build(BK_NBR_SORT, seg(C, mo, to, ns.off), ns.nb, st_));
        CK(launch_build(BK_VERTEX, seg(C, mo, to, vx.off), vx.nb, st_));
        CK(launch_build(BK_CIRCLE_FREE, seg(C, mo, to, cf.off), cf.nb, st_));
        CKS(scan(C, S1));
        CK(launch_build(BK_ATOM_FEATURES, seg(C, mo, to, af.off), af.nb, st_));
        CKS(scan(C, S2));
        CK(launch_build(BK_EC_FLAG, seg(C, mo, to, ef.off), ef.nb, st_));
        CKS(scan(C, S3));
        std::vector<int> h;
        CKS(read_ints(C, ao, (int)addr.size(), rb, h));
        for (int q = 0; q < nm_; ++q) {
            M[q].nvert = h[(size_t)5 * q];
            M[q].nface = h[(size_t)5 * q + 1];
            M[q].nec = h[(size_t)5 * q + 2];
            B[q].npool = h[(size_t)5 * q + 3];
            B[q].pool.use = B[q].npool <= B[q].pool.cap ? 1 : 0;
            B[q].nvx_big = h[(size_t)5 * q + 4];
        }
        return ESES_OK;
    }

    // -- stage 3: probe positions, exposed features, cut and tile counts
    eses_status stage_tiles(int tile_pool) {
        Planner P, TT, TZ;
        for (int q = 0; q < nm_; ++q) {
            Mol &m = M[q];
            BuildTmp &t = B[q];
            P.add(&m.vert_p, m.nvert);
            P.add(&m.vert_ijks, m.nvert);
            P.add(&m.ec_circ, m.nec);
            P.add(&m.face_atom, m.nface);
            P.add(&m.face_cut_off, m.nface + 1);
            P.add(&m.ec_cut_off, m.nec + 1);
            P.add(&m.tA_off, m.ntiles + 1);
            P.add(&m.tF_off, m.ntiles + 1);
            P.add(&m.tC_off, m.ntiles + 1);
            P.add(&m.tV_off, m.ntiles + 1);
            TT.add(&t.fcut_cnt, m.nface);
            TT.add(&t.eccut_cnt, m.nec);
            TT.add(&t.fcut_keep, 2LL * m.nface);
            TT.add(&t.eccut_keep, m.nec);
            TT.add(&t.cA, m.ntiles);
            TT.add(&t.cF, m.ntiles);
            TT.add(&t.cC, m.ntiles);
            TT.add(&t.cV, m.ntiles);
            t.tp.cap = tile_pool > 0 ? std::min(tile_pool, tile_keep_max()) : tile_keep_max();
            TT.add(&t.tp.pool, (long long)t.tp.cap * m.ntiles);
            TT.add(&t.tp.off, m.ntiles);
            TZ.add(&t.tp.unpooled, 1);
        }
        CKS(P.commit(c_->batch, st_, false));
        CKS(TT.commit(T_, st_, false));
        CKS(TZ.commit(T_, st_, true));
        size_t mo, to;
        StageCtl &C = begin(&mo, &to);
        Launch vp{BK_VERTEX_PLACE, false, 0, 0}, vf{BK_VERTEX, true, 0, 0},
            vo{BK_VERTEX_ORDER, false, 0, 0}, ei{BK_EC_IDS, false, 0, 0},
            fo{BK_FEATURE_OFF, false, 0, 0}, fl{BK_FACE_LIST, false, 0, 0},
            fc{BK_FACE_CUTS, false, 0, 0}, ec{BK_EC_CUTS, false, 0, 0},
            ti{BK_TILES, false, 0, 0};
        for (Launch *l : {&vp, &vf, &vo, &ei, &fo, &fl, &fc, &ec, &ti})
            l->off = starts(C, l->k, &l->nb);
        // the ordering pass only where the positions were pooled, the fill
        // pass only where some were not
        {
            std::vector<int> st((size_t)nm_ + 1, 0), sf((size_t)nm_ + 1, 0);
            long long t = 0, tf = 0;
            for (int q = 0; q < nm_; ++q) {
                st[(size_t)q] = (int)t;
                sf[(size_t)q] = (int)tf;
                if (B[q].pool.use) t += build_blocks(BK_VERTEX_ORDER, M[q], B[q]);
                if (!B[q].pool.use || B[q].nvx_big > 0) tf += build_blocks(BK_VERTEX, M[q], B[q]);
            }
            st[(size_t)nm_] = (int)t;
            sf[(size_t)nm_] = (int)tf;
            vo.nb = t;
            vo.off = C.put(st.data(), st.size());
            vf.nb = tf;
            vf.off = C.put(sf.data(), sf.size());
        }
        ScanList S1, S2, S3;
        for (int q = 0; q < nm_; ++q) {
            S1.add(B[q].fcut_cnt, M[q].face_cut_off, M[q].nface);
            S2.add(B[q].eccut_cnt, M[q].ec_cut_off, M[q].nec);
            S3.add(B[q].cA, M[q].tA_off, M[q].ntiles);
            S3.add(B[q].cF, M[q].tF_off, M[q].ntiles);
            S3.add(B[q].cC, M[q].tC_off, M[q].ntiles);
            S3.add(B[q].cV, M[q].tV_off, M[q].ntiles);
        }
        for (ScanList *S : {&S1, &S2, &S3}) {
            S->off = C.put(S->segs.data(), S->segs.size());
            CKS(T_.alloc(&S->sums, S->chunks + 1));
        }
        std::vector<const int *> addr;
        for (int q = 0; q < nm_; ++q) {
            addr.push_back(M[q].face_cut_off + M[q].nface);
            addr.push_back(M[q].ec_cut_off + M[q].nec);
            addr.push_back(M[q].tA_off + M[q].ntiles);
            addr.push_back(M[q].tF_off + M[q].ntiles);
            addr.push_back(M[q].tC_off + M[q].ntiles);
            addr.push_back(M[q].tV_off + M[q].ntiles);
            addr.push_back(B[q].tp.unpooled);
        }
        const size_t ao = C.put(addr.data(), addr.size());
        int *rb;
        CKS(T_.alloc(&rb, (long long)addr.size()));
        CKS(C.upload(T_, st_));
        CK(launch_build(BK_VERTEX_PLACE, seg(C, mo, to, vp.off), vp.nb, st_));
        CK(launch_build_fill(BK_VERTEX, seg(C, mo, to, vf.off), vf.nb, st_));
        CK(launch_build(BK_VERTEX_ORDER, seg(C, mo, to, vo.off), vo.nb, st_));
        CK(launch_build(BK_EC_IDS, seg(C, mo, to, ei.off), ei.nb, st_));
        CK(launch_build(BK_FEATURE_OFF, seg(C, mo, to, fo.off), fo.nb, st_));
        CK(launch_build(BK_FACE_LIST, seg(C, mo, to, fl.off), fl.nb, st_));
        CK(launch_build(BK_FACE_CUTS, seg(C, mo, to, fc.off), fc.nb, st_));  // counts
        CKS(scan(C, S1));
        CK(launch_build(BK_EC_CUTS, seg(C, mo, to, ec.off), ec.nb, st_));
        CKS(scan(C, S2));
        CK(launch_build(BK_TILES, seg(C, mo, to, ti.off), ti.nb, st_));
        CKS(scan(C, S3));
        std::vector<int> h;
        CKS(read_ints(C, ao, (int)addr.size(), rb, h));
        for (int q = 0; q < nm_; ++q) {
            const int *v = &h[(size_t)7 * q];
            nfc_.push_back(v[0]);
            necc_.push_back(v[1]);
            for (int k = 0; k < 4; ++k) tl_.push_back(v[2 + k]);
            B[q].tp_unpooled = v[6];
            eses_candidate_stats &s = c_->mols[q]->stats;
            const Mol &m = M[q];
            s.n_atoms = m.n;
            for (int a = 0; a < 3; ++a) s.dims[a] = m.dims[a];
            s.n_points = m.npts;
            s.n_neighbour_pairs = nbr_total_[(size_t)q];
            s.n_circles = m.ncirc;
            s.n_vertices = m.nvert;
            s.n_exposed_faces = m.nface;
            s.n_exposed_circles = m.nec;
            s.n_tiles = m.ntiles;
            s.tile_list_entries = (int64_t)v[2] + v[3] + v[4] + v[5];
        }
        return ESES_OK;
    }
    std::vector<int> nfc_, necc_, tl_;

    // -- stage 4: cut lists and tile lists
    eses_status stage_fill() {
        Planner P;
        for (int q = 0; q < nm_; ++q) {
            Mol &m = M[q];
            P.add(&m.face_cut, nfc_[(size_t)q]);
            P.add(&m.ec_cut, necc_[(size_t)q]);
            P.add(&m.tA, tl_[(size_t)4 * q]);
            P.add(&m.tF, tl_[(size_t)4 * q + 1]);
            P.add(&m.tC, tl_[(size_t)4 * q + 2]);
            P.add(&m.tV, tl_[(size_t)4 * q + 3]);
        }
        CKS(P.commit(c_->batch, st_, false));
        size_t mo, to;
        StageCtl &C = begin(&mo, &to);
        Launch fc{BK_FACE_CUTS, true, 0, 0}, ec{BK_EC_CUTS, true, 0, 0},
            tp{BK_TILES_PLACE, false, 0, 0}, tf{BK_TILES_FILL, false, 0, 0};
        for (Launch *l : {&fc, &ec, &tp, &tf}) l->off = starts(C, l->k, &l->nb);
        CKS(C.upload(T_, st_));
        CK(launch_build_fill(BK_FACE_CUTS, seg(C, mo, to, fc.off), fc.nb, st_));
        CK(launch_build_fill(BK_EC_CUTS, seg(C, mo, to, ec.off), ec.nb, st_));
        CK(launch_build(BK_TILES_PLACE, seg(C, mo, to, tp.off), tp.nb, st_));
        CK(launch_build(BK_TILES_FILL, seg(C, mo, to, tf.off), tf.nb, st_));
        // (a fill pass that met more entries than it counted sets diag[0],
        // checked at the next read-back: eses_edge_intersections)
        return ESES_OK;
    }
};

eses_status ensure_events(eses_candidates *c) {
    for (int q = 0; q < 6; ++q)
        if (!c->ev[q]) CK(hipEventCreate(&c->ev[q]));
    return ESES_OK;
}

// Device copies of the molecules' views and the heaviest-first list of
// (molecule, tile) units for the fused classification launch.
eses_status build_batch(eses_candidates *c, hipStream_t st) {
    Arena &B = c->batch;
    B.st = st;
    const int nm = (int)c->mols.size();
    std::vector<Mol> hm(nm);
    std::vector<int> base(nm + 1, 0);
    for (int q = 0; q < nm; ++q) {
        hm[q] = c->mols[q]->m;
        base[q + 1] = base[q] + hm[q].ntiles;
    }
    if ((long long)base[nm] > (1LL << 30)) {
        set_err("batch too large: %d tiles", base[nm]);
        return ESES_EINVAL;
    }
    c->nunits = base[nm];
    CKS(B.alloc(&c->mols_dev, nm));
    CKS(B.alloc(&c->tile_base_dev, nm + 1));
    CKS(B.alloc(&c->units, c->nunits));
    CKS(B.alloc(&c->cls, 2 * UNIT_CLASSES));
    CKS(B.alloc(&c->head, 1));
    CKS(B.alloc(&c->labels_dev, nm));
    CK(hipMemcpyAsync(c->mols_dev, hm.data(), sizeof(Mol) * nm, hipMemcpyHostToDevice, st));
    CK(hipMemcpyAsync(c->tile_base_dev, base.data(), sizeof(int) * (nm + 1),
                      hipMemcpyHostToDevice, st));
    CK(launch_units(c->mols_dev, c->tile_base_dev, nm, c->nunits, c->unit_order, c->cls,
                    c->cls + UNIT_CLASSES, c->units, st));
    CK(hipStreamSynchronize(st));  // host arrays above are released on return
    int dev = 0, ncu = 0;
    CK(hipGetDevice(&dev));
    CK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    for (int k = 0; k < 2; ++k) {
        const int per =
            c->blocks_per_cu > 0 ? c->blocks_per_cu : classify_batch_blocks_per_cu(k == 1);
        c->batch_blocks[k] = std::max(1, ncu * per);
    }
    return ESES_OK;
}

// The fused classification of a batch, recorded once per precision on a
// private stream and replayed on the caller's.
eses_status classify_batch(eses_candidates *c, bool fp32, uint8_t *const *labels,
                           hipStream_t st) {
    const int nm = (int)c->mols.size();
    CK(hipMemcpyAsync(c->labels_dev, labels, sizeof(uint8_t *) * nm, hipMemcpyHostToDevice, st));
    const int k = fp32 ? 1 : 0;
    if (!c->exec[k]) {
        hipStream_t cap;
        CK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
        hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess)
            e = launch_classify_batch(c->mols_dev, nm, c->labels_dev, c->units, (int)c->nunits,
                                      c->head, c->batch_blocks[fp32 ? 1 : 0], fp32, cap);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(cap, &g);
        if (e == hipSuccess) e = e2;
        if (e == hipSuccess) e = hipGraphInstantiate(&c->exec[k], g, nullptr, nullptr, 0);
        (void)hipStreamDestroy(cap);
        if (e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            c->exec[k] = nullptr;
            set_err("recording the fused classification failed: %s", hipGetErrorString(e));
            return ESES_EDEVICE;
        }
        c->graph[k] = g;
    }
    CK(hipGraphLaunch(c->exec[k], st));
    return ESES_OK;
}

// Host copies of one molecule's atoms (the caller's device inputs, in caller
// order) and concave probe list, and the exact arbiter built on them.
eses_status exact_arbiter(MolState *S, hipStream_t st) {
    if (S->exact) return ESES_OK;
    const Mol &m = S->m;
    std::vector<double> c((size_t)3 * m.n), r((size_t)m.n);
    CK(hipMemcpyAsync(c.data(), m.in_c, sizeof(double) * c.size(), hipMemcpyDeviceToHost, st));
    CK(hipMemcpyAsync(r.data(), m.in_r, sizeof(double) * r.size(), hipMemcpyDeviceToHost, st));
    std::vector<int32_t> pa((size_t)3 * std::max(m.nvert, 1));
    std::vector<int8_t> ps((size_t)std::max(m.nvert, 1));
    if (m.nvert > 0) {
        Arena T;
        T.st = st;
        double *dp;
        int *da;
        int8_t *dsg;
        eses_status s;
        if ((s = T.alloc(&dp, 3LL * m.nvert)) != ESES_OK || (s = T.alloc(&da, 3LL * m.nvert)) != ESES_OK ||
            (s = T.alloc(&dsg, m.nvert)) != ESES_OK) {
            T.release();
            return s;
        }
        hipError_t e = launch_export_vertices(m, dp, da, dsg, m.nvert, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(pa.data(), da, sizeof(int32_t) * 3 * m.nvert, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(ps.data(), dsg, sizeof(int8_t) * m.nvert, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        T.release();
        if (e != hipSuccess) {
            set_err("exact arbiter: %s", hipGetErrorString(e));
            return ESES_EDEVICE;
        }
    } else {
        CK(hipStreamSynchronize(st));
    }
    S->exact.reset(new eses::ExactMolecule(c.data(), r.data(), m.n, m.rho, pa.data(), ps.data(),
                                           m.nvert));
    return ESES_OK;
}

// Grid point coordinate fl(lo + fl(i h)) on the host: two rounded operations,
// kept apart so that they are not contracted into a fused multiply-add.
double host_grid_coord(double lo, double h, long long i) {
    volatile double ih = (double)i * h;
    return lo + ih;
}

// The exact re-decision of the points the classification left uncertain
// (their FP64 margins within the rounding bound): counts read back (one
// synchronisation), each molecule with uncertain points re-decided on the
// host and the labels written back.  A queue that overflowed is grown and the
// molecule classified again.
eses_status arbitrate(eses_candidates *c, bool fp32, uint8_t *const *labels, hipStream_t st) {
    const int nm = (int)c->mols.size();
    std::vector<int> cnt((size_t)nm, 0);
    if (nm == 1) {
        long long v = 0;
        CKS(read_scalars({{c->mols[0]->m.unc_n, false, &v}}, st));
        cnt[0] = (int)v;
    } else {
        if (!c->unc_counts) CKS(c->batch.alloc(&c->unc_counts, nm));
        CK(launch_unc_gather(c->mols_dev, nm, c->unc_counts, st));
        CK(hipMemcpyAsync(cnt.data(), c->unc_counts, sizeof(int) * nm, hipMemcpyDeviceToHost, st));
        CK(hipStreamSynchronize(st));
    }
    for (int q = 0; q < nm; ++q) {
        MolState *S = c->mols[q];
        Mol &m = S->m;
        S->n_exact = cnt[q];
        if (cnt[q] == 0) continue;
        if (cnt[q] > m.unc_cap) {
            // grow the queue and classify this molecule again
            m.unc_cap = cnt[q];
            CKS(S->arena.alloc(&m.unc_idx, m.unc_cap));
            if (nm > 1)
                CK(hipMemcpyAsync(c->mols_dev + q, &m, sizeof(Mol), hipMemcpyHostToDevice, st));
            CK(fill_i32(m.unc_n, 1, 0, st));
            CK(launch_classify(m, fp32, labels[q], st));
            long long v = 0;
            CKS(read_scalars({{m.unc_n, false, &v}}, st));
            if (v != cnt[q]) {
                set_err("internal: uncertain points changed between identical classifications");
                return ESES_EINTERNAL;
            }
        }
        const int n = cnt[q];
        std::vector<long long> idx((size_t)n);
        CK(hipMemcpyAsync(idx.data(), m.unc_idx, sizeof(long long) * n, hipMemcpyDeviceToHost, st));
        CKS(exact_arbiter(S, st));  // synchronises
        std::vector<uint8_t> val((size_t)n);
        const long long nx = m.dims[0], ny = m.dims[1];
        for (int k = 0; k < n; ++k) {
            const long long g = idx[(size_t)k];
            const double x[3] = {host_grid_coord(m.lo[0], m.h, g % nx),
                                 host_grid_coord(m.lo[1], m.h, (g / nx) % ny),
                                 host_grid_coord(m.lo[2], m.h, g / (nx * ny) + m.kz0)};
            val[(size_t)k] = (uint8_t)S->exact->label(x);
        }
        Arena T;
        T.st = st;
        long long *didx;
        uint8_t *dval;
        eses_status s;
        if ((s = T.alloc(&didx, n)) != ESES_OK || (s = T.alloc(&dval, n)) != ESES_OK) {
            T.release();
            return s;
        }
        hipError_t e = hipMemcpyAsync(didx, idx.data(), sizeof(long long) * n,
                                      hipMemcpyHostToDevice, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(dval, val.data(), (size_t)n, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = launch_scatter_labels(didx, dval, n, labels[q], st);
        // the host arrays are released on return
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        T.release();
        if (e != hipSuccess) {
            set_err("exact arbitration: %s", hipGetErrorString(e));
            return ESES_EDEVICE;
        }
    }
    return ESES_OK;
}

// Stage 3 for molecule q on stream st: crossing edges, grouping, roots.
// counts[q] receives the number of crossing edges.  With `timed` the
// handle's events bracket the kernels and their times are added up.
// Molecule q's crossing edges found, keyed into the output and grouped by
// tile (the root kernels' input, in P.job; its workspace stays in P.T until
// released).  With `timed`, HIP events bracket the detection and grouping.
struct EdgePrep {
    Arena T;
    EdgeJob job{};
    long long total = 0, nw = 0;
    int *ovf = nullptr;
};

eses_status edges_prepare(eses_candidates *c, size_t q, const uint8_t *lab,
                          const eses_isect_soa &o, EdgePrep &P, hipStream_t st, bool timed,
                          bool batch) {
    const Mol &m = c->mols[q]->m;
    Arena &T = P.T;
    T.st = st;
    long long nb = edge_detect_blocks(m);
    int *bcount;
    long long *boff, *tmp;
    eses_status s;
    if ((s = T.alloc(&bcount, nb + 1)) != ESES_OK || (s = T.alloc(&boff, nb + 2)) != ESES_OK ||
        (s = T.alloc(&tmp, scan_tmp_elems(nb) + 64)) != ESES_OK ||
        (s = T.alloc(&P.ovf, 1)) != ESES_OK)
        return s;
    long long nblk = 0;
    hipError_t e = timed ? hipEventRecord(c->ev[2], st) : hipSuccess;
    if (e == hipSuccess) e = launch_edge_detect_count(lab, m, bcount, &nblk, st);
    if (e == hipSuccess) e = scan_i64(bcount, nblk, boff, tmp, st);
    long long fill_overflow = 0;
    if (e == hipSuccess) {
        eses_status rs =
            read_scalars({{boff + nblk, true, &P.total}, {m.diag, false, &fill_overflow}}, st);
        if (rs == ESES_OK && fill_overflow != 0) {
            set_err("internal: %lld candidate list entries beyond their counted range",
                    fill_overflow);
            rs = ESES_EINTERNAL;
        }
        if (rs != ESES_OK) return rs;
    }
    const long long nw = P.nw = std::min<long long>(P.total, o.capacity);
    EdgeJob &J = P.job;
    int *tcount = nullptr, *ccount = nullptr, *coff = nullptr, *rank = nullptr,
        *order = nullptr, *units = nullptr, *ttmp = nullptr, *fb = nullptr, *nfb = nullptr;
    if (e == hipSuccess && nw > 0) {
        if ((s = T.alloc(&tcount, m.ntiles + 1)) != ESES_OK ||
            (s = T.alloc(&ccount, m.ntiles + 1)) != ESES_OK ||
            (s = T.alloc(&coff, m.ntiles + 1)) != ESES_OK ||
            (s = T.alloc(&rank, nw)) != ESES_OK ||
            (s = T.alloc(&order, edge_order_capacity(m, nw))) != ESES_OK ||
            (s = T.alloc(&units, edge_units_capacity(m))) != ESES_OK ||
            (s = T.alloc(&fb, nw)) != ESES_OK || (s = T.alloc(&nfb, 1)) != ESES_OK ||
            (s = T.alloc(&ttmp, scan_tmp_elems(m.ntiles) + 64)) != ESES_OK)
            return s;
    }
    if (e == hipSuccess && nw > 0)
        e = launch_edge_detect_write(lab, m, boff, o.capacity, (long long *)o.key, tcount, rank,
                                     st);
    if (e == hipSuccess) e = fill_i32(P.ovf, 1, 0, st);
    if (e == hipSuccess) e = fill_i32(m.diag + 3, 1, 0, st);  // ownerless records
    if (e == hipSuccess && nw > 0 && batch) e = fill_i32(nfb, 1, 0, st);  // fused launch
    if (e == hipSuccess && nw > 0)
        e = launch_edge_group(m, (const long long *)o.key, nw, tcount, ccount, coff, rank,
                              order, units, ttmp, st);
    if (e == hipSuccess && timed) e = hipEventRecord(c->ev[3], st);
    if (e != hipSuccess) {
        set_err("edge intersections: %s", hipGetErrorString(e));
        return ESES_EDEVICE;
    }
    J.L = dev(lab);
    J.keys = dev((const long long *)o.key);
    J.order = dev(order);
    J.tcount = dev(tcount);
    J.coff = dev(coff);
    J.units = dev(units);
    J.lam = dev(o.lambda);
    J.nrm = dev(o.normal);
    J.ptype = dev(o.patch_type);
    J.patoms = dev(o.atoms);
    J.fallback = dev(fb);
    J.nfallback = dev(nfb);
    J.mol = (int)q;
    return ESES_OK;
}

eses_status edges_one(eses_candidates *c, size_t q, const uint8_t *lab, const eses_isect_soa &o,
                      int64_t *counts, hipStream_t st, bool timed, char *carve = nullptr,
                      size_t carve_cap = 0) {
    const Mol &m = c->mols[q]->m;
    EdgePrep P;
    P.T.carve = carve;  // temporaries cut from a static region instead of allocated
    P.T.carve_cap = carve_cap;
    eses_status s = edges_prepare(c, q, lab, o, P, st, timed, false);
    if (s != ESES_OK) {
        P.T.release();
        return s;
    }
    const EdgeJob &J = P.job;
    hipError_t e = timed ? hipEventRecord(c->ev[4], st) : hipSuccess;
    if (e == hipSuccess && P.nw > 0)
        e = launch_edge_roots(m, lab, J.keys, P.nw, J.order, J.tcount, J.coff, (int *)J.units,
                              J.lam, J.nrm, J.ptype, J.patoms, J.fallback, J.nfallback, P.ovf,
                              st);
    if (e == hipSuccess && timed) e = hipEventRecord(c->ev[5], st);
    long long hovf = 0, hown = 0;
    if (e == hipSuccess) {
        eses_status rs = read_scalars({{P.ovf, false, &hovf}, {m.diag + 3, false, &hown}}, st);
        if (rs != ESES_OK) {
            P.T.release();
            return rs;
        }
    }
    if (e == hipSuccess && timed) {
        float a = 0.0f, b = 0.0f;
        e = hipEventElapsedTime(&a, c->ev[2], c->ev[3]);
        if (e == hipSuccess) e = hipEventElapsedTime(&b, c->ev[4], c->ev[5]);
        c->detect_ms += a;
        c->roots_ms += b;
    }
    P.T.release();
    if (e != hipSuccess) {
        set_err("edge intersections: %s", hipGetErrorString(e));
        return ESES_EDEVICE;
    }
    if (hovf) {
        set_err("more roots on one edge than the per-edge list holds");
        return ESES_EINTERNAL;
    }
    if (hown) {
        set_err("internal: %lld crossing edges whose label change no surface root explains",
                hown);
        return ESES_EINTERNAL;
    }
    counts[q] = P.total;
    return ESES_OK;
}

// Host side of the batched crossing-edge passes: the control images and the
// per-molecule results (kept until the stream has passed them).
struct EdgeBatchPrep {
    StageCtl ctl1, ctl2;
    std::vector<long long> total, nw;
    std::vector<EdgeJob> job;
};

// Whether every molecule's crossing edges can take the batched passes (edge
// offsets within a molecule, and the passes' block counts, fit an int).
bool edges_batchable(const eses_candidates *c) {
    long long blocks = 0;
    for (const auto &mp : c->mols) {
        const Mol &m = mp->m;
        if (3 * m.npts >= (1LL << 31) - 1) return false;
        blocks += edge_detect_blocks(m);
    }
    return blocks < (1LL << 31) - 1;
}

// Every molecule's crossing edges found, keyed and grouped by tile with one
// launch per pass over the whole batch and one read-back of the totals
// (see edges_batchable); P.job[q] is molecule q's job of the fused root
// launch when P.nw[q] > 0.  W holds the workspace.
eses_status edges_detect_batch(eses_candidates *c, const uint8_t *const *labels,
                               const eses_isect_soa *out, Arena &W, EdgeBatchPrep &P,
                               hipStream_t st) {
    const int nm = (int)c->mols.size();
    P.total.assign((size_t)nm, 0);
    P.nw.assign((size_t)nm, 0);
    P.job.assign((size_t)nm, EdgeJob{});
    std::vector<EdgeDetectJob> J((size_t)nm);
    std::vector<long long> nblk((size_t)nm);
    std::vector<int> sdet((size_t)nm + 1, 0);
    // pass 1: per-block counts and their scans, the totals read back
    const long long chunk = scan_seg_chunk();
    Planner A;
    std::vector<long long> c1((size_t)nm);
    long long nch1 = 0;
    for (int q = 0; q < nm; ++q) {
        const Mol &m = c->mols[q]->m;
        nblk[q] = edge_detect_blocks(m);
        sdet[q + 1] = sdet[q] + (int)nblk[q];
        c1[q] = nch1;
        nch1 += (nblk[q] + chunk - 1) / chunk;
        J[q] = EdgeDetectJob{};
        J[q].L = dev(labels[q]);
        A.add(&J[q].bcount, nblk[q]);
        A.add(&J[q].boff, nblk[q] + 1);
    }
    int *sums1 = nullptr, *tot = nullptr;
    A.add(&sums1, nch1);
    A.add(&tot, 2LL * nm);
    CKS(A.commit(W, st, false));
    std::vector<ScanSeg> seg1((size_t)nm);
    std::vector<const int *> addr((size_t)nm);
    for (int q = 0; q < nm; ++q) {
        seg1[q] = ScanSeg{J[q].bcount, J[q].boff, nblk[q], c1[q]};
        addr[q] = J[q].boff + nblk[q];
    }
    StageCtl &C1 = P.ctl1;
    const size_t jo = C1.put(J.data(), J.size());
    const size_t so = C1.put(sdet.data(), sdet.size());
    const size_t go = C1.put(seg1.data(), seg1.size());
    const size_t ao = C1.put(addr.data(), addr.size());
    CKS(C1.upload(W, st));
    CK(launch_edge_detect_count_batch(c->mols_dev, C1.at<EdgeDetectJob>(jo), C1.at<int>(so),
                                      sdet.data(), nm, st));
    CK(scan_seg(C1.at<ScanSeg>(go), nm, nch1, sums1, st));
    CK(launch_gather_ints(C1.at<const int *>(ao), nm, tot, st));
    CK(launch_diag_gather(c->mols_dev, nm, 0, tot + nm, st));
    std::vector<int> htot((size_t)2 * nm);
    CK(hipMemcpyAsync(htot.data(), tot, sizeof(int) * 2 * nm, hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    for (int q = 0; q < nm; ++q)
        if (htot[(size_t)nm + q] != 0) {
            set_err("internal: molecule %d: %d candidate list entries beyond their counted range",
                    q, htot[(size_t)nm + q]);
            return ESES_EINTERNAL;
        }
    // pass 2: keys, tile tallies and ranks, grouping by tile
    Planner Z, N;  // zeroed (tile tallies, unit headers, fallback counts), not zeroed
    std::vector<int> sw((size_t)nm + 1, 0), stl((size_t)nm + 1, 0), sed((size_t)nm + 1, 0);
    std::vector<ScanSeg> seg2;
    long long nch2 = 0;
    std::vector<int *> fb((size_t)nm, nullptr), nfb((size_t)nm, nullptr);
    for (int q = 0; q < nm; ++q) {
        const Mol &m = c->mols[q]->m;
        P.total[q] = htot[q];
        const long long w = P.nw[q] = std::min<long long>(P.total[q], out[q].capacity);
        J[q].keys = dev((long long *)out[q].key);
        J[q].nw = w;
        sw[q + 1] = sw[q] + (w > 0 ? (int)nblk[q] : 0);
        stl[q + 1] = stl[q] + (w > 0 ? (m.ntiles + 255) / 256 : 0);
        sed[q + 1] = sed[q] + (int)((w + 255) / 256);
        if (w <= 0) continue;
        Z.add(&J[q].tcount, m.ntiles + 1);
        Z.add(&J[q].units, edge_units_capacity(m));
        Z.add(&nfb[q], 1);
        N.add(&J[q].ccount, m.ntiles + 1);
        N.add(&J[q].coff, m.ntiles + 1);
        N.add(&J[q].rank, w);
        N.add(&J[q].order, edge_order_capacity(m, w));
        N.add(&fb[q], w);
    }
    std::vector<long long> c2((size_t)nm, 0);
    for (int q = 0; q < nm; ++q)
        if (P.nw[q] > 0) {
            c2[q] = nch2;
            nch2 += (c->mols[q]->m.ntiles + chunk - 1) / chunk;
        }
    int *sums2 = nullptr;
    N.add(&sums2, nch2);
    CKS(Z.commit(W, st, true));
    CKS(N.commit(W, st, false));
    for (int q = 0; q < nm; ++q)
        if (P.nw[q] > 0) seg2.push_back({J[q].ccount, J[q].coff, c->mols[q]->m.ntiles, c2[q]});
    StageCtl &C2 = P.ctl2;
    const size_t jo2 = C2.put(J.data(), J.size());
    const size_t wo = C2.put(sw.data(), sw.size());
    const size_t to = C2.put(stl.data(), stl.size());
    const size_t eo = C2.put(sed.data(), sed.size());
    const size_t go2 = C2.put(seg2.data(), seg2.size());
    CKS(C2.upload(W, st));
    EdgeBatchStarts S{C2.at<int>(wo), C2.at<int>(to), C2.at<int>(eo), sw.data(), stl.data(),
                      sed.data()};
    const EdgeDetectJob *jd = C2.at<EdgeDetectJob>(jo2);
    CK(launch_edge_detect_write_batch(c->mols_dev, jd, S, nm, st));
    CK(launch_edge_group_batch(c->mols_dev, jd, S, C2.at<ScanSeg>(go2), (int)seg2.size(), nch2,
                               sums2, nm, st));
    for (int q = 0; q < nm; ++q) {
        if (P.nw[q] <= 0) continue;
        EdgeJob &E = P.job[q];
        E.L = dev(labels[q]);
        E.keys = J[q].keys;
        E.order = J[q].order;
        E.tcount = J[q].tcount;
        E.coff = J[q].coff;
        E.units = J[q].units;
        E.lam = dev(out[q].lambda);
        E.nrm = dev(out[q].normal);
        E.ptype = dev(out[q].patch_type);
        E.patoms = dev(out[q].atoms);
        E.fallback = dev(fb[q]);
        E.nfallback = dev(nfb[q]);
        E.mol = q;
    }
    return ESES_OK;
}

// A batch: every molecule's crossing edges found and grouped (one launch per
// pass over the whole batch, or per molecule on the worker streams where a
// grid is too large for the batched passes), then all their tiles in one
// fused root launch on `st` (molecules with most crossing edges first) and
// one read-back.
eses_status edges_batch(eses_candidates *c, const uint8_t *const *labels,
                        const eses_isect_soa *out, int64_t *counts, hipStream_t st,
                        bool timed) {
    const int nm = (int)c->mols.size();
    std::vector<EdgePrep> prep;
    EdgeBatchPrep bp;
    Arena W;  // the batched passes' workspace
    W.st = st;
    auto release_all = [&]() {
        for (EdgePrep &P : prep) P.T.release();
        W.release();
    };
    // with `timed`, events on `st` bracket the detection and grouping and
    // the fused root launch
    if (timed) CK(hipEventRecord(c->ev[2], st));
    eses_status s = ESES_OK;
    if (!c->edges_per_molecule && edges_batchable(c)) {
        s = edges_detect_batch(c, labels, out, W, bp, st);
    } else {
        prep.resize((size_t)nm);
        s = run_on_workers(nm, st, [&](int q, hipStream_t ws) {
            return edges_prepare(c, q, labels[q], out[q], prep[q], ws, false, true);
        });
        bp.total.resize((size_t)nm);
        bp.nw.resize((size_t)nm);
        bp.job.resize((size_t)nm);
        for (int q = 0; q < nm; ++q) {
            bp.total[q] = prep[q].total;
            bp.nw[q] = prep[q].nw;
            bp.job[q] = prep[q].job;
        }
    }
    if (s == ESES_OK && timed && hipEventRecord(c->ev[3], st) != hipSuccess) s = ESES_EDEVICE;
    if (s != ESES_OK) {
        // the prepared workspace may still be in use on the streams
        (void)hipStreamSynchronize(st);
        release_all();
        return s;
    }
    std::vector<int> ord;
    for (int q = 0; q < nm; ++q)
        if (bp.nw[q] > 0) ord.push_back(q);
    std::stable_sort(ord.begin(), ord.end(),
                     [&](int a, int b) { return bp.nw[a] > bp.nw[b]; });
    std::vector<EdgeJob> jobs;
    for (int q : ord) jobs.push_back(bp.job[q]);
    const int nj = (int)jobs.size();
    Arena B;
    B.st = st;
    EdgeJob *jobs_dev = nullptr;
    int *prefix = nullptr, *ctl = nullptr;
    long long hovf = 0;
    if ((s = B.alloc(&jobs_dev, nj)) != ESES_OK || (s = B.alloc(&prefix, nj + 1)) != ESES_OK ||
        (s = B.alloc(&ctl, 2)) != ESES_OK) {
        (void)hipStreamSynchronize(st);
        B.release();
        release_all();
        return s;
    }
    hipError_t e = hipSuccess;
    if (nj > 0)
        e = hipMemcpyAsync(jobs_dev, jobs.data(), sizeof(EdgeJob) * nj, hipMemcpyHostToDevice,
                           st);
    if (e == hipSuccess) e = fill_i32(ctl, 2, 0, st);
    if (e == hipSuccess && timed) e = hipEventRecord(c->ev[4], st);
    if (e == hipSuccess)
        e = launch_edge_roots_batch(c->mols_dev, jobs_dev, nj, prefix, ctl, ctl + 1, st);
    if (e == hipSuccess && timed) e = hipEventRecord(c->ev[5], st);
    std::vector<int> own((size_t)nm, 0);
    if (e == hipSuccess && !c->unc_counts) {
        s = c->batch.alloc(&c->unc_counts, nm);
        if (s != ESES_OK) e = hipErrorOutOfMemory;
    }
    if (e == hipSuccess) e = launch_diag_gather(c->mols_dev, nm, 3, c->unc_counts, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(own.data(), c->unc_counts, sizeof(int) * nm, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) s = read_scalars({{ctl + 1, false, &hovf}}, st);
    else (void)hipStreamSynchronize(st);
    if (e == hipSuccess && s == ESES_OK && timed) {
        float a = 0.0f, b = 0.0f;
        e = hipEventElapsedTime(&a, c->ev[2], c->ev[3]);
        if (e == hipSuccess) e = hipEventElapsedTime(&b, c->ev[4], c->ev[5]);
        c->detect_ms += a;
        c->roots_ms += b;
    }
    B.release();
    release_all();
    if (e != hipSuccess) {
        set_err("edge intersections: %s", hipGetErrorString(e));
        return ESES_EDEVICE;
    }
    if (s != ESES_OK) return s;
    if (hovf) {
        set_err("more roots on one edge than the per-edge list holds");
        return ESES_EINTERNAL;
    }
    for (int q = 0; q < nm; ++q)
        if (own[(size_t)q]) {
            set_err("internal: molecule %d: %d crossing edges whose label change no surface "
                    "root explains", q, own[(size_t)q]);
            return ESES_EINTERNAL;
        }
    for (int q = 0; q < nm; ++q) counts[q] = bp.total[q];
    return ESES_OK;
}

// Static device scratch of the allocation-free edge entry point: one copy per
// GPU, held until the process ends.  Host code never passes `scratch` itself
// (on the host it only names the symbol); the device address of each GPU's
// copy is looked up once, with that GPU current, and used instead.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;

}  // namespace

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {

eses_status scratch_address(char **out) {
    static std::mutex mu;
    static std::map<int, char *> addr;
    int dev = 0;
    CK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(mu);
    auto it = addr.find(dev);
    if (it == addr.end()) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            set_err("hipGetSymbolAddress of the static scratch failed: %s", hipGetErrorString(e));
            return ESES_EDEVICE;
        }
        it = addr.emplace(dev, (char *)p).first;
    }
    *out = it->second;
    return ESES_OK;
}

// Marks the calling thread as inside an allocation-free entry point.
struct NoAllocScope {
    NoAllocScope() { g_noalloc = true; }
    ~NoAllocScope() { g_noalloc = false; }
};

}  // namespace

extern "C" {

const char *eses_last_error(void) { return g_err.c_str(); }

const char *eses_version(void) { return "eses-gfx950 0.1"; }

eses_status eses_bbox_from_atoms(const double *c, const double *r, int64_t n, double margin,
                                 double lo[3], double hi[3]) {
    g_err.clear();
    if (!c || !r || !lo || !hi || n < 1 || !std::isfinite(margin) || margin < 0.0) {
        set_err("eses_bbox_from_atoms: bad argument");
        return ESES_EINVAL;
    }
    for (int a = 0; a < 3; ++a) {
        lo[a] = INFINITY;
        hi[a] = -INFINITY;
    }
    for (int64_t i = 0; i < n; ++i) {
        if (!std::isfinite(r[i]) || !(r[i] > 0.0) || !finite3(c + 3 * i)) {
            set_err("eses_bbox_from_atoms: atom %lld is not finite or has radius <= 0", (long long)i);
            return ESES_EINVAL;
        }
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::fmin(lo[a], c[3 * i + a] - r[i]);
            hi[a] = std::fmax(hi[a], c[3 * i + a] + r[i]);
        }
    }
    for (int a = 0; a < 3; ++a) {
        lo[a] -= margin;
        hi[a] += margin;
    }
    return ESES_OK;
}

eses_status eses_exact_labels(const double *centers, const double *radii, int64_t n_atoms,
                              double probe_radius, const int32_t *probe_atoms,
                              const int8_t *probe_sign, int64_t n_probes, const double *points,
                              int64_t n_points, uint8_t *labels) {
    g_err.clear();
    if (!centers || !radii || n_atoms < 1 || !(std::isfinite(probe_radius) && probe_radius > 0.0) ||
        n_probes < 0 || (n_probes > 0 && (!probe_atoms || !probe_sign)) || n_points < 0 ||
        (n_points > 0 && (!points || !labels))) {
        set_err("eses_exact_labels: bad argument");
        return ESES_EINVAL;
    }
    for (int64_t i = 0; i < n_atoms; ++i)
        if (!finite3(centers + 3 * i) || !std::isfinite(radii[i]) || !(radii[i] > 0.0)) {
            set_err("eses_exact_labels: atom %lld is not finite or has radius <= 0", (long long)i);
            return ESES_EINVAL;
        }
    for (int64_t v = 0; v < n_probes; ++v)
        for (int t = 0; t < 3; ++t)
            if (probe_atoms[3 * v + t] < 0 || probe_atoms[3 * v + t] >= n_atoms) {
                set_err("eses_exact_labels: probe %lld names no atom", (long long)v);
                return ESES_EINVAL;
            }
    for (int64_t q = 0; q < n_points; ++q)
        if (!finite3(points + 3 * q)) {
            set_err("eses_exact_labels: point %lld is not finite", (long long)q);
            return ESES_EINVAL;
        }
    eses::ExactMolecule em(centers, radii, n_atoms, probe_radius, probe_atoms, probe_sign,
                           n_probes);
    for (int64_t q = 0; q < n_points; ++q) labels[q] = (uint8_t)em.label(points + 3 * q);
    return ESES_OK;
}

eses_status eses_grid_dims(const eses_molecule *mol, int32_t dims[3]) {
    g_err.clear();
    if (!dims) {
        set_err("dims is NULL");
        return ESES_EINVAL;
    }
    return dims_of(mol, dims);
}

eses_status eses_build_candidates(const eses_molecule *mols, int32_t n_mols,
                                  const eses_config *cfg, void *stream, eses_candidates **out) {
    g_err.clear();
    if (!out) {
        set_err("out is NULL");
        return ESES_EINVAL;
    }
    *out = nullptr;
    if (!mols || n_mols < 1) {
        set_err("need at least one molecule");
        return ESES_EINVAL;
    }
    int tile = 8, force_recheck = 0, edge_fallback = 0, vertex_pool = 0, tile_pool = 0,
        unc_queue = 0;
    if (cfg) {
        if (cfg->tile != 0) tile = cfg->tile;
        force_recheck = cfg->force_recheck;
        edge_fallback = cfg->edge_fallback;
        vertex_pool = cfg->vertex_pool;
        tile_pool = cfg->tile_pool;
        if (cfg->blocks_per_cu < 0 || cfg->blocks_per_cu > 64) {
            set_err("blocks_per_cu must be in [0, 64]");
            return ESES_EINVAL;
        }
        if (vertex_pool < 0 || tile_pool < 0) {
            set_err("vertex_pool and tile_pool must be >= 0");
            return ESES_EINVAL;
        }
        if (cfg->unit_order != 0 && cfg->unit_order != 1) {
            set_err("unit_order must be 0 or 1");
            return ESES_EINVAL;
        }
        if (cfg->unc_queue < 0) {
            set_err("unc_queue must be >= 0");
            return ESES_EINVAL;
        }
        unc_queue = cfg->unc_queue;
        if (tile != 4 && tile != 8) {
            set_err("tile must be 4 or 8");
            return ESES_EINVAL;
        }
    }
    hipStream_t st = (hipStream_t)stream;
    eses_candidates *c = new eses_candidates();
    c->stream = st;
    for (int32_t q = 0; q < n_mols; ++q) c->mols.push_back(new MolState());
    for (MolState *S : c->mols) S->arena.st = st;
    {
        // every stage over all molecules from this thread (one launch per
        // build kernel and one read-back per stage)
        Builder b(c, mols, n_mols, st);
        eses_status s = b.run(tile, force_recheck, edge_fallback, vertex_pool, tile_pool,
                              unc_queue);
        if (s != ESES_OK) {
            std::string msg = g_err;
            (void)hipStreamSynchronize(st);  // the build's temporaries may still be in use
            eses_free_candidates(c);
            g_err = msg;
            return s;
        }
    }
    if (n_mols > 1) {
        c->blocks_per_cu = cfg ? cfg->blocks_per_cu : 0;
        c->unit_order = cfg ? cfg->unit_order : 0;
        c->edges_per_molecule = cfg ? cfg->edges_per_molecule : 0;
        eses_status s = build_batch(c, st);
        if (s != ESES_OK) {
            std::string msg = g_err;
            eses_free_candidates(c);
            g_err = msg;
            return s;
        }
    }
    *out = c;
    return ESES_OK;
}

eses_status eses_candidates_info(const eses_candidates *c, int32_t mol, eses_candidate_stats *st) {
    g_err.clear();
    if (!c || !st || mol < 0 || mol >= (int32_t)c->mols.size()) {
        set_err("bad handle, molecule index or stats pointer");
        return ESES_EINVAL;
    }
    *st = c->mols[mol]->stats;
    return ESES_OK;
}

eses_status eses_copy_vertices(const eses_candidates *c, int32_t mol, double *p, int32_t *atoms,
                               int8_t *sign, int64_t capacity, int64_t *count, void *stream) {
    g_err.clear();
    if (!c || mol < 0 || mol >= (int32_t)c->mols.size() || !count || capacity < 0 ||
        (capacity > 0 && (!p || !atoms || !sign))) {
        set_err("bad argument");
        return ESES_EINVAL;
    }
    hipStream_t st = (hipStream_t)stream;
    const Mol &m = c->mols[mol]->m;
    *count = m.nvert;
    long long nw = std::min<long long>(m.nvert, capacity);
    CK(launch_export_vertices(m, p, atoms, sign, nw, st));
    CK(hipStreamSynchronize(st));
    if (m.nvert > capacity) {
        set_err("capacity %lld below %d concave probe positions", (long long)capacity, m.nvert);
        return ESES_ECAPACITY;
    }
    return ESES_OK;
}

eses_status eses_classify(eses_candidates *c, eses_precision prec, uint8_t *const *labels,
                          eses_classify_stats *stats, void *stream) {
    g_err.clear();
    if (!c || !labels) {
        set_err("bad handle or labels");
        return ESES_EINVAL;
    }
    if (prec != ESES_FP64 && prec != ESES_FP32_RECHECK) {
        set_err("unknown precision");
        return ESES_EINVAL;
    }
    hipStream_t st = (hipStream_t)stream;
    for (size_t q = 0; q < c->mols.size(); ++q)
        if (!labels[q]) {
            set_err("labels[%zu] is NULL", q);
            return ESES_EINVAL;
        }
    if (stats)
        for (size_t q = 0; q < c->mols.size(); ++q) CK(fill_i32(c->mols[q]->m.diag + 1, 1, 0, st));
    const bool timed = g_timing.load() != 0;
    if (timed) {
        CKS(ensure_events(c));
        CK(hipEventRecord(c->ev[0], st));
    }
    if (c->mols.size() > 1) {
        CKS(classify_batch(c, prec == ESES_FP32_RECHECK, labels, st));
    } else {
        CK(fill_i32(c->mols[0]->m.unc_n, 1, 0, st));
        CK(launch_classify(c->mols[0]->m, prec == ESES_FP32_RECHECK, labels[0], st));
    }
    if (timed) {
        CK(hipEventRecord(c->ev[1], st));
        c->cls_timed = true;
    }
    CKS(arbitrate(c, prec == ESES_FP32_RECHECK, labels, st));
    if (stats) {
        const size_t nm = c->mols.size();
        const size_t per = 2 + WC_COUNT;
        unsigned long long *d = nullptr;
        CK(hipMallocAsync((void **)&d, sizeof(unsigned long long) * nm * per, st));
        std::vector<unsigned long long> h(nm * per);
        CK(fill_u32((uint32_t *)d, (long long)(2 * nm * per), 0u, st));
        std::vector<int> rechecked(nm);
        for (size_t q = 0; q < nm; ++q) {
            CK(launch_count_inside(labels[q], c->mols[q]->m.npts, d + q * per, st));
            CK(launch_classify_work(c->mols[q]->m, d + q * per + 2, st));
            CK(hipMemcpyAsync(&rechecked[q], c->mols[q]->m.diag + 1, sizeof(int),
                              hipMemcpyDeviceToHost, st));
        }
        CK(hipMemcpyAsync(h.data(), d, sizeof(unsigned long long) * h.size(), hipMemcpyDeviceToHost, st));
        CK(hipFreeAsync(d, st));
        CK(hipStreamSynchronize(st));
        for (size_t q = 0; q < nm; ++q) {
            const unsigned long long *w = h.data() + q * per;
            eses_classify_stats &o = stats[q];
            o.n_points = c->mols[q]->m.npts;
            o.n_inside = (int64_t)w[0];
            o.n_rechecked = rechecked[q];
            o.tests_atom = (int64_t)w[2 + WC_ATOM];
            o.tests_vertex = (int64_t)w[2 + WC_VERTEX];
            o.tests_face = (int64_t)w[2 + WC_FACE];
            o.tests_face_cut = (int64_t)w[2 + WC_FACE_CUT];
            o.tests_circle = (int64_t)w[2 + WC_CIRCLE];
            o.tests_circle_cut = (int64_t)w[2 + WC_CIRCLE_CUT];
            o.n_shell = (int64_t)w[2 + WC_CASE_SHELL];
            o.n_exact = c->mols[q]->n_exact;
        }
    }
    return ESES_OK;
}

eses_status eses_edge_intersections(eses_candidates *c, const uint8_t *const *labels,
                                    const eses_isect_soa *out, int64_t *counts, void *stream) {
    g_err.clear();
    if (!c || !labels || !out || !counts) {
        set_err("bad argument");
        return ESES_EINVAL;
    }
    hipStream_t st = (hipStream_t)stream;
    const bool timed = g_timing.load() != 0;
    if (timed) CKS(ensure_events(c));
    c->detect_ms = c->roots_ms = 0.0;
    const int nm = (int)c->mols.size();
    for (int q = 0; q < nm; ++q) {
        const eses_isect_soa &o = out[q];
        if (!labels[q] || o.capacity < 0 ||
            (o.capacity > 0 && (!o.key || !o.lambda || !o.normal || !o.patch_type || !o.atoms))) {
            set_err("molecule %d: bad labels or output descriptor", q);
            return ESES_EINVAL;
        }
    }
    if (nm == 1) {
        eses_status s = edges_one(c, 0, labels[0], out[0], counts, st, timed);
        if (s != ESES_OK) {
            g_err = "molecule 0: " + g_err;
            return s;
        }
    } else {
        CKS(edges_batch(c, labels, out, counts, st, timed));
    }
    for (int q = 0; q < nm; ++q)
        if (counts[q] > out[q].capacity) {
            set_err("an output capacity is below the number of crossing edges (see counts)");
            return ESES_ECAPACITY;
        }
    return ESES_OK;
}

eses_status eses_edge_intersections_noalloc(eses_candidates *c, const uint8_t *labels,
                                            const eses_isect_soa *out, int64_t *count,
                                            void *stream) {
    g_err.clear();
    if (!c || !labels || !out || !count) {
        set_err("bad argument");
        return ESES_EINVAL;
    }
    if (c->mols.size() != 1) {
        set_err("the allocation-free form takes a handle of one molecule");
        return ESES_EINVAL;
    }
    if (out->capacity < 0 || (out->capacity > 0 && (!out->key || !out->lambda || !out->normal ||
                                                    !out->patch_type || !out->atoms))) {
        set_err("bad output descriptor");
        return ESES_EINVAL;
    }
    char *base = nullptr;
    CKS(scratch_address(&base));
    hipStream_t st = (hipStream_t)stream;
    NoAllocScope scope;
    eses_status s = edges_one(c, 0, labels, *out, count, st, false, base, NOALLOC_SCRATCH_BYTES);
    if (s != ESES_OK) {
        // work queued before the failure may still use the scratch
        (void)hipStreamSynchronize(st);
        return s;
    }
    if (*count > out->capacity) {
        set_err("the output capacity is below the number of crossing edges (see count)");
        return ESES_ECAPACITY;
    }
    return ESES_OK;
}

// Out-of-core form: the grid in z-slabs of P planes (P a multiple of the tile
// edge).  A slab view of the molecule is the same candidate set with the
// grid cut to planes [k0, k1) plus one more (the z-edges of plane k1 - 1 end
// there), its tile lists starting at the slab's first tile layer and kz0 = k0,
// so that its points keep their coordinates.  Each slab is classified (with
// exact arbitration) and solved into one of two device buffers on `st`; its
// own planes' labels and its records below plane k1 - k0 (keys moved to the
// whole grid's numbering) are copied to the caller's host arrays on a second
// stream, overlapping the next slab's work.
eses_status eses_stream_slabs(eses_candidates *c, eses_precision prec, int32_t slab_planes,
                              uint8_t *labels_host, const eses_isect_soa *out_host,
                              int64_t *count, void *stream) {
    g_err.clear();
    if (!c || !labels_host || !out_host || !count) {
        set_err("bad argument");
        return ESES_EINVAL;
    }
    if (c->mols.size() != 1) {
        set_err("the slab form takes a handle of one molecule");
        return ESES_EINVAL;
    }
    if (prec != ESES_FP64 && prec != ESES_FP32_RECHECK) {
        set_err("unknown precision");
        return ESES_EINVAL;
    }
    const eses_isect_soa &oh = *out_host;
    if (oh.capacity < 0 || (oh.capacity > 0 && (!oh.key || !oh.lambda || !oh.normal ||
                                               !oh.patch_type || !oh.atoms))) {
        set_err("bad output descriptor");
        return ESES_EINVAL;
    }
    MolState *S = c->mols[0];
    const Mol M = S->m;
    const int T = M.tile;
    if (slab_planes < T || slab_planes % T != 0) {
        set_err("slab_planes must be a positive multiple of the tile edge (%d)", T);
        return ESES_EINVAL;
    }
    const bool fp32 = prec == ESES_FP32_RECHECK;
    hipStream_t st = (hipStream_t)stream;
    const long long nx = M.dims[0], ny = M.dims[1], nz = M.dims[2], plane = nx * ny;
    const long long P = std::min<long long>(slab_planes, nz);
    // restores the handle's own view (and keeps a grown uncertain-point queue)
    struct ViewGuard {
        MolState *S;
        Mol M;
        ~ViewGuard() {
            M.unc_idx = S->m.unc_idx;
            M.unc_cap = S->m.unc_cap;
            S->m = M;
        }
    } guard{S, M};
    Arena A;
    A.st = st;
    hipStream_t cs = nullptr;
    hipEvent_t ready = nullptr, copied[2] = {nullptr, nullptr};
    auto cleanup = [&]() {
        if (cs) {
            (void)hipStreamSynchronize(cs);
            (void)hipStreamDestroy(cs);
        }
        if (ready) (void)hipEventDestroy(ready);
        for (hipEvent_t &e : copied)
            if (e) (void)hipEventDestroy(e);
        A.release();
    };
    eses_status res = ESES_OK;
    auto fail = [&](eses_status s) {
        res = s;
        cleanup();
        return s;
    };
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ready, hipEventDisableTiming);
    for (hipEvent_t &ev : copied)
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) {
        set_err("slab streams: %s", hipGetErrorString(e));
        return fail(ESES_EDEVICE);
    }
    uint8_t *lab[2];
    long long *nown_dev;
    eses_status s;
    if ((s = A.alloc(&lab[0], plane * (P + 1))) != ESES_OK ||
        (s = A.alloc(&lab[1], plane * (P + 1))) != ESES_OK || (s = A.alloc(&nown_dev, 1)) != ESES_OK)
        return fail(s);
    eses_isect_soa od[2] = {};
    auto grow = [&](eses_isect_soa &o, long long cap) -> eses_status {
        eses_status r;
        if ((r = A.alloc(&o.key, cap)) != ESES_OK || (r = A.alloc(&o.lambda, cap)) != ESES_OK ||
            (r = A.alloc(&o.normal, 3 * cap)) != ESES_OK ||
            (r = A.alloc(&o.patch_type, cap)) != ESES_OK || (r = A.alloc(&o.atoms, 3 * cap)) != ESES_OK)
            return r;
        o.capacity = cap;
        return ESES_OK;
    };
    long long pos = 0;
    for (long long k0 = 0, si = 0; k0 < nz; k0 += P, ++si) {
        const int b = (int)(si & 1);
        const long long k1 = std::min(nz, k0 + P);
        // buffer b is free once the copies of slab si - 2 are done
        if (si >= 2 && hipStreamWaitEvent(st, copied[b], 0) != hipSuccess) {
            set_err("slab streams: wait failed");
            return fail(ESES_EDEVICE);
        }
        Mol V = M;
        V.unc_idx = S->m.unc_idx;
        V.unc_cap = S->m.unc_cap;
        V.kz0 = M.kz0 + (int)k0;
        V.dims[2] = (int)(k1 - k0 + (k1 < nz ? 1 : 0));
        V.npts = plane * V.dims[2];
        const long long tz0 = k0 / T;
        V.tdims[2] = (V.dims[2] + T - 1) / T;
        V.ntiles = V.tdims[0] * V.tdims[1] * V.tdims[2];
        const long long t0 = tz0 * (long long)M.tdims[0] * M.tdims[1];
        V.tA_off = M.tA_off + t0;
        V.tF_off = M.tF_off + t0;
        V.tC_off = M.tC_off + t0;
        V.tV_off = M.tV_off + t0;
        S->m = V;
        // classification of the slab (and exact arbitration)
        e = fill_i32(V.unc_n, 1, 0, st);
        if (e == hipSuccess) e = launch_classify(V, fp32, lab[b], st);
        if (e != hipSuccess) {
            set_err("slab classification: %s", hipGetErrorString(e));
            return fail(ESES_EDEVICE);
        }
        uint8_t *lb = lab[b];
        if ((s = arbitrate(c, fp32, &lb, st)) != ESES_OK) return fail(s);
        // crossing edges of the slab view, into device buffer b
        if (od[b].capacity == 0 && (s = grow(od[b], std::max<long long>(4096, plane))) != ESES_OK)
            return fail(s);
        int64_t cnt = 0;
        if ((s = edges_one(c, 0, lb, od[b], &cnt, st, false)) != ESES_OK) return fail(s);
        if (cnt > od[b].capacity) {
            if ((s = grow(od[b], cnt + cnt / 4)) != ESES_OK) return fail(s);
            if ((s = edges_one(c, 0, lb, od[b], &cnt, st, false)) != ESES_OK) return fail(s);
        }
        // records of the slab's own points, keyed in the whole grid
        long long n_own = 0;
        e = launch_slab_keys((long long *)od[b].key, cnt, 3 * plane * (k1 - k0), 3 * plane * k0,
                             nown_dev, st);
        if (e != hipSuccess) {
            set_err("slab keys: %s", hipGetErrorString(e));
            return fail(ESES_EDEVICE);
        }
        if ((s = read_scalars({{nown_dev, true, &n_own}}, st)) != ESES_OK) return fail(s);
        // copies to the host on the copy stream
        e = hipEventRecord(ready, st);
        if (e == hipSuccess) e = hipStreamWaitEvent(cs, ready, 0);
        if (e == hipSuccess)
            e = hipMemcpyAsync(labels_host + k0 * plane, lb, (size_t)(plane * (k1 - k0)),
                               hipMemcpyDeviceToHost, cs);
        const long long room = std::max<long long>(0, oh.capacity - pos);
        const long long nc = std::min(n_own, room);
        if (e == hipSuccess && nc > 0) {
            e = hipMemcpyAsync(oh.key + pos, od[b].key, sizeof(int64_t) * nc, hipMemcpyDeviceToHost, cs);
            if (e == hipSuccess)
                e = hipMemcpyAsync(oh.lambda + pos, od[b].lambda, sizeof(double) * nc,
                                   hipMemcpyDeviceToHost, cs);
            if (e == hipSuccess)
                e = hipMemcpyAsync(oh.normal + 3 * pos, od[b].normal, sizeof(double) * 3 * nc,
                                   hipMemcpyDeviceToHost, cs);
            if (e == hipSuccess)
                e = hipMemcpyAsync(oh.patch_type + pos, od[b].patch_type, nc,
                                   hipMemcpyDeviceToHost, cs);
            if (e == hipSuccess)
                e = hipMemcpyAsync(oh.atoms + 3 * pos, od[b].atoms, sizeof(int32_t) * 3 * nc,
                                   hipMemcpyDeviceToHost, cs);
        }
        if (e == hipSuccess) e = hipEventRecord(copied[b], cs);
        if (e != hipSuccess) {
            set_err("slab copies: %s", hipGetErrorString(e));
            return fail(ESES_EDEVICE);
        }
        pos += n_own;
    }
    if (hipStreamSynchronize(cs) != hipSuccess) {
        set_err("slab copies failed");
        return fail(ESES_EDEVICE);
    }
    cleanup();
    *count = pos;
    if (pos > oh.capacity) {
        set_err("the output capacity is below the number of crossing edges (see count)");
        return ESES_ECAPACITY;
    }
    return res;
}

eses_status eses_mesh(eses_candidates *c, const uint8_t *const *labels,
                      const eses_isect_soa *isect, const int64_t *counts,
                      int32_t *const *triangles, const int64_t *tri_capacity,
                      eses_mesh_stats *stats, void *stream) {
    g_err.clear();
    if (!c || !labels || !isect || !counts || !stats || (triangles && !tri_capacity)) {
        set_err("bad argument");
        return ESES_EINVAL;
    }
    const int nm = (int)c->mols.size();
    hipStream_t st = (hipStream_t)stream;
    bool short_cap = false;
    for (int q = 0; q < nm; ++q) {
        const Mol &m = c->mols[q]->m;
        if (!labels[q] || counts[q] < 0 || counts[q] > isect[q].capacity ||
            (counts[q] > 0 && (!isect[q].key || !isect[q].lambda))) {
            set_err("molecule %d: labels or records missing (count beyond capacity?)", q);
            return ESES_EINVAL;
        }
        Arena T;
        T.st = st;
        double *out;
        int *cnt, *bad;
        long long *boff, *tmp;
        const long long nb = (m.npts + 255) / 256;
        eses_status s;
        if ((s = T.alloc(&out, 2 * nb + 2)) != ESES_OK || (s = T.alloc(&cnt, nb + 1)) != ESES_OK ||
            (s = T.alloc(&bad, 1)) != ESES_OK || (s = T.alloc(&boff, nb + 2)) != ESES_OK ||
            (s = T.alloc(&tmp, scan_tmp_elems(nb) + 64)) != ESES_OK) {
            T.release();
            return s;
        }
        long long nblk = 0, total = 0, hbad = 0;
        double h[2] = {0.0, 0.0};
        hipError_t e = fill_i32(bad, 1, 0, st);
        if (e == hipSuccess)
            e = launch_mesh(m, labels[q], (const long long *)isect[q].key, isect[q].lambda, counts[q],
                            out, cnt, bad, &nblk, st);
        if (e == hipSuccess) e = scan_i64(cnt, nblk, boff, tmp, st);
        if (e == hipSuccess) e = hipMemcpyAsync(h, out, sizeof(h), hipMemcpyDeviceToHost, st);
        if (e != hipSuccess) {
            (void)hipStreamSynchronize(st);
            T.release();
            set_err("mesh: %s", hipGetErrorString(e));
            return ESES_EDEVICE;
        }
        if ((s = read_scalars({{boff + nblk, true, &total}, {bad, false, &hbad}}, st)) != ESES_OK) {
            T.release();
            return s;
        }
        if (hbad) {
            T.release();
            set_err("molecule %d: %lld cut cube edges without a crossing record", q, hbad);
            return ESES_EINVAL;
        }
        stats[q].area = h[0];
        stats[q].volume = h[1];
        stats[q].n_triangles = total;
        if (triangles && triangles[q] && tri_capacity[q] > 0) {
            e = launch_mesh_write(m, labels[q], (const long long *)isect[q].key, isect[q].lambda,
                                  counts[q], boff, tri_capacity[q], triangles[q], st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (e != hipSuccess) {
                T.release();
                set_err("mesh: %s", hipGetErrorString(e));
                return ESES_EDEVICE;
            }
        }
        if (triangles && total > tri_capacity[q]) short_cap = true;
        T.release();
    }
    if (short_cap) {
        set_err("a triangle capacity is below the number of triangles (see n_triangles)");
        return ESES_ECAPACITY;
    }
    return ESES_OK;
}

eses_status eses_fill_cavities(eses_candidates *c, uint8_t *const *labels, int64_t *n_filled,
                               void *stream) {
    g_err.clear();
    if (!c || !labels) {
        set_err("bad handle or labels");
        return ESES_EINVAL;
    }
    const int nm = (int)c->mols.size();
    for (int q = 0; q < nm; ++q)
        if (!labels[q]) {
            set_err("labels[%d] is NULL", q);
            return ESES_EINVAL;
        }
    hipStream_t st = (hipStream_t)stream;
    Arena T;
    T.st = st;
    int *changed;
    unsigned long long *filled;
    eses_status s;
    if ((s = T.alloc(&changed, 1)) != ESES_OK || (s = T.alloc(&filled, nm)) != ESES_OK) {
        T.release();
        return s;
    }
    auto fail = [&](hipError_t e) {
        (void)hipStreamSynchronize(st);
        T.release();
        set_err("cavity fill: %s", hipGetErrorString(e));
        return ESES_EDEVICE;
    };
    hipError_t e = fill_u32((uint32_t *)filled, 2LL * nm, 0u, st);
    for (int q = 0; q < nm && e == hipSuccess; ++q) e = launch_fill_seed(labels[q], c->mols[q]->m.dims, st);
    if (e == hipSuccess && nm > 1) {
        e = hipMemcpyAsync(c->labels_dev, labels, sizeof(uint8_t *) * nm, hipMemcpyHostToDevice, st);
        if (e == hipSuccess && !c->fill_units) {
            std::vector<int2> u;
            for (int q = 0; q < nm; ++q) {
                const Mol &m = c->mols[q]->m;
                long long nt = 1;
                for (int a = 0; a < 3; ++a) nt *= (m.dims[a] + 7) / 8;
                for (long long t = 0; t < nt; ++t) u.push_back(make_int2(q, (int)t));
            }
            if (c->batch.alloc(&c->fill_units, (long long)u.size()) != ESES_OK) {
                T.release();
                return ESES_ENOMEM;
            }
            e = hipMemcpyAsync(c->fill_units, u.data(), sizeof(int2) * u.size(),
                               hipMemcpyHostToDevice, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);  // u is released on return
            c->n_fill_units = (long long)u.size();
        }
    }
    // passes until no tile changes (each pass reaches at least one new point
    // while any is left to reach, so the loop ends)
    for (long long pass = 0; e == hipSuccess; ++pass) {
        e = fill_i32(changed, 1, 0, st);
        if (e != hipSuccess) break;
        if (nm == 1) e = launch_fill_pass1(labels[0], c->mols[0]->m.dims, changed, st);
        else e = launch_fill_pass(c->mols_dev, c->labels_dev, c->fill_units, (int)c->n_fill_units,
                                  changed, st);
        if (e != hipSuccess) break;
        long long ch = 0;
        if ((s = read_scalars({{changed, false, &ch}}, st)) != ESES_OK) {
            T.release();
            return s;
        }
        if (!ch) break;
    }
    for (int q = 0; q < nm && e == hipSuccess; ++q)
        e = launch_fill_finish(labels[q], c->mols[q]->m.npts, filled + q, st);
    std::vector<unsigned long long> h((size_t)nm);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h.data(), filled, sizeof(unsigned long long) * nm, hipMemcpyDeviceToHost,
                           st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(e);
    T.release();
    if (n_filled)
        for (int q = 0; q < nm; ++q) n_filled[q] = (int64_t)h[(size_t)q];
    return ESES_OK;
}

void eses_set_timing(int enable) { g_timing.store(enable ? 1 : 0); }

eses_status eses_get_kernel_times(const eses_candidates *c, eses_kernel_times *out) {
    g_err.clear();
    if (!c || !out) {
        set_err("bad argument");
        return ESES_EINVAL;
    }
    out->classify_ms = 0.0;
    if (c->cls_timed) {
        float a = 0.0f;
        CK(hipEventSynchronize(c->ev[1]));
        CK(hipEventElapsedTime(&a, c->ev[0], c->ev[1]));
        out->classify_ms = a;
    }
    out->edge_detect_ms = c->detect_ms;
    out->edge_roots_ms = c->roots_ms;
    return ESES_OK;
}

eses_status eses_edge_work(eses_candidates *c, const uint8_t *const *labels,
                           eses_edge_stats *stats, void *stream) {
    g_err.clear();
    if (!c || !labels || !stats) {
        set_err("bad argument");
        return ESES_EINVAL;
    }
    hipStream_t st = (hipStream_t)stream;
    for (size_t q = 0; q < c->mols.size(); ++q) {
        const Mol &m = c->mols[q]->m;
        if (!labels[q]) {
            set_err("labels[%zu] is NULL", q);
            return ESES_EINVAL;
        }
        Arena T;
        T.st = st;
        long long nb = edge_detect_blocks(m);
        int *bcount, *ovf;
        long long *boff, *tmp;
        unsigned long long *work;
        eses_status s;
        if ((s = T.alloc(&bcount, nb + 1)) != ESES_OK || (s = T.alloc(&boff, nb + 2)) != ESES_OK ||
            (s = T.alloc(&tmp, scan_tmp_elems(nb) + 64)) != ESES_OK ||
            (s = T.alloc(&ovf, 1)) != ESES_OK || (s = T.alloc(&work, EDGE_WORK_COUNTERS)) != ESES_OK) {
            T.release();
            return s;
        }
        long long nblk = 0, total = 0;
        hipError_t e = launch_edge_detect_count(labels[q], m, bcount, &nblk, st);
        if (e == hipSuccess) e = scan_i64(bcount, nblk, boff, tmp, st);
        if (e == hipSuccess) e = hipMemcpyAsync(&total, boff + nblk, sizeof(long long), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        long long *keys = nullptr;
        int *tcount = nullptr, *ccount = nullptr, *coff = nullptr, *rank = nullptr,
            *order = nullptr, *units = nullptr, *ttmp = nullptr, *fb = nullptr, *nfb = nullptr;
        if (e == hipSuccess && total > 0) {
            if ((s = T.alloc(&keys, total)) != ESES_OK || (s = T.alloc(&tcount, m.ntiles + 1)) != ESES_OK ||
                (s = T.alloc(&ccount, m.ntiles + 1)) != ESES_OK ||
                (s = T.alloc(&coff, m.ntiles + 1)) != ESES_OK ||
                (s = T.alloc(&rank, total)) != ESES_OK ||
                (s = T.alloc(&order, edge_order_capacity(m, total))) != ESES_OK ||
                (s = T.alloc(&units, edge_units_capacity(m))) != ESES_OK ||
                (s = T.alloc(&fb, total)) != ESES_OK || (s = T.alloc(&nfb, 1)) != ESES_OK ||
                (s = T.alloc(&ttmp, scan_tmp_elems(m.ntiles) + 64)) != ESES_OK) {
                T.release();
                return s;
            }
        }
        if (e == hipSuccess) e = fill_u32((uint32_t *)work, 2 * EDGE_WORK_COUNTERS, 0u, st);
        if (e == hipSuccess) e = fill_i32(ovf, 1, 0, st);
        if (e == hipSuccess && total > 0)
            e = launch_edge_detect_write(labels[q], m, boff, total, keys, tcount, rank, st);
        if (e == hipSuccess && total > 0)
            e = launch_edge_group(m, keys, total, tcount, ccount, coff, rank, order, units, ttmp,
                                  st);
        if (e == hipSuccess && total > 0)
            e = launch_edge_work(m, labels[q], keys, total, order, tcount, coff, units, fb, nfb, ovf,
                                 work, st);
        unsigned long long h[EDGE_WORK_COUNTERS] = {0};
        if (e == hipSuccess) e = hipMemcpyAsync(h, work, sizeof(h), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        T.release();
        if (e != hipSuccess) {
            set_err("edge statistics: %s", hipGetErrorString(e));
            return ESES_EDEVICE;
        }
        eses_edge_stats &o = stats[q];
        o.n_edges = (int64_t)h[0];
        o.reach_sphere = (int64_t)h[1];
        o.reach_torus = (int64_t)h[2];
        o.quad_solves = (int64_t)h[3];
        o.quartic_solves = (int64_t)h[4];
        o.horner_flops = (int64_t)h[5];
        o.cut_tests = (int64_t)h[6];
        o.label_evals = (int64_t)h[7];
        for (int k = 0; k < 6; ++k) o.label_tests[k] = (int64_t)h[8 + k];
        o.cone_tests = (int64_t)h[15];
    }
    return ESES_OK;
}

void eses_set_allocator(eses_alloc_fn alloc, eses_release_fn release, void *ctx) {
    ExtAlloc &ea = ext_alloc();
    std::lock_guard<std::mutex> lock(ea.mu);
    const bool on = alloc && release;
    ea.alloc = on ? alloc : nullptr;
    ea.release = on ? release : nullptr;
    ea.ctx = on ? ctx : nullptr;
}

eses_status eses_trim_cache(void) {
    g_err.clear();
    BlockCache &bc = block_cache();
    std::lock_guard<std::mutex> lock(bc.mu);
    int cur = 0;
    (void)hipGetDevice(&cur);
    hipError_t err = hipSuccess;
    for (auto &kv : bc.free) {
        const int dev = std::get<0>(kv.first);
        if (hipSetDevice(dev) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
            err = hipGetLastError();
            continue;
        }
        for (void *p : kv.second) {
            hipError_t e = hipFree(p);
            if (e != hipSuccess) err = e;
        }
        kv.second.clear();
    }
    bc.free.clear();
    (void)hipSetDevice(cur);
    if (err != hipSuccess) {
        set_err("eses_trim_cache: %s", hipGetErrorString(err));
        return ESES_EDEVICE;
    }
    return ESES_OK;
}

void eses_free_candidates(eses_candidates *c) {
    if (!c) return;
    for (int k = 0; k < 2; ++k) {
        if (c->exec[k]) (void)hipGraphExecDestroy(c->exec[k]);
        if (c->graph[k]) (void)hipGraphDestroy(c->graph[k]);
    }
    c->batch.release();
    for (int q = 0; q < 6; ++q)
        if (c->ev[q]) (void)hipEventDestroy(c->ev[q]);
    for (MolState *S : c->mols) {
        S->arena.release();
        delete S;
    }
    (void)hipStreamSynchronize(c->stream);
    delete c;
}

}  // extern "C"
