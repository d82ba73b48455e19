// Host runtime of the pyhea library: validation, the binary64 objective
// contract on the host, and the chain driver behind pyhea_mc_run/pyhea_mc_batch.
#include "runtime.h"

#include <algorithm>
#include <list>
#include <climits>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>

#include "autotune.h"
#include "sro_bits.h"

namespace pyhea {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }
const std::string &last_error() { return g_last_error; }

pyhea_status device_error(hipError_t e, const char *what) {
    set_error(std::string("HIP error in ") + what + ": " + hipGetErrorString(e));
    return PYHEA_EDEVICE;
}

hipError_t pool_alloc(void **ptr, size_t bytes, hipStream_t stream) {
    static std::mutex mu;
    static bool tuned[64] = {false};
    int dev = 0;
    hipError_t r = hipGetDevice(&dev);
    if (r != hipSuccess) return r;
    if (dev >= 0 && dev < 64) {
        std::lock_guard<std::mutex> lock(mu);
        if (!tuned[dev]) {
            hipMemPool_t pool;
            if ((r = hipDeviceGetDefaultMemPool(&pool, dev)) != hipSuccess) return r;
            uint64_t keep = kPoolRetainBytes;
            if ((r = hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep)) != hipSuccess) return r;
            tuned[dev] = true;
        }
    }
    return hipMallocAsync(ptr, bytes, stream);
}

hipError_t set_max_lds(const void *fn, size_t lds) {
    static std::mutex mu;
    static std::map<std::pair<int, const void *>, size_t> done;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(mu);
    auto it = done.find({dev, fn});
    if (it != done.end() && it->second >= lds) return hipSuccess;
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e == hipSuccess) done[{dev, fn}] = lds;
    return e;
}

int max_lds_per_block() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 64 * 1024;
    static int cached[64] = {0};
    if (dev >= 0 && dev < 64 && cached[dev]) return cached[dev];
    int v = 64 * 1024;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) v = (int)prop.sharedMemPerBlock;
    if (dev >= 0 && dev < 64) cached[dev] = v;
    return v;
}

int cu_count() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    static int cached[64] = {0};
    if (dev >= 0 && dev < 64 && cached[dev]) return cached[dev];
    int v = 256;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
    if (dev >= 0 && dev < 64) cached[dev] = v;
    return v;
}

pyhea_status check_objective(const Geometry &g, const pyhea_objective *obj) {
    if (!obj || !obj->target || !obj->weight) {
        set_error("objective, target and weight must not be NULL");
        return PYHEA_EINVAL;
    }
    const int E = g.S * g.M * g.M;
    for (int e = 0; e < E; ++e)
        if (!std::isfinite(obj->target[e])) {
            set_error("target alphas must be finite");
            return PYHEA_EINVAL;
        }
    for (int k = 0; k < g.S; ++k)
        if (!std::isfinite(obj->weight[k]) || obj->weight[k] < 0.0) {
            set_error("shell weights must be finite and >= 0");
            return PYHEA_EINVAL;
        }
    return PYHEA_OK;
}

pyhea_status check_params(const pyhea_mc_params *p) {
    if (!p) {
        set_error("params must not be NULL");
        return PYHEA_EINVAL;
    }
    if (p->cand_per_step < 1 || p->cand_per_step > kMaxB) {
        set_error("cand_per_step must be in [1, 256]");
        return PYHEA_EINVAL;
    }
    if (p->n_trials < 0 || p->n_trials / p->cand_per_step >= (int64_t(1) << 32)) {
        set_error("n_trials must be >= 0 and n_trials / cand_per_step < 2^32");
        return PYHEA_EINVAL;
    }
    if (p->commit_mode != PYHEA_MODE_DISJOINT && p->commit_mode != PYHEA_MODE_BEST) {
        set_error("commit_mode must be PYHEA_MODE_DISJOINT or PYHEA_MODE_BEST");
        return PYHEA_EINVAL;
    }
    if (p->depth_limit < 0) {
        set_error("depth_limit must be >= 0");
        return PYHEA_EINVAL;
    }
    if (!std::isfinite(p->accept_tol)) {
        set_error("accept_tol must be finite");
        return PYHEA_EINVAL;
    }
    return PYHEA_OK;
}

bool species_totals(const Geometry &g, const int64_t *counts, int64_t *n) {
    bool ok = true;
    for (int i = 0; i < g.M; ++i) {
        int64_t r = 0;
        for (int j = 0; j < g.M; ++j) r += counts[i * g.M + j];
        n[i] = r / g.z[0];
        ok = ok && n[i] > 0;
    }
    return ok;
}

void ratio_table(const Geometry &g, const int64_t *n, double *R) {
    for (int k = 0; k < g.S; ++k)
        for (int i = 0; i < g.M; ++i)
            for (int j = 0; j < g.M; ++j)
                R[(k * g.M + i) * g.M + j] = (double)g.N / (double)(n[i] * n[j] * (int64_t)g.z[k]);
}

namespace {
// the bit-sliced kernel's launch shape for K configurations of g (false: gather)
bool bit_shape(const Geometry &g, int64_t K, BitDesc *bd) {
    const int forced = forced_eval_kernel();
    const int split = forced == 2 ? 1 : forced == 3 ? 4 : 2;
    return forced != 0 && fill_bit_desc(g, max_lds_per_block(), K, split, bd);
}

// the streaming kernel's launch shape for K configurations of g (false: not taken)
bool stream_shape(const Geometry &g, int64_t K, StreamDesc *sd) {
    if (forced_eval_kernel() != 4) return false;
    int G = 0, threads = 0;
    forced_stream_shape(&G, &threads);
    return fill_stream_desc(g, max_lds_per_block(), cu_count(), K, G, threads, sd);
}
}  // namespace

size_t count_partial_bytes(const Geometry &g, int64_t K) {
    BitDesc bd;
    StreamDesc sd;
    if (K <= 0 || stream_shape(g, K, &sd) || !bit_shape(g, K, &bd) || bd.nchunks <= 1) return 0;
    return (size_t)K * bd.nchunks * bd.partial_stride * 4;
}

pyhea_status count_configs(const Geometry &g, int64_t K, const int8_t *species, int32_t *counts,
                           int32_t *bad, hipStream_t stream, const double *tw, double *S_F, bool *fused,
                           void *partial_scratch) {
    if (fused) *fused = false;
    if (K <= 0) return PYHEA_OK;
    StreamDesc sd;
    if (stream_shape(g, K, &sd)) {
        const bool fuse = S_F != nullptr;   // the counting launch finishes Eq. 2-3 too
        PYHEA_HIP(launch_count_stream(g, sd, K, species, counts, bad, fuse ? tw : nullptr, fuse ? S_F : nullptr,
                                      stream));
        if (fused) *fused = fuse;
        return PYHEA_OK;
    }
    BitDesc bd;
    if (bit_shape(g, K, &bd)) {
        void *partial = partial_scratch;
        const bool own = partial == nullptr && bd.nchunks > 1;
        if (own) PYHEA_HIP(pool_alloc(&partial, (size_t)K * bd.nchunks * bd.partial_stride * 4, stream));
        const bool fuse = S_F != nullptr;   // the counting launch finishes Eq. 2-3 too
        const hipError_t e = launch_count_bits(g, bd, K, species, (int32_t *)partial, counts, bad,
                                               fuse ? tw : nullptr, fuse ? S_F : nullptr, stream);
        if (own) (void)hipFreeAsync(partial, stream);
        PYHEA_HIP(e);
        if (fused) *fused = fuse;
        return PYHEA_OK;
    }
    EvalDesc ed;
    fill_eval_desc(g, &ed);
    PYHEA_HIP(launch_count_gather(ed, K, species, counts, bad, stream));
    return PYHEA_OK;
}

namespace {
size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// eval_batch scratch: flags [K] int32 | target, weight table | partial sums
struct EvalScratch {
    size_t tw, partial, total;
};
EvalScratch eval_scratch_layout(const Geometry &g, int64_t K) {
    EvalScratch l;
    l.tw = align256((size_t)K * 4);
    l.partial = align256(l.tw + (size_t)kMaxTable * 8);
    l.total = l.partial + count_partial_bytes(g, K);
    return l;
}
}  // namespace

size_t eval_batch_scratch_bytes(const Geometry &g, int64_t K) { return eval_scratch_layout(g, K).total; }

pyhea_status eval_batch(const Geometry &g, int64_t K, const int8_t *species, const pyhea_objective *obj,
                        int32_t *counts, double *S_F, hipStream_t stream, void *scratch) {
    if (K <= 0) return PYHEA_OK;
    const int E = g.S * g.M * g.M;
    const EvalScratch lay = eval_scratch_layout(g, K);
    void *own = nullptr;
    if (!scratch) {
        PYHEA_HIP(pool_alloc(&own, lay.total, stream));
        scratch = own;
    }
    char *base = (char *)scratch;
    int32_t *bad = (int32_t *)base;
    double *tdev = (double *)(base + lay.tw);
    pyhea_status st = PYHEA_OK;
    hipError_t e = hipSuccess;
    if (obj) {
        SmallTable tw{};
        std::memcpy(tw.v, obj->target, E * 8);
        std::memcpy(tw.v + E, obj->weight, g.S * 8);
        e = launch_upload(tw, E + kMaxShells, tdev, stream);
    }
    bool fused = false;
    if (e == hipSuccess)
        st = count_configs(g, K, species, counts, bad, stream, obj ? tdev : nullptr, obj ? S_F : nullptr, &fused,
                           lay.total > lay.partial ? base + lay.partial : nullptr);
    if (e == hipSuccess && st == PYHEA_OK && obj && !fused) {
        EvalDesc ed;
        fill_eval_desc(g, &ed);
        e = launch_objective_epilogue(ed, K, counts, bad, tdev, tdev + E, S_F, nullptr, stream);
    }
    if (own) (void)hipFreeAsync(own, stream);
    if (e != hipSuccess) return device_error(e, "eval_batch");
    return st;
}

namespace {

// Stream-ordered allocation, freed on the same stream.
struct DeviceBuffer {
    void *ptr = nullptr;
    hipStream_t stream = nullptr;
    ~DeviceBuffer() {
        if (ptr) (void)hipFreeAsync(ptr, stream);
    }
};

// Auxiliary streams (default priority, non-blocking) on which launches of
// different shapes run beside the caller's stream; created once per device,
// kept until exit.  Three, so that with the caller's stream they map onto the
// four hardware queues a process gets by default.  Set 1 is a separate main
// stream and three auxiliary streams used only to record graphs, so that a
// recording never meets work that other calls put on set 0.
constexpr int kAuxStreams = 3;

bool stream_set(int set, hipStream_t *out, int count) {
    static std::mutex mu;
    static hipStream_t pool[2][64][kAuxStreams + 1];
    static bool made[2][64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return false;
    std::lock_guard<std::mutex> lock(mu);
    if (!made[set][dev]) {
        for (int i = 0; i <= kAuxStreams; ++i)
            if (hipStreamCreateWithFlags(&pool[set][dev][i], hipStreamNonBlocking) != hipSuccess) return false;
        made[set][dev] = true;
    }
    for (int i = 0; i < count; ++i) out[i] = pool[set][dev][i];
    return true;
}

bool aux_streams(hipStream_t *out) { return stream_set(0, out, kAuxStreams); }

// Events that fork work from `main` onto aux streams and join it back.
struct Fork {
    hipStream_t main = nullptr;
    hipStream_t aux[kAuxStreams] = {};
    int used = 0;
    std::vector<hipEvent_t> events;
    ~Fork() {
        // left without end() on an error path: let the aux streams drain before
        // anything they read is released on the caller's stream
        for (int i = 0; i < used; ++i) (void)hipStreamSynchronize(aux[i]);
        for (hipEvent_t e : events) (void)hipEventDestroy(e);
    }
    // launch i goes to the caller's stream (i % (used + 1) == 0) or aux stream;
    // aux_set: the auxiliary streams to use (nullptr: the shared ones)
    hipError_t begin(hipStream_t m, int n_launches, const hipStream_t *aux_set = nullptr) {
        main = m;
        used = std::min(n_launches - 1, kAuxStreams);
        if (used > 0 && aux_set) {
            for (int i = 0; i < kAuxStreams; ++i) aux[i] = aux_set[i];
        } else if (used <= 0 || !aux_streams(aux)) {
            used = 0;  // everything stays on the caller's stream
            return hipSuccess;
        }
        hipEvent_t e;
        hipError_t r = hipEventCreateWithFlags(&e, hipEventDisableTiming);
        if (r != hipSuccess) return r;
        events.push_back(e);
        if ((r = hipEventRecord(e, main)) != hipSuccess) return r;
        for (int i = 0; i < used; ++i)
            if ((r = hipStreamWaitEvent(aux[i], e, 0)) != hipSuccess) return r;
        return hipSuccess;
    }
    hipStream_t stream(int i) const {
        const int r = used ? i % (used + 1) : 0;
        return r == 0 ? main : aux[r - 1];
    }
    hipError_t end() {
        for (int i = 0; i < used; ++i) {
            hipEvent_t e;
            hipError_t r = hipEventCreateWithFlags(&e, hipEventDisableTiming);
            if (r != hipSuccess) return r;
            events.push_back(e);
            if ((r = hipEventRecord(e, aux[i])) != hipSuccess) return r;
            if ((r = hipStreamWaitEvent(main, e, 0)) != hipSuccess) return r;
        }
        used = 0;
        return hipSuccess;
    }
};

}  // namespace

namespace {

// Measures the candidate launch shapes of chain j on a scratch copy of its
// configuration: after kProbeWarm steps the chain state (configuration, counts,
// counters) is saved, and every candidate runs the same segment from that
// state -- kProbeBase steps, and kProbeBase + kProbeSteps steps -- so that all
// see the same trials and commits (a shape never changes the trajectory); the
// difference of the two times is the per-step cost without the launch's
// fixed load and write-back (the median of kProbeReps such differences).  The
// cost model's shape `model` is always a candidate, and another shape replaces
// it only if it is at least kProbeMargin cheaper per step: shapes that differ
// only in how commits are grouped cost the same between commits, and a short
// segment cannot tell them apart.  Sets *ok false if the chain is invalid (the
// real run reports it).
constexpr int kProbeWarm = 64;
constexpr int kProbeBase = 16;
constexpr int kProbeSteps = 320;
constexpr int kProbeReps = 3;
constexpr double kProbeMargin = 0.03;

pyhea_status probe_launch(const ChainJob &j, int n_chains, int lds_budget, const LaunchShape &model,
                          hipStream_t stream, LaunchShape *best, double *us_per_step, bool *ok) {
    *ok = false;
    const Geometry &g = j.g;
    const int B = j.params.cand_per_step;
    std::vector<LaunchShape> cand = candidate_launches(g, B, lds_budget, n_chains);
    int im = -1;
    for (int i = 0; i < (int)cand.size(); ++i)
        if (cand[i].store == model.store && cand[i].W == model.W && cand[i].bal == model.bal && cand[i].K == model.K &&
            cand[i].CH == model.CH)
            im = i;
    if (im < 0) {
        cand.insert(cand.begin(), model);
        im = 0;
    }
    if (cand.size() < 2) return PYHEA_OK;
    const int nc = (int)cand.size();
    const size_t E = (size_t)g.S * g.M * g.M;
    size_t off = 0;
    const size_t o_sp = off;
    off = align256(off + (size_t)g.N);
    const size_t o_snap = off;   // saved configuration | counts | state
    off = align256(off + (size_t)g.N);
    const size_t o_snap_counts = off;
    off = align256(off + E * 4);
    const size_t o_snap_state = off;
    off = align256(off + sizeof(ChainState));
    const size_t o_pad = off;
    off = align256(off + (size_t)g.Npad);
    const size_t o_counts = off;   // counts | bad | state: zeroed together
    off += E * 4;
    const size_t o_bad = off;
    off += 8;
    const size_t o_state = off;
    off += sizeof(ChainState);
    const size_t zero_end = (off + 3) & ~size_t(3);
    off = align256(off);
    const size_t o_R = off;
    off = align256(off + E * 8);
    const size_t y_begin = off;   // target | descs | task | tile0: one upload
    const size_t o_target = off;
    off = align256(off + E * 8);
    const size_t o_descs = off;
    off = align256(off + (size_t)nc * sizeof(ChainDesc));
    const size_t o_task = off;
    off += sizeof(CountTask);
    const size_t o_tile0 = off;
    off += 4;
    const size_t y_end = off;
    DeviceBuffer arena;
    arena.stream = stream;
    PYHEA_HIP(pool_alloc(&arena.ptr, off, stream));
    char *base = (char *)arena.ptr;

    std::vector<char> hy(y_end - y_begin, 0);
    auto hy_at = [&](size_t o) { return hy.data() + (o - y_begin); };
    std::memcpy(hy_at(o_target), j.target.data(), E * 8);
    ChainDesc d;
    std::memset(&d, 0, sizeof(d));
    fill_chain_geometry(g, &d);
    d.seed = j.params.seed;
    d.chain_id = j.params.chain_id;
    d.B = B;
    d.n_trials = INT64_MAX / 2;   // never exhausted: kProbeSteps bounds each launch
    d.mode = j.params.commit_mode;
    d.depth_limit = 0;
    d.tau = j.params.accept_tol;
    for (int k = 0; k < kMaxShells; ++k) d.w[k] = k < g.S ? j.weight[k] : 0.0;
    d.species = (int8_t *)(base + o_sp);
    d.R = (const double *)(base + o_R);
    d.target = (const double *)(base + o_target);
    d.counts = (int32_t *)(base + o_counts);
    d.state = (ChainState *)(base + o_state);
    d.sym = symmetric_target(j.target.data(), g.S, g.M);
    ChainDesc *hd = (ChainDesc *)hy_at(o_descs);
    for (int i = 0; i < nc; ++i) {
        hd[i] = d;
        hd[i].store = cand[i].store;
        hd[i].lds_bytes = cand[i].lds;
        hd[i].pad_global = cand[i].store == kStoreGlobal ? (int8_t *)(base + o_pad) : nullptr;
    }
    CountTask *task = (CountTask *)hy_at(o_task);
    fill_eval_desc(g, &task->ed);
    task->species = d.species;
    task->counts = d.counts;
    task->bad = (int32_t *)(base + o_bad);
    *(uint32_t *)hy_at(o_tile0) = 0;

    PYHEA_HIP(launch_zero_i32((int32_t *)(base + o_counts), (int64_t)((zero_end - o_counts) / 4), stream));
    PYHEA_HIP(hipMemcpyAsync(base + o_sp, j.species_dev, (size_t)g.N, hipMemcpyDeviceToDevice, stream));
    PYHEA_HIP(hipMemcpyAsync(base + y_begin, hy.data(), hy.size(), hipMemcpyHostToDevice, stream));
    {
        const uint32_t tile = count_tile_for((uint64_t)g.N);
        PYHEA_HIP(launch_count_tasks((const CountTask *)(base + o_task), (const uint32_t *)(base + o_tile0), 1,
                                     count_tiles((uint32_t)g.N, tile), tile, (int)E, stream));
    }
    const ChainDesc *ddev = (const ChainDesc *)(base + o_descs);
    PYHEA_HIP(launch_chain_ratio(ddev, 1, (const int32_t *)(base + o_bad), stream));

    const int nev = 2 * nc * kProbeReps;
    std::vector<hipEvent_t> ev(nev, nullptr);
    struct EventGuard {
        std::vector<hipEvent_t> &v;
        ~EventGuard() {
            for (hipEvent_t e : v)
                if (e) (void)hipEventDestroy(e);
        }
    } guard{ev};
    for (auto &e : ev) PYHEA_HIP(hipEventCreate(&e));
    auto run = [&](int i, int steps) -> hipError_t {
        const LaunchShape &c = cand[i];
        hipError_t e = hipSuccess;
        if (c.store == kStoreGlobal && (e = launch_pad_fill(ddev + i, 1, stream)) != hipSuccess) return e;
        e = launch_mc(ddev + i, 1, c.store, g.M, g.S, B, c.W, c.bal, c.K, c.CH, c.lds, steps, stream);
        if (e == hipSuccess && c.store == kStoreGlobal) e = launch_pad_drain(ddev + i, 1, stream);
        return e;
    };
    PYHEA_HIP(run(0, kProbeWarm));   // past the first, most commit-heavy steps
    auto copy = [&](size_t dst, size_t src, size_t bytes) {
        return hipMemcpyAsync(base + dst, base + src, bytes, hipMemcpyDeviceToDevice, stream);
    };
    PYHEA_HIP(copy(o_snap, o_sp, (size_t)g.N));
    PYHEA_HIP(copy(o_snap_counts, o_counts, E * 4));
    PYHEA_HIP(copy(o_snap_state, o_state, sizeof(ChainState)));
    std::vector<hipEvent_t> ev2(nev, nullptr);
    EventGuard guard2{ev2};
    for (auto &e : ev2) PYHEA_HIP(hipEventCreate(&e));
    // repetitions outermost, so that a slow spell of the device touches every candidate alike
    for (int r = 0; r < kProbeReps; ++r)
        for (int i = 0; i < nc; ++i)
            for (int len = 0; len < 2; ++len) {
                PYHEA_HIP(copy(o_sp, o_snap, (size_t)g.N));
                PYHEA_HIP(copy(o_counts, o_snap_counts, E * 4));
                PYHEA_HIP(copy(o_state, o_snap_state, sizeof(ChainState)));
                std::vector<hipEvent_t> &v = len == 0 ? ev : ev2;
                const int x = 2 * (r * nc + i);
                PYHEA_HIP(hipEventRecord(v[x], stream));
                PYHEA_HIP(run(i, len == 0 ? kProbeBase : kProbeBase + kProbeSteps));
                PYHEA_HIP(hipEventRecord(v[x + 1], stream));
            }
    ChainState st;
    PYHEA_HIP(hipMemcpyAsync(&st, base + o_state, sizeof(st), hipMemcpyDeviceToHost, stream));
    PYHEA_HIP(hipStreamSynchronize(stream));
    if (st.status != 0) return PYHEA_OK;   // invalid chain: the real run reports it
    std::vector<double> cost(nc);
    for (int i = 0; i < nc; ++i) {
        double d[kProbeReps];
        for (int r = 0; r < kProbeReps; ++r) {
            const int x = 2 * (r * nc + i);
            float ms0 = 0.0f, ms1 = 0.0f;
            PYHEA_HIP(hipEventElapsedTime(&ms0, ev[x], ev[x + 1]));
            PYHEA_HIP(hipEventElapsedTime(&ms1, ev2[x], ev2[x + 1]));
            d[r] = 1e3 * ((double)ms1 - (double)ms0) / kProbeSteps;
        }
        std::sort(d, d + kProbeReps);
        cost[i] = d[kProbeReps / 2];
    }
    int bi = im;
    for (int i = 0; i < nc; ++i)
        if (cost[i] < cost[bi]) bi = i;
    if (cost[bi] > (1.0 - kProbeMargin) * cost[im]) bi = im;
    *best = cand[bi];
    *us_per_step = cost[bi];
    *ok = true;
    return PYHEA_OK;
}

}  // namespace

namespace {

// Page-locked host staging for a chain call's upload and read-back: copies
// from and to it are single DMA transfers, and the upload returns at once.
// Buffers are leased from a pool and kept until exit.  A lease is returned
// only after its stream has drained, so no copy still reads or writes a
// buffer the next call fills.
struct PinnedBuf {
    char *p = nullptr;
    size_t cap = 0;
};
std::mutex g_pin_mu;
auto *g_pin_free = new std::vector<PinnedBuf>();

struct PinnedLease {
    PinnedBuf b;
    hipStream_t stream = nullptr;
    bool drained = false;
    ~PinnedLease() {
        if (!b.p) return;
        if (!drained) (void)hipStreamSynchronize(stream);
        std::lock_guard<std::mutex> lock(g_pin_mu);
        g_pin_free->push_back(b);
    }
};

hipError_t pinned_lease(size_t bytes, hipStream_t stream, PinnedLease *out) {
    out->stream = stream;
    {
        std::lock_guard<std::mutex> lock(g_pin_mu);
        for (size_t i = 0; i < g_pin_free->size(); ++i)
            if ((*g_pin_free)[i].cap >= bytes) {
                out->b = (*g_pin_free)[i];
                g_pin_free->erase(g_pin_free->begin() + (long)i);
                return hipSuccess;
            }
    }
    const size_t cap = std::max<size_t>((bytes + (size_t(1) << 20) - 1) & ~((size_t(1) << 20) - 1), size_t(1) << 20);
    void *p = nullptr;
    const hipError_t e = hipHostMalloc(&p, cap, hipHostMallocDefault);
    if (e != hipSuccess) return e;
    out->b.p = (char *)p;
    out->b.cap = cap;
    return hipSuccess;
}

// Recorded device work of chain calls: a persistent arena and the graph that
// runs a call's launches on it (run_chains).  A structure is recorded the
// second time it is seen, so one-off calls never pay for recording.  Plans are
// never destroyed: at most kMaxPlans are made per process, and calls of other
// structures then run eagerly.  (A test that dropped the least recently used
// plan -- destroying its executable graph and freeing its arena -- ended in a
// host segmentation fault whose cause was not found, so nothing is dropped.)
// A call holds its plan's mutex from the upload to the read-back, so calls of
// one structure from several threads take turns on its arena.
struct ChainPlan {
    std::vector<int64_t> key;
    void *arena = nullptr;
    hipGraph_t graph = nullptr;   // kept beside its executable form
    hipGraphExec_t exec = nullptr;
    bool failed = false;          // recording was refused: calls run eagerly
    std::mutex mu;
};
constexpr size_t kMaxPlans = 32;
constexpr size_t kSeenKeys = 16;
std::mutex g_plan_mu;
auto *g_plans = new std::list<ChainPlan *>();          // most recently used first; never freed
auto *g_seen = new std::list<std::vector<int64_t>>();  // structures seen once

// The plan for `key` (arena of `bytes`), or none: on the first sighting, and
// once kMaxPlans plans exist.
hipError_t chain_plan(const std::vector<int64_t> &key, size_t bytes, ChainPlan **out) {
    *out = nullptr;
    std::lock_guard<std::mutex> lock(g_plan_mu);
    for (auto it = g_plans->begin(); it != g_plans->end(); ++it)
        if ((*it)->key == key) {
            *out = *it;
            g_plans->splice(g_plans->begin(), *g_plans, it);
            return hipSuccess;
        }
    if (g_plans->size() >= kMaxPlans) return hipSuccess;
    auto seen = std::find(g_seen->begin(), g_seen->end(), key);
    if (seen == g_seen->end()) {
        g_seen->push_front(key);
        if (g_seen->size() > kSeenKeys) g_seen->pop_back();
        return hipSuccess;
    }
    g_seen->erase(seen);
    void *arena = nullptr;
    const hipError_t e = hipMalloc(&arena, bytes);
    if (e != hipSuccess) return e;
    ChainPlan *p = new ChainPlan();
    p->key = key;
    p->arena = arena;
    g_plans->push_front(p);
    *out = p;
    return hipSuccess;
}

// Records work(stream, aux streams) into p->graph and p->exec on the recording
// streams.  On failure the plan stays without a graph and its calls run eagerly.
template <class Work>
hipError_t record_plan(ChainPlan *p, Work &work) {
    hipStream_t st[kAuxStreams + 1];
    if (!stream_set(1, st, kAuxStreams + 1)) return hipErrorInvalidValue;
    hipError_t e = hipStreamBeginCapture(st[0], hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) return e;
    const hipError_t ew = work(st[0], st + 1);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(st[0], &graph);
    if (ew != hipSuccess || e != hipSuccess) return ew != hipSuccess ? ew : e;
    p->graph = graph;
    e = hipGraphInstantiate(&p->exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) p->exec = nullptr;
    return e;
}

}  // namespace

pyhea_status run_chains(std::vector<ChainJob> &jobs, pyhea_mc_stats *stats,
                        std::vector<std::vector<int64_t>> *final_counts, hipStream_t stream,
                        int variant) {
    const int n = (int)jobs.size();
    if (n == 0) return PYHEA_OK;
    const int lds_budget = max_lds_per_block();

    // Device arena, in three blocks so that each crosses the bus in one copy:
    //   X (read back): counts | recount | bad | bad2 | state     (zeroed on the device)
    //   Y (uploaded before counting): target | descs | count tasks (initial, final) | tile0
    //   Z (written on the device from the initial counts): R
    // One upload, one read-back: the calls between them are ordered on the stream.
    // followed by the padded HBM copies of chains that keep their configuration in HBM.
    std::vector<size_t> eoff(n + 1, 0);
    for (int c = 0; c < n; ++c) eoff[c + 1] = eoff[c] + (size_t)jobs[c].g.S * jobs[c].g.M * jobs[c].g.M;
    const size_t Etot = eoff[n];
    size_t off = 0;
    const size_t o_counts = off;
    off += Etot * 4;
    const size_t o_recount = off;
    off += Etot * 4;
    const size_t o_bad = off;
    off += (size_t)n * 4;
    const size_t o_bad2 = off;
    off += (size_t)n * 4;
    off = (off + 7) & ~size_t(7);
    const size_t o_state = off;
    off += (size_t)n * sizeof(ChainState);
    const size_t x_end = off;
    off = align256(off);
    const size_t y_begin = off;
    const size_t o_target = off;
    off += Etot * 8;
    off = align256(off);
    const size_t o_descs = off;
    off += (size_t)n * sizeof(ChainDesc);
    off = align256(off);
    const size_t o_tasks = off;
    off += (size_t)2 * n * sizeof(CountTask);
    const size_t o_tile0 = off;
    off += (size_t)n * 4;
    const size_t y_end = off;
    off = align256(off);
    const size_t o_R = off;
    off += Etot * 8;
    std::vector<LaunchShape> shape(n);
    std::vector<int> measured(n, 0);
    std::vector<size_t> o_pad(n, 0);
    // Single chains are measured.  A batch keeps the cost model's shapes: a lone
    // chain on an idle GPU (what a probe sees) prefers commits one by one, but
    // with two chains per CU the 512-chain batch ran 12 % slower that way
    // (5.97e9 against 6.8e9 trial swaps/s with the model's commit chunks).
    const bool measure = variant < 0 && measure_enabled() && n == 1;
    for (int c = 0; c < n; ++c)
        shape[c] = choose_launch(jobs[c].g, jobs[c].params.cand_per_step, lds_budget, variant < 0 ? 0 : variant, n);
    if (measure) {
        // (Written for groups: chains that share a launch under the cost model
        // would keep sharing one, the group's longest chain measured for all.)
        std::map<std::tuple<int, int, int, int, int, int>, std::vector<int>> fam;
        for (int c = 0; c < n; ++c)
            fam[{shape[c].store, jobs[c].g.M, jobs[c].g.S, jobs[c].params.cand_per_step, shape[c].W, shape[c].bal}]
                .push_back(c);
        for (auto &kv : fam) {
            const std::vector<int> &members = kv.second;
            int rep = members[0];
            for (int c : members)
                if (jobs[c].params.n_trials * jobs[c].g.Z > jobs[rep].params.n_trials * jobs[rep].g.Z) rep = c;
            const int B = jobs[rep].params.cand_per_step;
            const TuneKey key = tune_key(jobs[rep].g, B, n);
            LaunchShape t;
            bool have = tuned_launch(key, &t);
            if (!have) {
                double us = 0.0;
                bool ok = false;
                const pyhea_status ps = probe_launch(jobs[rep], n, lds_budget, shape[rep], stream, &t, &us, &ok);
                if (ps != PYHEA_OK) return ps;
                if (ok) record_tuned_launch(key, t, us);
                have = ok;
            }
            if (!have || t.W != jobs[rep].g.S) continue;
            bool fits = true;
            for (int c : members) fits = fits && launch_lds_bytes(jobs[c].g, B, t) <= lds_budget;
            if (!fits) continue;
            for (int c : members) {
                shape[c] = t;
                shape[c].lds = (int)launch_lds_bytes(jobs[c].g, B, t);
                measured[c] = 1;
            }
        }
    }
    for (int c = 0; c < n; ++c) {
        if (shape[c].store == kStoreGlobal) {
            off = align256(off);
            o_pad[c] = off;
            off += (size_t)jobs[c].g.Npad;
        }
    }
    // launch groups: chains of one shape share a launch, longest chains first
    // (trials x offsets gathered per trial) so that its tail is short; then the
    // launch whose longest chain is longest (per-trial cost taken as offsets
    // gathered plus count entries evaluated) goes first, so it starts first
    struct Launch {
        int first, count, store, M, S, B, W, bal, K, CH, lds;
    };
    std::vector<Launch> launches;
    std::vector<int> pos(n);   // descriptor position of each chain
    {
        std::map<std::tuple<int, int, int, int, int, int, int, int>, std::vector<int>> groups;
        for (int c = 0; c < n; ++c)
            groups[{shape[c].store, jobs[c].g.M, jobs[c].g.S, jobs[c].params.cand_per_step, shape[c].W, shape[c].bal,
                    shape[c].K, shape[c].CH}]
                .push_back(c);
        int at = 0;
        std::vector<std::pair<int64_t, Launch>> byw;
        for (auto &kv : groups) {
            std::vector<int> idx = kv.second;
            std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
                return jobs[a].params.n_trials * jobs[a].g.Z > jobs[b].params.n_trials * jobs[b].g.Z;
            });
            Launch L{at, (int)idx.size(), std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first),
                     std::get<3>(kv.first), std::get<4>(kv.first), std::get<5>(kv.first), std::get<6>(kv.first),
                     std::get<7>(kv.first), 0};
            int64_t w = 0;
            for (int c : idx) {
                L.lds = std::max(L.lds, shape[c].lds);
                pos[c] = at++;
                const Geometry &g = jobs[c].g;
                w = std::max<int64_t>(w, jobs[c].params.n_trials * (int64_t)(g.zstart[g.S] + g.M * g.M));
            }
            byw.push_back({w, L});
        }
        std::stable_sort(byw.begin(), byw.end(),
                         [](const std::pair<int64_t, Launch> &x, const std::pair<int64_t, Launch> &y) {
                             return x.first > y.first;
                         });
        for (auto &x : byw) launches.push_back(x.second);
    }
    uint32_t n_tiles = 0;
    uint64_t total_sites = 0;
    int max_E = 0;
    for (int c = 0; c < n; ++c) {
        total_sites += (uint64_t)jobs[c].g.N;
        max_E = std::max(max_E, jobs[c].g.S * jobs[c].g.M * jobs[c].g.M);
    }
    const uint32_t count_tile = count_tile_for(total_sites);
    std::vector<uint32_t> tile0v(n);
    for (int c = 0; c < n; ++c) {
        tile0v[c] = n_tiles;
        n_tiles += count_tiles((uint32_t)jobs[c].g.N, count_tile);
    }

    // The device work of the call is fixed by the arena layout and the launches:
    // a call of a structure seen before replays the graph recorded for it, with
    // only the uploaded block (descriptors, tasks, targets) new.
    int dev = 0;
    PYHEA_HIP(hipGetDevice(&dev));
    std::vector<int64_t> key = {dev, n, (int64_t)off, (int64_t)x_end, (int64_t)y_begin, (int64_t)y_end,
                                (int64_t)o_descs, (int64_t)o_tasks, (int64_t)o_tile0, (int64_t)o_bad, n_tiles,
                                count_tile, max_E};
    for (const Launch &L : launches)
        key.insert(key.end(), {L.first, L.count, L.store, L.M, L.S, L.B, L.W, L.bal, L.K, L.CH, L.lds});
    ChainPlan *plan = nullptr;
    if (graphs_enabled()) PYHEA_HIP(chain_plan(key, off, &plan));
    std::unique_lock<std::mutex> plan_lock;
    DeviceBuffer arena;
    arena.stream = stream;
    char *base;
    if (plan) {
        plan_lock = std::unique_lock<std::mutex>(plan->mu);
        base = (char *)plan->arena;
    } else {
        PYHEA_HIP(pool_alloc(&arena.ptr, off, stream));
        base = (char *)arena.ptr;
    }

    const CountTask *tasks = nullptr;
    const uint32_t *tile0 = nullptr;
    const ChainDesc *ddev = nullptr;
    auto rebase = [&](char *b) {
        base = b;
        tasks = (const CountTask *)(base + o_tasks);
        tile0 = (const uint32_t *)(base + o_tile0);
        ddev = (const ChainDesc *)(base + o_descs);
    };
    rebase(base);

    // the device work after the upload: zeroed read-back block; initial pair counts
    // of every chain's configuration in one launch, then the ratio tables from
    // them (an invalid chain is marked and skipped); the chains, one launch per
    // group, groups side by side on auxiliary streams; the states' final
    // objective; a fresh recount of every final configuration
    auto device_work = [&](hipStream_t s, const hipStream_t *aux_set) -> hipError_t {
        hipError_t e;
        if ((e = launch_zero_i32((int32_t *)base, (int64_t)(x_end / 4), s)) != hipSuccess) return e;
        if ((e = launch_count_tasks(tasks, tile0, n, n_tiles, count_tile, max_E, s)) != hipSuccess) return e;
        if ((e = launch_chain_ratio(ddev, n, (const int32_t *)(base + o_bad), s)) != hipSuccess) return e;
        {
            Fork fork;
            if ((e = fork.begin(s, (int)launches.size(), aux_set)) != hipSuccess) return e;
            for (size_t l = 0; l < launches.size(); ++l) {
                const Launch &L = launches[l];
                hipStream_t ls = fork.stream((int)l);
                if (L.store == kStoreGlobal && (e = launch_pad_fill(ddev + L.first, L.count, ls)) != hipSuccess)
                    return e;
                if ((e = launch_mc(ddev + L.first, L.count, L.store, L.M, L.S, L.B, L.W, L.bal, L.K, L.CH, L.lds,
                                   INT_MAX, ls)) != hipSuccess)
                    return e;
                if (L.store == kStoreGlobal && (e = launch_pad_drain(ddev + L.first, L.count, ls)) != hipSuccess)
                    return e;
            }
            if ((e = fork.end()) != hipSuccess) return e;
        }
        if ((e = launch_final_objective(ddev, n, s)) != hipSuccess) return e;
        return launch_count_tasks(tasks + n, tile0, n, n_tiles, count_tile, max_E, s);
    };
    if (plan && !plan->exec) {
        if (plan->failed || record_plan(plan, device_work) != hipSuccess) {
            plan->failed = true;
            // recording refused (now or before): this call, and later calls of the
            // structure, run eagerly
            (void)hipGetLastError();
            plan_lock.unlock();
            plan = nullptr;
            PYHEA_HIP(pool_alloc(&arena.ptr, off, stream));
            rebase((char *)arena.ptr);
        }
    }

    // block Y on the host: targets, chain descriptors (ordered by launch group), count
    // tasks; staged with the read-back block X in one page-locked lease
    const size_t ny = y_end - y_begin;
    PinnedLease lease;
    PYHEA_HIP(pinned_lease(ny + align256(x_end), stream, &lease));
    char *hyp = lease.b.p;
    char *hxp = lease.b.p + ny;
    std::memset(hyp, 0, ny);
    auto hy_at = [&](size_t o) { return hyp + (o - y_begin); };
    for (int c = 0; c < n; ++c)
        std::memcpy(hy_at(o_target) + eoff[c] * 8, jobs[c].target.data(), jobs[c].target.size() * 8);
    {
        ChainDesc *hd = (ChainDesc *)hy_at(o_descs);
        for (int c = 0; c < n; ++c) {
            const ChainJob &j = jobs[c];
            ChainDesc &d = hd[pos[c]];
            std::memset(&d, 0, sizeof(d));
            fill_chain_geometry(j.g, &d);
            d.seed = j.params.seed;
            d.chain_id = j.params.chain_id;
            d.B = j.params.cand_per_step;
            d.n_trials = j.params.n_trials;
            d.mode = j.params.commit_mode;
            d.depth_limit = j.params.depth_limit;
            d.tau = j.params.accept_tol;
            for (int k = 0; k < kMaxShells; ++k) d.w[k] = k < j.g.S ? j.weight[k] : 0.0;
            d.species = j.species_dev;
            d.pad_global = shape[c].store == kStoreGlobal ? (int8_t *)(base + o_pad[c]) : nullptr;
            d.R = (const double *)(base + o_R) + eoff[c];
            d.target = (const double *)(base + o_target) + eoff[c];
            d.counts = (int32_t *)(base + o_counts) + eoff[c];
            d.log = j.log_dev;
            d.log_cap = j.log_dev ? j.log_cap : 0;
            d.state = (ChainState *)(base + o_state) + c;
            d.store = shape[c].store;
            d.lds_bytes = shape[c].lds;
            d.sym = symmetric_target(j.target.data(), j.g.S, j.g.M);
        }
        CountTask *ht = (CountTask *)hy_at(o_tasks);
        uint32_t *t0 = (uint32_t *)hy_at(o_tile0);
        for (int c = 0; c < n; ++c) {
            CountTask &a = ht[c], &b = ht[n + c];
            fill_eval_desc(jobs[c].g, &a.ed);
            a.species = jobs[c].species_dev;
            a.counts = (int32_t *)(base + o_counts) + eoff[c];
            a.bad = (int32_t *)(base + o_bad) + pos[c];   // descriptor order, read by the ratio kernel
            b = a;
            b.counts = (int32_t *)(base + o_recount) + eoff[c];
            b.bad = (int32_t *)(base + o_bad2) + c;
            t0[c] = tile0v[c];
        }
    }
    bool replayed = false;
    PYHEA_HIP(hipMemcpyAsync(base + y_begin, hyp, ny, hipMemcpyHostToDevice, stream));
    if (plan) {
        PYHEA_HIP(hipGraphLaunch(plan->exec, stream));
        replayed = true;
    } else {
        PYHEA_HIP(device_work(stream, nullptr));
    }
    PYHEA_HIP(hipMemcpyAsync(hxp, base, x_end, hipMemcpyDeviceToHost, stream));
    PYHEA_HIP(hipStreamSynchronize(stream));
    lease.drained = true;
    const int32_t *cnt = (const int32_t *)(hxp + o_counts);
    const int32_t *rec = (const int32_t *)(hxp + o_recount);
    const ChainState *sts = (const ChainState *)(hxp + o_state);
    if (final_counts) final_counts->assign(n, {});
    int first_invalid = -1;
    for (int c = 0; c < n; ++c) {
        pyhea_mc_stats &s = stats[c];
        if (sts[c].status != 0) {   // invalid ids or an absent species: the chain did not run
            std::memset(&s, 0, sizeof(s));
            s.status = sts[c].status;
            if (first_invalid < 0) first_invalid = c;
            continue;
        }
        if (!std::equal(cnt + eoff[c], cnt + eoff[c + 1], rec + eoff[c])) {
            set_error("chain " + std::to_string(c) + ": maintained pair counts differ from a recount");
            return PYHEA_EDEVICE;
        }
        std::vector<int64_t> c64(rec + eoff[c], rec + eoff[c + 1]);
        std::memset(&s, 0, sizeof(s));
        s.trials = sts[c].trials;
        s.null_trials = sts[c].null_trials;
        s.commits = sts[c].commits;
        s.steps = sts[c].steps;
        s.stop_reason = sts[c].stop_reason;
        s.status = PYHEA_OK;
        s.S = sts[c].S;
        s.F = sts[c].F;
        s.log_len = jobs[c].log_dev ? std::min(s.commits, jobs[c].log_cap) : 0;
        s.shape = shape_code(shape[c]);
        s.shape_measured = measured[c];
        s.graph = replayed ? 1 : 0;
        if (final_counts) (*final_counts)[c] = c64;
    }
    if (first_invalid >= 0) {
        set_error("chain " + std::to_string(first_invalid) +
                  ": species ids must lie in [0, n_species) and every species must occur (that chain and any other "
                  "invalid one were left unchanged; the valid chains ran)");
        return PYHEA_EINVAL;
    }
    return PYHEA_OK;
}

}  // namespace pyhea
