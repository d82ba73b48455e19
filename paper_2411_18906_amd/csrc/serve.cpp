// Serving API: continuous batching of Monte Carlo structure-generation jobs.
//
// A worker thread owns the GPU work.  Each round it (1) retires jobs whose
// chains finished in the previous round (results copied to host, device
// memory released), (2) admits queued jobs in arrival order while a slot is
// free and their HBM footprint fits the budget (configuration, padded copy,
// counts and tables stay resident on the device), and (3) advances every
// resident job with one persistent launch per launch shape, the shapes on
// separate streams so they overlap.  The launch whose chains take longest per
// step runs `steps_per_round` steps; every other launch runs as many more
// steps (up to kMaxStepScale times as many) as its chains' measured time per
// step allows in the same time, so that a round's launches end together
// instead of the fast ones idling until the slowest ends.  A job's
// trajectory depends only on its own inputs (seed, chain id = job id, B,
// budget): rounds are cut at step boundaries and the chain state (step, trial
// and depth counters, counts, configuration) persists between launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <climits>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "pyhea.h"
#include "autotune.h"
#include "runtime.h"

using namespace pyhea;

namespace {

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

enum JobPhase { kQueued, kResident, kDone, kCancelled, kFailed };

// One device allocation per resident job:
//   small block: counts | recount | bad | bad2 | state | R | target
//   species (N bytes), then the padded HBM copy for jobs that keep it in HBM.
struct JobLayout {
    size_t counts, recount, bad, bad2, state, R, target, small_end, species, pad, total;
};

JobLayout job_layout(const Geometry &g, int store) {
    const size_t E = (size_t)g.S * g.M * g.M;
    JobLayout l;
    size_t off = 0;
    l.counts = off;
    off += E * 4;
    l.recount = off;
    off += E * 4;
    l.bad = off;
    off += 4;
    l.bad2 = off;
    off += 4;
    off = (off + 7) & ~size_t(7);
    l.state = off;
    off += sizeof(ChainState);
    l.R = off;
    off += E * 8;
    l.target = off;
    off += E * 8;
    l.small_end = off;
    off = (off + 255) & ~size_t(255);
    l.species = off;
    off += (size_t)g.N;
    off = (off + 255) & ~size_t(255);
    l.pad = off;
    if (store == kStoreGlobal) off += (size_t)g.Npad;
    l.total = (off + 255) & ~size_t(255);
    return l;
}

struct Job {
    uint64_t id = 0;
    Geometry g;
    pyhea_mc_params params{};
    std::vector<double> target, weight;
    std::vector<int8_t> species;  // input, then the final configuration
    JobPhase phase = kQueued;
    bool cancel = false;
    int32_t status = PYHEA_OK;
    pyhea_mc_stats stats{};
    int64_t t_submit = 0, t_admit = 0, t_finish = 0;
    // device residency
    int64_t footprint = 0;
    void *mem = nullptr;
    ChainDesc desc{};
    int store = kStoreLds8;
    int lds = 0;
    int W = 1, bal = 0, K = 1, CH = 0;
    int shape_measured = 0;
    JobLayout lay{};
};

int64_t job_footprint(const Geometry &g, int store) { return (int64_t)job_layout(g, store).total; }

// Streams a round's launches are spread over.  The HIP runtime serves a
// process's streams from a fixed number of hardware queues (GPU_MAX_HW_QUEUES,
// 4 unless the environment sets more) and launches that share a queue run one
// after another, so the launches overlap as far as the queues allow.
constexpr int kServeStreams = 16;
// A launch runs at most this many times the round's base step count.
constexpr int kMaxStepScale = 16;

// The launch shape of a group of resident jobs (one persistent launch each round).
using GroupKey = std::tuple<int, int, int, int, int, int, int, int>;

struct Server {
    int device = 0;
    int64_t budget = 0;
    int max_slots = 0;
    int steps_per_round = 256;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::unordered_map<uint64_t, std::unique_ptr<Job>> jobs;
    std::deque<uint64_t> queue;
    std::vector<Job *> resident;
    bool stop = false;
    int pollers = 0;   // threads blocked in pyhea_serve_poll (close waits for them to leave)
    std::thread worker;
    int64_t n_submitted = 0, n_admitted = 0, n_finished = 0, n_rejected = 0, n_rounds = 0;
    int64_t bytes_resident = 0;
    std::vector<hipStream_t> streams;
    // milliseconds per MC step of each launch shape's last launches (a running
    // mean), and the events that time each launch of a round
    std::map<GroupKey, double> ms_per_step;
    std::vector<hipEvent_t> events;
    // device tables sized for max_slots: the round's descriptors, their gathered
    // states, and (for admission and retirement) descriptors and count tasks
    void *desc_dev = nullptr, *state_dev = nullptr, *aux_desc_dev = nullptr, *task_dev = nullptr;
    int lds_budget = 0;
    std::string worker_error;

    void run();
    // admits `js` (device memory, uploads, initial counts); returns per job success
    std::vector<bool> admit(const std::vector<Job *> &js, hipStream_t s);
    void retire(const std::vector<Job *> &js, hipStream_t s);
    void release(Job *j, hipStream_t s);
};

void fill_desc(Job *j) {
    const Geometry &g = j->g;
    char *base = (char *)j->mem;
    ChainDesc &d = j->desc;
    std::memset(&d, 0, sizeof(d));
    fill_chain_geometry(g, &d);
    d.seed = j->params.seed;
    d.chain_id = j->params.chain_id;
    d.B = j->params.cand_per_step;
    d.n_trials = j->params.n_trials;
    d.mode = j->params.commit_mode;
    d.depth_limit = j->params.depth_limit;
    d.tau = j->params.accept_tol;
    for (int k = 0; k < kMaxShells; ++k) d.w[k] = k < g.S ? j->weight[k] : 0.0;
    d.species = (int8_t *)(base + j->lay.species);
    d.pad_global = j->store == kStoreGlobal ? (int8_t *)(base + j->lay.pad) : nullptr;
    d.R = (const double *)(base + j->lay.R);
    d.target = (const double *)(base + j->lay.target);
    d.counts = (int32_t *)(base + j->lay.counts);
    d.log = nullptr;
    d.log_cap = 0;
    d.state = (ChainState *)(base + j->lay.state);
    d.store = j->store;
    d.lds_bytes = j->lds;
    d.sym = symmetric_target(j->target.data(), g.S, g.M);
}

CountTask count_task(const Job *j, bool recount) {
    CountTask t;
    fill_eval_desc(j->g, &t.ed);
    char *base = (char *)j->mem;
    t.species = (const int8_t *)(base + j->lay.species);
    t.counts = (int32_t *)(base + (recount ? j->lay.recount : j->lay.counts));
    t.bad = (int32_t *)(base + (recount ? j->lay.bad2 : j->lay.bad));
    return t;
}

// Pair counts of the given jobs' configurations in one launch.
bool count_jobs(const std::vector<Job *> &js, bool recount, void *task_dev, hipStream_t s) {
    if (js.empty()) return true;
    const size_t n = js.size();
    std::vector<char> host(n * sizeof(CountTask) + n * 4);
    CountTask *t = (CountTask *)host.data();
    uint32_t *t0 = (uint32_t *)(host.data() + n * sizeof(CountTask));
    uint64_t total_sites = 0;
    int max_E = 0;
    for (size_t i = 0; i < n; ++i) {
        total_sites += (uint64_t)js[i]->g.N;
        max_E = std::max(max_E, js[i]->g.S * js[i]->g.M * js[i]->g.M);
    }
    const uint32_t tile = count_tile_for(total_sites);
    uint32_t tiles = 0;
    for (size_t i = 0; i < n; ++i) {
        t[i] = count_task(js[i], recount);
        t0[i] = tiles;
        tiles += count_tiles((uint32_t)js[i]->g.N, tile);
    }
    bool ok = hipMemcpyAsync(task_dev, host.data(), host.size(), hipMemcpyHostToDevice, s) == hipSuccess;
    ok = ok && launch_count_tasks((const CountTask *)task_dev,
                                  (const uint32_t *)((char *)task_dev + n * sizeof(CountTask)), (int)n, tiles, tile,
                                  max_E, s) == hipSuccess;
    return ok;
}

std::vector<bool> Server::admit(const std::vector<Job *> &js, hipStream_t s) {
    std::vector<bool> good(js.size(), false);
    std::vector<Job *> live;
    std::vector<ChainDesc> pads;
    for (size_t i = 0; i < js.size(); ++i) {
        Job *j = js[i];
        const Geometry &g = j->g;
        j->lay = job_layout(g, j->store);
        if (pool_alloc(&j->mem, j->lay.total, s) != hipSuccess) {
            j->mem = nullptr;
            continue;
        }
        char *base = (char *)j->mem;
        // zeroed counts, flags and state, then R (n_i from the host copy) and the target
        const size_t E = (size_t)g.S * g.M * g.M;
        std::vector<char> small(j->lay.small_end, 0);
        int64_t n[kMaxSpecies] = {0};
        for (int8_t v : j->species) n[v]++;
        ratio_table(g, n, (double *)(small.data() + j->lay.R));
        std::memcpy(small.data() + j->lay.target, j->target.data(), E * 8);
        // host memory is pageable, so both copies complete before they return
        bool ok = hipMemcpyAsync(base, small.data(), small.size(), hipMemcpyHostToDevice, s) == hipSuccess;
        ok = ok && hipMemcpyAsync(base + j->lay.species, j->species.data(), g.N, hipMemcpyHostToDevice, s) ==
                       hipSuccess;
        if (!ok) {
            (void)hipFreeAsync(j->mem, s);
            j->mem = nullptr;
            continue;
        }
        fill_desc(j);
        if (j->store == kStoreGlobal) pads.push_back(j->desc);
        live.push_back(j);
        good[i] = true;
    }
    bool ok = count_jobs(live, false, task_dev, s);
    if (ok && !pads.empty()) {
        ok = hipMemcpyAsync(aux_desc_dev, pads.data(), pads.size() * sizeof(ChainDesc), hipMemcpyHostToDevice, s) ==
             hipSuccess;
        ok = ok && launch_pad_fill((const ChainDesc *)aux_desc_dev, (int)pads.size(), s) == hipSuccess;
    }
    ok = ok && hipStreamSynchronize(s) == hipSuccess;
    if (!ok) std::fill(good.begin(), good.end(), false);
    return good;
}

void Server::retire(const std::vector<Job *> &js, hipStream_t s) {
    if (js.empty()) return;
    std::vector<ChainDesc> pads;
    for (Job *j : js)
        if (j->store == kStoreGlobal) pads.push_back(j->desc);
    bool ok = true;
    if (!pads.empty()) {
        ok = hipMemcpyAsync(aux_desc_dev, pads.data(), pads.size() * sizeof(ChainDesc), hipMemcpyHostToDevice, s) ==
             hipSuccess;
        ok = ok && launch_pad_drain((const ChainDesc *)aux_desc_dev, (int)pads.size(), s) == hipSuccess;
    }
    ok = ok && count_jobs(js, true, task_dev, s);
    // S and F of the final counts into each job's state
    std::vector<ChainDesc> ds;
    for (Job *j : js) ds.push_back(j->desc);
    ok = ok && hipMemcpyAsync(aux_desc_dev, ds.data(), ds.size() * sizeof(ChainDesc), hipMemcpyHostToDevice, s) ==
                   hipSuccess;
    ok = ok && launch_final_objective((const ChainDesc *)aux_desc_dev, (int)ds.size(), s) == hipSuccess;
    std::vector<std::vector<char>> small(js.size());
    for (size_t i = 0; ok && i < js.size(); ++i) {
        Job *j = js[i];
        small[i].resize(j->lay.R);  // counts, recount, flags, state
        ok = hipMemcpyAsync(small[i].data(), j->mem, small[i].size(), hipMemcpyDeviceToHost, s) == hipSuccess;
        ok = ok && hipMemcpyAsync(j->species.data(), (char *)j->mem + j->lay.species, j->g.N,
                                  hipMemcpyDeviceToHost, s) == hipSuccess;
    }
    ok = ok && hipStreamSynchronize(s) == hipSuccess;
    for (size_t i = 0; i < js.size(); ++i) {
        Job *j = js[i];
        std::memset(&j->stats, 0, sizeof(j->stats));
        const Geometry &g = j->g;
        const size_t E = (size_t)g.S * g.M * g.M;
        const int32_t *cm = ok ? (const int32_t *)(small[i].data() + j->lay.counts) : nullptr;
        const int32_t *cr = ok ? (const int32_t *)(small[i].data() + j->lay.recount) : nullptr;
        if (!ok || !std::equal(cm, cm + E, cr)) {
            j->status = PYHEA_EDEVICE;
        } else {
            ChainState st;
            std::memcpy(&st, small[i].data() + j->lay.state, sizeof(st));
            j->stats.trials = st.trials;
            j->stats.null_trials = st.null_trials;
            j->stats.commits = st.commits;
            j->stats.steps = st.steps;
            j->stats.stop_reason = st.stop_reason;
            j->stats.S = st.S;
            j->stats.F = st.F;
        }
        j->stats.shape = j->store * 10000 + j->K * 100 + j->CH;
        j->stats.shape_measured = j->shape_measured;
        j->stats.status = j->status;
    }
}

void Server::release(Job *j, hipStream_t s) {
    if (j->mem) (void)hipFreeAsync(j->mem, s);
    j->mem = nullptr;
    bytes_resident -= j->footprint;
}

void Server::run() {
    (void)hipSetDevice(device);
    hipStream_t s0 = streams[0];
    std::vector<ChainState> states;
    for (;;) {
        std::vector<Job *> to_admit;
        {
            std::unique_lock<std::mutex> lk(mu);
            // admit in arrival order while slots and budget allow
            for (auto it = queue.begin(); it != queue.end();) {
                Job *j = jobs.count(*it) ? jobs[*it].get() : nullptr;
                if (!j || j->phase != kQueued) {
                    it = queue.erase(it);
                    continue;
                }
                if ((int)(resident.size() + to_admit.size()) >= max_slots) break;
                if (bytes_resident + j->footprint > budget) {
                    ++it;
                    continue;
                }
                bytes_resident += j->footprint;
                to_admit.push_back(j);
                it = queue.erase(it);
            }
            if (resident.empty() && to_admit.empty()) {
                if (stop) return;
                cv_work.wait(lk, [&] { return stop || !queue.empty(); });
                if (stop && queue.empty()) return;
                continue;
            }
        }
        if (!to_admit.empty()) {
            const std::vector<bool> good = admit(to_admit, s0);
            std::lock_guard<std::mutex> lk(mu);
            const int64_t t = now_ns();
            for (size_t i = 0; i < to_admit.size(); ++i) {
                Job *j = to_admit[i];
                if (!good[i]) {
                    release(j, s0);
                    j->status = PYHEA_ENOMEM;
                    j->phase = kFailed;
                    j->t_finish = t;
                    ++n_finished;
                    continue;
                }
                j->phase = kResident;
                j->t_admit = t;
                resident.push_back(j);
                ++n_admitted;
            }
            cv_done.notify_all();
        }
        std::vector<Job *> run_set;
        {
            std::lock_guard<std::mutex> lk(mu);
            run_set = resident;
            if (stop) run_set.clear();
        }
        if (run_set.empty()) {
            std::lock_guard<std::mutex> lk(mu);
            if (stop) return;
            continue;
        }
        // one round: group by launch shape, one stream per group
        std::map<GroupKey, std::vector<Job *>> groups;
        for (Job *j : run_set)
            groups[{j->store, j->g.M, j->g.S, j->params.cand_per_step, j->W, j->bal, j->K, j->CH}].push_back(j);
        std::vector<ChainDesc> descs;
        std::vector<Job *> order;
        std::vector<std::pair<size_t, std::vector<Job *>>> launches;
        std::vector<GroupKey> keys;
        for (auto &kv : groups) {
            keys.push_back(kv.first);
            launches.push_back({descs.size(), kv.second});
            for (Job *j : kv.second) {
                descs.push_back(j->desc);
                order.push_back(j);
            }
        }
        // steps per launch: the slowest measured shape runs the base count, the
        // others as many steps as fit in the time it takes (shapes not yet
        // measured run the base count)
        std::vector<int> steps(launches.size(), steps_per_round);
        {
            double t_round = 0.0;
            for (const GroupKey &k : keys) {
                auto it = ms_per_step.find(k);
                if (it != ms_per_step.end()) t_round = std::max(t_round, it->second * steps_per_round);
            }
            for (size_t gi = 0; gi < launches.size(); ++gi) {
                auto it = ms_per_step.find(keys[gi]);
                if (it == ms_per_step.end() || !(it->second > 0.0)) continue;
                const double n = std::floor(t_round / it->second);
                const double cap = std::min<double>((double)steps_per_round * kMaxStepScale, (double)(INT_MAX / 2));
                steps[gi] = (int)std::min<double>(cap, std::max<double>((double)steps_per_round, n));
            }
        }
        while (events.size() < 2 * launches.size()) {
            hipEvent_t e = nullptr;
            if (hipEventCreate(&e) != hipSuccess) break;
            events.push_back(e);
        }
        const bool timed = events.size() >= 2 * launches.size();
        bool ok = hipMemcpyAsync(desc_dev, descs.data(), descs.size() * sizeof(ChainDesc), hipMemcpyHostToDevice,
                                 s0) == hipSuccess;
        hipEvent_t ready = nullptr;
        ok = ok && hipEventCreateWithFlags(&ready, hipEventDisableTiming) == hipSuccess;
        ok = ok && hipEventRecord(ready, s0) == hipSuccess;
        for (size_t gi = 0; ok && gi < launches.size(); ++gi) {
            auto &L = launches[gi];
            const Job *j0 = L.second[0];
            int lds = 0;
            for (Job *j : L.second) lds = std::max(lds, j->lds);
            hipStream_t s = streams[gi % streams.size()];
            ok = s == s0 || hipStreamWaitEvent(s, ready, 0) == hipSuccess;
            if (timed) ok = ok && hipEventRecord(events[2 * gi], s) == hipSuccess;
            ok = ok && launch_mc((const ChainDesc *)desc_dev + L.first, (int)L.second.size(), j0->store, j0->g.M,
                                 j0->g.S, j0->params.cand_per_step, j0->W, j0->bal, j0->K, j0->CH, lds,
                                 steps[gi], s) == hipSuccess;
            if (timed) ok = ok && hipEventRecord(events[2 * gi + 1], s) == hipSuccess;
        }
        for (size_t i = 0; i < streams.size(); ++i) ok = ok && hipStreamSynchronize(streams[i]) == hipSuccess;
        if (ready) (void)hipEventDestroy(ready);
        // every job's state in one read-back
        states.resize(order.size());
        ok = ok && launch_gather_states((const ChainDesc *)desc_dev, (int)order.size(), (ChainState *)state_dev,
                                        s0) == hipSuccess;
        ok = ok && hipMemcpyAsync(states.data(), state_dev, order.size() * sizeof(ChainState), hipMemcpyDeviceToHost,
                                  s0) == hipSuccess;
        ok = ok && hipStreamSynchronize(s0) == hipSuccess;
        // time per step of each shape, from launches in which no chain ended early
        if (ok && timed) {
            size_t at = 0;
            for (size_t gi = 0; gi < launches.size(); ++gi) {
                bool ended = false;
                for (size_t i = 0; i < launches[gi].second.size(); ++i) ended = ended || states[at + i].done;
                at += launches[gi].second.size();
                float ms = 0.0f;
                if (ended || hipEventElapsedTime(&ms, events[2 * gi], events[2 * gi + 1]) != hipSuccess) continue;
                const double v = (double)ms / steps[gi];
                auto it = ms_per_step.find(keys[gi]);
                if (it == ms_per_step.end())
                    ms_per_step[keys[gi]] = v;
                else
                    it->second = 0.5 * (it->second + v);
            }
        }
        std::vector<Job *> finished, cancelled;
        {
            std::lock_guard<std::mutex> lk(mu);
            ++n_rounds;
            for (size_t i = 0; i < order.size(); ++i) {
                Job *j = order[i];
                if (!ok) {
                    j->status = PYHEA_EDEVICE;
                    finished.push_back(j);
                } else if (j->cancel) {
                    cancelled.push_back(j);
                } else if (states[i].done) {
                    finished.push_back(j);
                }
            }
        }
        std::vector<Job *> good;
        for (Job *j : finished)
            if (j->status == PYHEA_OK) good.push_back(j);
        retire(good, s0);
        {
            std::lock_guard<std::mutex> lk(mu);
            const int64_t t = now_ns();
            for (Job *j : finished) {
                j->phase = j->status == PYHEA_OK ? kDone : kFailed;
                j->stats.status = j->status;
                j->t_finish = t;
                release(j, s0);
                resident.erase(std::find(resident.begin(), resident.end(), j));
                ++n_finished;
            }
            for (Job *j : cancelled) {
                release(j, s0);
                j->phase = kCancelled;
                j->status = PYHEA_ECANCELLED;
                j->t_finish = t;
                resident.erase(std::find(resident.begin(), resident.end(), j));
                ++n_finished;
            }
            if (!ok) worker_error = "device error during a serving round";
        }
        cv_done.notify_all();
    }
}

Server *as_server(void *p) { return static_cast<Server *>(p); }

}  // namespace

extern "C" {

pyhea_status pyhea_serve_open(int64_t hbm_budget_bytes, int32_t max_slots, int32_t steps_per_round,
                              void **server) {
    if (!server || hbm_budget_bytes <= 0 || max_slots < 1 || max_slots > 65535 || steps_per_round < 0) {
        set_error("serve_open: need server != NULL, budget > 0, 1 <= max_slots <= 65535, steps_per_round >= 0");
        return PYHEA_EINVAL;
    }
    auto *s = new Server();
    PYHEA_HIP(hipGetDevice(&s->device));
    s->budget = hbm_budget_bytes;
    s->max_slots = max_slots;
    s->steps_per_round = steps_per_round > 0 ? steps_per_round : 256;
    s->lds_budget = max_lds_per_block();
    s->streams.resize(kServeStreams);  // [0]: admission, retirement and read-back; all: the rounds' launches
    for (auto &st : s->streams) {
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            delete s;
            set_error("serve_open: stream creation failed");
            return PYHEA_EDEVICE;
        }
    }
    const size_t slots = (size_t)max_slots;
    if (hipMalloc(&s->desc_dev, sizeof(ChainDesc) * slots) != hipSuccess ||
        hipMalloc(&s->state_dev, sizeof(ChainState) * slots) != hipSuccess ||
        hipMalloc(&s->aux_desc_dev, sizeof(ChainDesc) * slots) != hipSuccess ||
        hipMalloc(&s->task_dev, (sizeof(CountTask) + 4) * slots) != hipSuccess) {
        for (void *p : {s->desc_dev, s->state_dev, s->aux_desc_dev, s->task_dev})
            if (p) (void)hipFree(p);
        for (auto st : s->streams) (void)hipStreamDestroy(st);
        delete s;
        set_error("serve_open: table allocation failed");
        return PYHEA_ENOMEM;
    }
    s->worker = std::thread([s] { s->run(); });
    *server = s;
    set_error("");
    return PYHEA_OK;
}

pyhea_status pyhea_serve_submit(void *server, uint64_t job_id, const pyhea_lattice *lat, const pyhea_objective *obj,
                                const pyhea_mc_params *params, const int8_t *species_host) {
    Server *s = as_server(server);
    if (!s || !species_host) {
        set_error("serve_submit: server and species_host must not be NULL");
        return PYHEA_EINVAL;
    }
    auto j = std::make_unique<Job>();
    std::string err;
    if (build_geometry(lat, &j->g, &err) != PYHEA_OK) {
        set_error("serve_submit: " + err);
        std::lock_guard<std::mutex> lk(s->mu);
        ++s->n_rejected;
        return PYHEA_EINVAL;
    }
    pyhea_status st = check_objective(j->g, obj);
    if (st == PYHEA_OK) st = check_params(params);
    if (st != PYHEA_OK) {
        std::lock_guard<std::mutex> lk(s->mu);
        ++s->n_rejected;
        return st;
    }
    const Geometry &g = j->g;
    j->species.assign(species_host, species_host + g.N);
    int64_t n[kMaxSpecies] = {0};
    for (int8_t v : j->species) {
        if (v < 0 || v >= g.M) {
            set_error("serve_submit: species ids must lie in [0, n_species)");
            std::lock_guard<std::mutex> lk(s->mu);
            ++s->n_rejected;
            return PYHEA_EINVAL;
        }
        n[v]++;
    }
    for (int i = 0; i < g.M; ++i)
        if (n[i] == 0) {
            set_error("serve_submit: every species must occur");
            std::lock_guard<std::mutex> lk(s->mu);
            ++s->n_rejected;
            return PYHEA_EINVAL;
        }
    j->id = job_id;
    j->params = *params;
    j->params.chain_id = (uint32_t)job_id;
    const int E = g.S * g.M * g.M;
    j->target.assign(obj->target, obj->target + E);
    j->weight.assign(obj->weight, obj->weight + g.S);
    // shapes for a full server (max_slots chains resident) keep small chains'
    // workgroups narrow so that many share a CU; a job whose configuration
    // lives in HBM takes the shape of a chain with a CU to itself (more steps
    // per pass): such jobs are few under any HBM budget, and their time per step
    // sets the pace of a round
    LaunchShape ls = choose_launch(g, params->cand_per_step, s->lds_budget, 0, s->max_slots);
    if (ls.store == kStoreGlobal) ls = choose_launch(g, params->cand_per_step, s->lds_budget, 0, 256);
    // a shape measured earlier for this kind of chain (the server itself never probes)
    LaunchShape t;
    if (measure_enabled() && tuned_launch(tune_key(g, params->cand_per_step, s->max_slots), &t)) {
        t.lds = (int)launch_lds_bytes(g, params->cand_per_step, t);
        if (t.lds <= s->lds_budget && t.W == g.S) {
            ls = t;
            j->shape_measured = 1;
        }
    }
    j->store = ls.store;
    j->lds = ls.lds;
    j->W = ls.W;
    j->bal = ls.bal;
    j->CH = ls.CH;
    j->K = ls.K;
    j->footprint = job_footprint(g, j->store);
    std::lock_guard<std::mutex> lk(s->mu);
    if (j->footprint > s->budget) {
        set_error("serve_submit: the job's HBM footprint exceeds the server budget");
        ++s->n_rejected;
        return PYHEA_ENOMEM;
    }
    if (s->jobs.count(job_id)) {
        set_error("serve_submit: duplicate job id");
        ++s->n_rejected;
        return PYHEA_EINVAL;
    }
    j->t_submit = now_ns();
    s->queue.push_back(job_id);
    s->jobs[job_id] = std::move(j);
    ++s->n_submitted;
    s->cv_work.notify_all();
    set_error("");
    return PYHEA_OK;
}

pyhea_status pyhea_serve_poll(void *server, uint64_t job_id, int8_t *species_out_host, pyhea_mc_stats *stats_host,
                              int64_t *times_ns_host, int32_t blocking) {
    Server *s = as_server(server);
    if (!s) {
        set_error("serve_poll: server must not be NULL");
        return PYHEA_EINVAL;
    }
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->jobs.find(job_id);
    if (it == s->jobs.end()) {
        set_error("serve_poll: unknown job id");
        return PYHEA_ENOENT;
    }
    Job *j = it->second.get();
    auto finished = [&] { return j->phase == kDone || j->phase == kCancelled || j->phase == kFailed; };
    if (!finished()) {
        if (!blocking) return PYHEA_EBUSY;
        // close() marks every unfinished job cancelled and then waits until no
        // poller is left inside the server before freeing it
        ++s->pollers;
        s->cv_done.wait(lk, [&] { return finished() || s->stop; });
        --s->pollers;
        if (s->pollers == 0) s->cv_done.notify_all();
        if (!finished()) {
            set_error("serve_poll: server stopped");
            return PYHEA_EDEVICE;
        }
    }
    if (stats_host) *stats_host = j->stats;
    if (times_ns_host) {
        times_ns_host[0] = j->t_submit;
        times_ns_host[1] = j->t_admit;
        times_ns_host[2] = j->t_finish;
    }
    const int32_t status = j->phase == kCancelled ? PYHEA_ECANCELLED : j->status;
    if (species_out_host && j->phase == kDone) std::memcpy(species_out_host, j->species.data(), j->g.N);
    s->jobs.erase(it);
    if (status != PYHEA_OK) set_error("serve_poll: job ended with an error");
    return status;
}

pyhea_status pyhea_serve_cancel(void *server, uint64_t job_id) {
    Server *s = as_server(server);
    if (!s) return PYHEA_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(job_id);
    if (it == s->jobs.end()) {
        set_error("serve_cancel: unknown job id");
        return PYHEA_ENOENT;
    }
    Job *j = it->second.get();
    if (j->phase == kQueued) {
        j->phase = kCancelled;
        j->status = PYHEA_ECANCELLED;
        j->t_finish = now_ns();
        ++s->n_finished;
        s->cv_done.notify_all();
    } else if (j->phase == kResident) {
        j->cancel = true;
    }
    return PYHEA_OK;
}

pyhea_status pyhea_serve_counters(void *server, int64_t *out8_host) {
    Server *s = as_server(server);
    if (!s || !out8_host) return PYHEA_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    int64_t queued = 0;
    for (auto &kv : s->jobs) queued += kv.second->phase == kQueued;
    out8_host[0] = s->n_submitted;
    out8_host[1] = s->n_admitted;
    out8_host[2] = s->n_finished;
    out8_host[3] = s->n_rejected;
    out8_host[4] = (int64_t)s->resident.size();
    out8_host[5] = queued;
    out8_host[6] = s->n_rounds;
    out8_host[7] = s->bytes_resident;
    return PYHEA_OK;
}

pyhea_status pyhea_serve_close(void *server) {
    Server *s = as_server(server);
    if (!s) return PYHEA_EINVAL;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->queue.clear();
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    (void)hipSetDevice(s->device);
    {
        // resident jobs give back their device memory; unfinished jobs end as
        // cancelled; blocked pollers wake, read that and leave before the
        // server is freed
        std::unique_lock<std::mutex> lk(s->mu);
        for (Job *j : s->resident) {
            if (j->mem) (void)hipFreeAsync(j->mem, s->streams[0]);
            j->mem = nullptr;
        }
        s->resident.clear();
        const int64_t t = now_ns();
        for (auto &kv : s->jobs) {
            Job *j = kv.second.get();
            if (j->phase == kQueued || j->phase == kResident) {
                j->phase = kCancelled;
                j->status = PYHEA_ECANCELLED;
                j->t_finish = t;
            }
        }
        s->cv_done.notify_all();
        s->cv_done.wait(lk, [&] { return s->pollers == 0; });
    }
    (void)hipStreamSynchronize(s->streams[0]);
    for (void *p : {s->desc_dev, s->state_dev, s->aux_desc_dev, s->task_dev})
        if (p) (void)hipFree(p);
    for (hipEvent_t e : s->events) (void)hipEventDestroy(e);
    for (auto st : s->streams) (void)hipStreamDestroy(st);
    delete s;
    return PYHEA_OK;
}

}  // extern "C"
