// C ABI of the pyhea library (see include/pyhea.h for the contract of every
// entry point).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <mutex>
#include <string>
#include <vector>

#include "autotune.h"
#include "pyhea.h"
#include "runtime.h"
#include "sites.h"

namespace pyhea {
const std::string &last_error();
}

using namespace pyhea;

namespace {

hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

struct AsyncBuffer {
    void *ptr = nullptr;
    hipStream_t stream = nullptr;
    ~AsyncBuffer() {
        if (ptr) (void)hipFreeAsync(ptr, stream);
    }
};

pyhea_status guard(pyhea_status s) {
    if (s == PYHEA_OK) set_error("");
    return s;
}

}  // namespace

extern "C" {

int32_t pyhea_version(void) { return 1 * 10000 + 0 * 100 + 0; }

const char *pyhea_last_error(void) { return pyhea::last_error().c_str(); }

pyhea_status pyhea_sro_eval(const pyhea_lattice *lat, const int8_t *species_dev, const pyhea_objective *obj,
                            int64_t *counts_host, double *alpha_host, double *S_F_host, void *stream_) {
    Geometry g;
    std::string err;
    if (build_geometry(lat, &g, &err) != PYHEA_OK) {
        set_error(err);
        return PYHEA_EINVAL;
    }
    if (!species_dev) {
        set_error("species_dev must not be NULL");
        return PYHEA_EINVAL;
    }
    if (obj) {
        const pyhea_status s = check_objective(g, obj);
        if (s != PYHEA_OK) return s;
    }
    hipStream_t stream = as_stream(stream_);
    const int E = g.S * g.M * g.M;
    // device block: counts [E] | bad | alpha [E] | S, F | target [E], weight [S]
    const size_t o_bad = ((size_t)E * 4 + 7) & ~size_t(7);
    const size_t o_alpha = o_bad + 8;
    const size_t o_sf = o_alpha + (size_t)E * 8;
    const size_t o_tw = o_sf + 16;
    AsyncBuffer buf;
    buf.stream = stream;
    PYHEA_HIP(pool_alloc(&buf.ptr, o_tw + (size_t)(E + kMaxShells) * 8, stream));
    char *base = (char *)buf.ptr;
    int32_t *counts = (int32_t *)base;
    int32_t *bad = (int32_t *)(base + o_bad);
    double *tdev = (double *)(base + o_tw);
    {
        const pyhea_status s = count_configs(g, 1, species_dev, counts, bad, stream);
        if (s != PYHEA_OK) return s;
    }
    if (obj) {
        SmallTable tw{};
        std::memcpy(tw.v, obj->target, E * 8);
        std::memcpy(tw.v + E, obj->weight, g.S * 8);
        PYHEA_HIP(launch_upload(tw, E + kMaxShells, tdev, stream));
    }
    // alpha, S and F (Eq. 2-3) on the device, then one read-back
    EvalDesc ed;
    fill_eval_desc(g, &ed);
    PYHEA_HIP(launch_objective_epilogue(ed, 1, counts, bad, obj ? tdev : nullptr, obj ? tdev + E : nullptr,
                                        (double *)(base + o_sf), (double *)(base + o_alpha), stream));
    std::vector<char> h(o_tw);
    PYHEA_HIP(hipMemcpyAsync(h.data(), base, o_tw, hipMemcpyDeviceToHost, stream));
    PYHEA_HIP(hipStreamSynchronize(stream));
    const int32_t *c32 = (const int32_t *)h.data();
    int32_t badh;
    std::memcpy(&badh, h.data() + o_bad, 4);
    std::vector<int64_t> c64(c32, c32 + E);
    int64_t n[kMaxSpecies];
    if (badh || !species_totals(g, c64.data(), n)) {
        set_error("species ids must lie in [0, n_species) and every species must occur");
        return PYHEA_EINVAL;
    }
    if (counts_host) std::memcpy(counts_host, c64.data(), E * 8);
    if (alpha_host) std::memcpy(alpha_host, h.data() + o_alpha, E * 8);
    if (obj && S_F_host) std::memcpy(S_F_host, h.data() + o_sf, 16);
    return guard(PYHEA_OK);
}

} // extern "C"

namespace {

// Argument checks shared by the two batched evaluation entry points.
pyhea_status check_eval_batch(const pyhea_lattice *lat, int64_t n_configs, const int8_t *species_dev,
                              const pyhea_objective *obj, int32_t *counts_dev, double *S_F_dev, Geometry *g) {
    std::string err;
    if (build_geometry(lat, g, &err) != PYHEA_OK) {
        set_error(err);
        return PYHEA_EINVAL;
    }
    if (n_configs < 0 || (n_configs > 0 && (!species_dev || !counts_dev))) {
        set_error("n_configs must be >= 0 and species_dev/counts_dev non-NULL");
        return PYHEA_EINVAL;
    }
    if ((obj == nullptr) != (S_F_dev == nullptr)) {
        set_error("obj and S_F_dev must be given together");
        return PYHEA_EINVAL;
    }
    if (obj) return check_objective(*g, obj);
    return PYHEA_OK;
}

// Scratch of pyhea_sro_eval_batch_noalloc: a fixed device array that every GPU
// the library runs on holds until the process ends.  In host code `scratch`
// names a host-side stand-in, never the device memory: the device address is
// taken once per device with hipGetSymbolAddress and only that address is
// passed to kernels.  Calls that overlap on one device share the array and
// race; each call overwrites what it reads (no part needs to start at zero).
constexpr size_t kNoAllocScratchBytes = size_t(16) << 20;
__device__ __align__(256) char scratch[kNoAllocScratchBytes];

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_addr[kMaxScratchDevices];

pyhea_status noalloc_scratch(void **addr) {
    int dev = -1;
    PYHEA_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxScratchDevices) {
        set_error("device index out of range for the fixed scratch table");
        return PYHEA_EDEVICE;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void *p = nullptr;
        PYHEA_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) {
            set_error("hipGetSymbolAddress returned no address for the fixed scratch array");
            return PYHEA_EDEVICE;
        }
        g_scratch_addr[dev] = p;
    }
    *addr = g_scratch_addr[dev];
    return PYHEA_OK;
}

}  // namespace

extern "C" {

pyhea_status pyhea_sro_eval_batch(const pyhea_lattice *lat, int64_t n_configs, const int8_t *species_dev,
                                  const pyhea_objective *obj, int32_t *counts_dev, double *S_F_dev,
                                  void *stream_) {
    Geometry g;
    pyhea_status s = check_eval_batch(lat, n_configs, species_dev, obj, counts_dev, S_F_dev, &g);
    if (s != PYHEA_OK) return s;
    if (n_configs == 0) return guard(PYHEA_OK);
    s = eval_batch(g, n_configs, species_dev, obj, counts_dev, S_F_dev, as_stream(stream_));
    return s == PYHEA_OK ? guard(s) : s;
}

pyhea_status pyhea_sro_eval_batch_noalloc(const pyhea_lattice *lat, int64_t n_configs,
                                          const int8_t *species_dev, const pyhea_objective *obj,
                                          int32_t *counts_dev, double *S_F_dev, void *stream_) {
    Geometry g;
    pyhea_status s = check_eval_batch(lat, n_configs, species_dev, obj, counts_dev, S_F_dev, &g);
    if (s != PYHEA_OK) return s;
    if (n_configs == 0) return guard(PYHEA_OK);
    const size_t need = eval_batch_scratch_bytes(g, n_configs);
    if (need > kNoAllocScratchBytes) {
        set_error("pyhea_sro_eval_batch_noalloc: " + std::to_string(n_configs) + " configurations need " +
                  std::to_string(need) + " bytes of scratch, more than the fixed " +
                  std::to_string(kNoAllocScratchBytes) + "-byte array; split the batch");
        return PYHEA_EINVAL;
    }
    void *addr = nullptr;
    s = noalloc_scratch(&addr);
    if (s != PYHEA_OK) return s;
    s = eval_batch(g, n_configs, species_dev, obj, counts_dev, S_F_dev, as_stream(stream_), addr);
    return s == PYHEA_OK ? guard(s) : s;
}

pyhea_status pyhea_map_sites(const pyhea_lattice *lat, const double *box_host, double max_disp, int64_t n_atoms,
                             const double *xyz_dev, const int8_t *types_dev, int8_t *species_dev,
                             int32_t *atom_of_site_dev, void *stream_) {
    Geometry g;
    std::string err;
    if (build_geometry(lat, &g, &err) != PYHEA_OK) {
        set_error(err);
        return PYHEA_EINVAL;
    }
    if (!box_host || !species_dev || (n_atoms > 0 && (!xyz_dev || !types_dev))) {
        set_error("box_host, species_dev, xyz_dev and types_dev must not be NULL");
        return PYHEA_EINVAL;
    }
    for (int ax = 0; ax < 3; ++ax)
        if (!std::isfinite(box_host[ax]) || box_host[ax] <= 0.0) {
            set_error("box edge lengths must be finite and > 0");
            return PYHEA_EINVAL;
        }
    if (!std::isfinite(max_disp) || max_disp < 0.0) {
        set_error("max_disp must be finite and >= 0");
        return PYHEA_EINVAL;
    }
    if (n_atoms != g.N) {
        set_error("n_atoms (" + std::to_string(n_atoms) + ") must equal the number of lattice sites (" +
                  std::to_string(g.N) + ")");
        return PYHEA_EINVAL;
    }
    if (g.N > INT32_MAX) {
        set_error("too many sites for 32-bit atom indices");
        return PYHEA_EINVAL;
    }
    hipStream_t stream = as_stream(stream_);
    SiteMapDesc md{};
    md.lattice = g.lattice;
    md.A = g.A;
    for (int ax = 0; ax < 3; ++ax) {
        md.L[ax] = g.L[ax];
        md.scale[ax] = 2.0 * g.L[ax] / box_host[ax];
    }
    md.M = g.M;
    md.N = g.N;
    md.max_disp2 = max_disp * max_disp;
    // device block: flags [4] | owner [N] (unless the caller's)
    AsyncBuffer buf;
    buf.stream = stream;
    const size_t own = atom_of_site_dev ? 0 : (size_t)g.N * 4;
    PYHEA_HIP(pool_alloc(&buf.ptr, 256 + own, stream));
    int32_t *flags = (int32_t *)buf.ptr;
    int32_t *owner = atom_of_site_dev ? atom_of_site_dev : (int32_t *)((char *)buf.ptr + 256);
    PYHEA_HIP(launch_map_sites(md, n_atoms, xyz_dev, types_dev, owner, flags, species_dev, stream));
    int32_t fh[4] = {0, 0, 0, 0};
    PYHEA_HIP(hipMemcpyAsync(fh, flags, sizeof(fh), hipMemcpyDeviceToHost, stream));
    PYHEA_HIP(hipStreamSynchronize(stream));
    if (fh[0]) {
        set_error("an atom lies farther than max_disp from every lattice site");
        return PYHEA_EINVAL;
    }
    if (fh[2]) {
        set_error("atom types must lie in [0, n_species)");
        return PYHEA_EINVAL;
    }
    if (fh[1] || fh[3]) {
        set_error("two atoms are nearest to one lattice site (another site is vacant)");
        return PYHEA_EINVAL;
    }
    return guard(PYHEA_OK);
}

pyhea_status pyhea_trial_eval(const pyhea_lattice *lat, const pyhea_objective *obj, const int8_t *species_dev,
                              int64_t n_pairs, const int32_t *pairs_dev, double *dS_dev, int32_t *dN_dev,
                              void *stream_) {
    Geometry g;
    std::string err;
    if (build_geometry(lat, &g, &err) != PYHEA_OK) {
        set_error(err);
        return PYHEA_EINVAL;
    }
    pyhea_status s = check_objective(g, obj);
    if (s != PYHEA_OK) return s;
    if (n_pairs < 0 || !species_dev || (n_pairs > 0 && (!pairs_dev || !dS_dev))) {
        set_error("n_pairs must be >= 0 and species/pairs/dS pointers non-NULL");
        return PYHEA_EINVAL;
    }
    hipStream_t stream = as_stream(stream_);
    const int E = g.S * g.M * g.M;
    AsyncBuffer buf;
    buf.stream = stream;
    PYHEA_HIP(pool_alloc(&buf.ptr, 256 + E * 4 + (E + kMaxShells) * 8 + 256, stream));
    int32_t *bad = (int32_t *)buf.ptr;
    int32_t *counts = (int32_t *)((char *)buf.ptr + 256);
    double *tdev = (double *)((char *)buf.ptr + 256 + ((E * 4 + 255) & ~255));
    EvalDesc ed;
    fill_eval_desc(g, &ed);
    PYHEA_HIP(launch_count_gather(ed, 1, species_dev, counts, bad, stream));
    std::vector<int32_t> c32(E);
    int32_t badh = 0;
    PYHEA_HIP(hipMemcpyAsync(c32.data(), counts, E * 4, hipMemcpyDeviceToHost, stream));
    PYHEA_HIP(hipMemcpyAsync(&badh, bad, 4, hipMemcpyDeviceToHost, stream));
    PYHEA_HIP(hipStreamSynchronize(stream));
    std::vector<int64_t> c64(c32.begin(), c32.end());
    int64_t n[kMaxSpecies];
    if (badh || !species_totals(g, c64.data(), n)) {
        set_error("species ids must lie in [0, n_species) and every species must occur");
        return PYHEA_EINVAL;
    }
    std::vector<double> tw(E + kMaxShells, 0.0);
    std::memcpy(tw.data(), obj->target, E * 8);
    std::memcpy(tw.data() + E, obj->weight, g.S * 8);
    PYHEA_HIP(hipMemcpyAsync(tdev, tw.data(), tw.size() * 8, hipMemcpyHostToDevice, stream));
    PYHEA_HIP(launch_trial_eval(ed, species_dev, counts, tdev, tdev + E, n_pairs, pairs_dev, dS_dev, dN_dev,
                                stream));
    PYHEA_HIP(hipStreamSynchronize(stream));
    return guard(PYHEA_OK);
}

static pyhea_status make_job(const pyhea_lattice *lat, const pyhea_objective *obj, const pyhea_mc_params *params,
                             ChainJob *job, const char *who) {
    std::string err;
    if (build_geometry(lat, &job->g, &err) != PYHEA_OK) {
        set_error(std::string(who) + err);
        return PYHEA_EINVAL;
    }
    pyhea_status s = check_objective(job->g, obj);
    if (s != PYHEA_OK) return s;
    s = check_params(params);
    if (s != PYHEA_OK) return s;
    job->params = *params;
    const int E = job->g.S * job->g.M * job->g.M;
    job->target.assign(obj->target, obj->target + E);
    job->weight.assign(obj->weight, obj->weight + job->g.S);
    return PYHEA_OK;
}

pyhea_status pyhea_mc_run(const pyhea_lattice *lat, const pyhea_objective *obj, const pyhea_mc_params *params,
                          int8_t *species_dev, uint32_t *log_dev, int64_t log_cap, pyhea_mc_stats *stats_host,
                          int64_t *counts_host, void *stream) {
    std::vector<ChainJob> jobs(1);
    pyhea_status s = make_job(lat, obj, params, &jobs[0], "");
    if (s != PYHEA_OK) return s;
    if (!species_dev || !stats_host || log_cap < 0) {
        set_error("species_dev and stats_host must not be NULL; log_cap >= 0");
        return PYHEA_EINVAL;
    }
    jobs[0].species_dev = species_dev;
    jobs[0].log_dev = log_dev;
    jobs[0].log_cap = log_cap;
    std::vector<std::vector<int64_t>> fc;
    s = run_chains(jobs, stats_host, &fc, as_stream(stream), forced_variant());
    if (s != PYHEA_OK) return s;
    if (counts_host) std::memcpy(counts_host, fc[0].data(), fc[0].size() * 8);
    return guard(PYHEA_OK);
}

pyhea_status pyhea_mc_batch(int32_t n_chains, const pyhea_lattice *lats, const pyhea_objective *objs,
                            const pyhea_mc_params *params, int8_t *species_dev, const int64_t *offsets_host,
                            uint32_t *log_dev, const int64_t *log_offsets_host, pyhea_mc_stats *stats_host,
                            void *stream) {
    if (n_chains < 0 || (n_chains > 0 && (!lats || !objs || !params || !species_dev || !offsets_host ||
                                          !stats_host))) {
        set_error("n_chains must be >= 0 and the descriptor arrays non-NULL");
        return PYHEA_EINVAL;
    }
    if (log_dev && !log_offsets_host) {
        set_error("log_offsets_host is required with log_dev");
        return PYHEA_EINVAL;
    }
    std::vector<ChainJob> jobs(n_chains);
    for (int c = 0; c < n_chains; ++c) {
        const std::string who = "chain " + std::to_string(c) + ": ";
        pyhea_status s = make_job(&lats[c], &objs[c], &params[c], &jobs[c], who.c_str());
        if (s != PYHEA_OK) return s;
        if (offsets_host[c + 1] - offsets_host[c] != jobs[c].g.N || offsets_host[c] < 0) {
            set_error(who + "offsets do not match the chain's site count");
            return PYHEA_EINVAL;
        }
        jobs[c].species_dev = species_dev + offsets_host[c];
        if (log_dev) {
            jobs[c].log_dev = log_dev + 4 * log_offsets_host[c];
            jobs[c].log_cap = log_offsets_host[c + 1] - log_offsets_host[c];
            if (jobs[c].log_cap < 0) {
                set_error(who + "log offsets must be non-decreasing");
                return PYHEA_EINVAL;
            }
        }
    }
    pyhea_status s = run_chains(jobs, stats_host, nullptr, as_stream(stream), forced_variant());
    return s == PYHEA_OK ? guard(s) : s;
}

pyhea_status pyhea_trial_eval_full(const pyhea_lattice *lat, const pyhea_objective *obj, const int8_t *species_dev,
                                   int64_t n_pairs, const int32_t *pairs_dev, double *dS_dev, void *stream_) {
    Geometry g;
    std::string err;
    if (build_geometry(lat, &g, &err) != PYHEA_OK) {
        set_error(err);
        return PYHEA_EINVAL;
    }
    pyhea_status s = check_objective(g, obj);
    if (s != PYHEA_OK) return s;
    if (n_pairs < 0 || !species_dev || (n_pairs > 0 && (!pairs_dev || !dS_dev))) {
        set_error("n_pairs must be >= 0 and species/pairs/dS pointers non-NULL");
        return PYHEA_EINVAL;
    }
    hipStream_t stream = as_stream(stream_);
    const int64_t N = g.N;
    const int E = g.S * g.M * g.M;
    // swapped copies in chunks of at most 256 MB
    const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(n_pairs, (int64_t(256) << 20) / N));
    const size_t o_cnt = ((size_t)chunk * N + 255) & ~size_t(255);
    const size_t o_sf = (o_cnt + (size_t)chunk * E * 4 + 255) & ~size_t(255);
    const size_t o_s0 = o_sf + (size_t)chunk * 16;
    const size_t o_bad = o_s0 + 16;
    AsyncBuffer buf;
    buf.stream = stream;
    PYHEA_HIP(pool_alloc(&buf.ptr, o_bad + 256, stream));
    char *base = (char *)buf.ptr;
    int8_t *copies = (int8_t *)base;
    int32_t *counts = (int32_t *)(base + o_cnt);
    double *SF = (double *)(base + o_sf);
    double *S0 = (double *)(base + o_s0);
    int32_t *bad = (int32_t *)(base + o_bad);
    PYHEA_HIP(launch_upload(SmallTable{}, 1, (double *)bad, stream));   // clears the flag word
    // S(before) from a full evaluation of the configuration itself
    s = pyhea_sro_eval_batch(lat, 1, species_dev, obj, counts, S0, stream);
    if (s != PYHEA_OK) return s;
    double s0h[2];
    PYHEA_HIP(hipMemcpyAsync(s0h, S0, 16, hipMemcpyDeviceToHost, stream));
    PYHEA_HIP(hipStreamSynchronize(stream));
    if (std::isnan(s0h[0])) {
        set_error("species ids must lie in [0, n_species) and every species must occur");
        return PYHEA_EINVAL;
    }
    for (int64_t c0 = 0; c0 < n_pairs; c0 += chunk) {
        const int nc = (int)std::min<int64_t>(chunk, n_pairs - c0);
        PYHEA_HIP(launch_swap_copies(species_dev, N, pairs_dev + 2 * c0, nc, copies, bad, stream));
        s = pyhea_sro_eval_batch(lat, nc, copies, obj, counts, SF, stream);
        if (s != PYHEA_OK) return s;
        PYHEA_HIP(launch_sub_objective(SF, S0, nc, dS_dev + c0, stream));
    }
    int32_t badh = 0;
    PYHEA_HIP(hipMemcpyAsync(&badh, bad, 4, hipMemcpyDeviceToHost, stream));
    PYHEA_HIP(hipStreamSynchronize(stream));
    if (badh) {
        set_error("site ids must lie in [0, N)");
        return PYHEA_EINVAL;
    }
    return guard(PYHEA_OK);
}

static pyhea_status random_desc(int64_t N, int32_t M, const int64_t *comp, uint64_t seed, uint32_t iteration,
                                uint32_t slot0, RandomConfigDesc *d) {
    if (N < 1 || N > (int64_t(1) << 30) || M < 1 || M > 8 || !comp) {
        set_error("N must be in [1, 2^30], M in [1, 8], composition non-NULL");
        return PYHEA_EINVAL;
    }
    std::memset(d, 0, sizeof(*d));
    d->seed = seed;
    d->iteration = iteration;
    d->slot0 = slot0;
    d->M = M;
    int64_t total = 0;
    for (int j = 0; j < M; ++j) {
        if (comp[j] < 0) {
            set_error("species counts must be >= 0");
            return PYHEA_EINVAL;
        }
        d->prefix[j] = (uint32_t)total;
        total += comp[j];
        if (total > N) break;
    }
    if (total != N) {
        set_error("species counts must add up to N");
        return PYHEA_EINVAL;
    }
    d->prefix[M] = (uint32_t)N;
    return PYHEA_OK;
}

pyhea_status pyhea_random_configs(int64_t N, int32_t M, const int64_t *composition_host, uint64_t seed,
                                  uint32_t iteration, uint32_t slot0, int32_t n_configs, int8_t *out_dev,
                                  void *stream) {
    RandomConfigDesc d;
    pyhea_status s = random_desc(N, M, composition_host, seed, iteration, slot0, &d);
    if (s != PYHEA_OK) return s;
    if (n_configs < 0 || (n_configs > 0 && !out_dev)) {
        set_error("n_configs must be >= 0 and out_dev non-NULL");
        return PYHEA_EINVAL;
    }
    PYHEA_HIP(launch_random_configs((uint32_t)N, d, n_configs, out_dev, as_stream(stream)));
    return guard(PYHEA_OK);
}

pyhea_status pyhea_global_search(const pyhea_lattice *lat, const pyhea_objective *obj,
                                 const int64_t *composition_host, const pyhea_global_params *params,
                                 int8_t *best_dev, double *history_host, pyhea_global_stats *stats_host,
                                 void *stream_) {
    if (!params || !best_dev || !stats_host || !obj) {
        set_error("params, obj, best_dev and stats_host must not be NULL");
        return PYHEA_EINVAL;
    }
    const pyhea_global_params &P = *params;
    if (P.n_solutions < 1 || P.iterations < 1 || P.n_refine < 1 || P.n_refine > P.n_solutions ||
        !(P.discard_frac >= 0.0 && P.discard_frac <= 1.0)) {
        set_error("need n_solutions >= 1, iterations >= 1, 1 <= n_refine <= n_solutions, 0 <= p_a <= 1");
        return PYHEA_EINVAL;
    }
    ChainJob proto;
    pyhea_status s = make_job(lat, obj, &P.local, &proto, "");
    if (s != PYHEA_OK) return s;
    const Geometry &g = proto.g;
    const int64_t N = g.N;
    if ((int64_t)P.n_solutions * P.iterations > (int64_t)UINT32_MAX) {
        set_error("n_solutions * iterations must fit the 32-bit chain id");
        return PYHEA_EINVAL;
    }
    RandomConfigDesc rd;
    s = random_desc(N, g.M, composition_host, P.local.seed, 0, 0, &rd);
    if (s != PYHEA_OK) return s;
    for (int j = 0; j < g.M; ++j)
        if (composition_host[j] < 1) {
            set_error("every species needs at least one site (Eq. 2 divides by its count)");
            return PYHEA_EINVAL;
        }
    const int n = P.n_solutions, T = P.n_refine;
    const int R = std::max(0, std::min(T / 2, T - (int)std::ceil(P.discard_frac * T)));
    hipStream_t stream = as_stream(stream_);
    const int E = g.S * g.M * g.M;
    // pool [n][N] | refine [T][N] | counts [n][E] int32 | S_F [n][2]
    const size_t o_ref = ((size_t)n * N + 255) & ~size_t(255);
    const size_t o_cnt = (o_ref + (size_t)T * N + 255) & ~size_t(255);
    const size_t o_sf = (o_cnt + (size_t)n * E * 4 + 255) & ~size_t(255);
    AsyncBuffer buf;
    buf.stream = stream;
    PYHEA_HIP(pool_alloc(&buf.ptr, o_sf + (size_t)n * 16, stream));
    int8_t *pool = (int8_t *)buf.ptr;
    int8_t *refine = pool + o_ref;
    int32_t *counts = (int32_t *)((char *)buf.ptr + o_cnt);
    double *SF = (double *)((char *)buf.ptr + o_sf);
    std::vector<double> sf(2 * (size_t)n);
    std::vector<pyhea_mc_stats> ms(T);
    pyhea_global_stats st{};
    st.S = st.F = std::numeric_limits<double>::infinity();
    int kept = 0;
    for (int t = 0; t < P.iterations; ++t) {
        // new random solutions in the slots without a seed
        rd.iteration = (uint32_t)t;
        rd.slot0 = (uint32_t)kept;
        PYHEA_HIP(launch_random_configs((uint32_t)N, rd, n - kept, pool + (int64_t)kept * N, stream));
        // fitness of every solution (Eq. 3)
        s = pyhea_sro_eval_batch(lat, n, pool, obj, counts, SF, stream);
        if (s != PYHEA_OK) return s;
        PYHEA_HIP(hipMemcpyAsync(sf.data(), SF, sf.size() * 8, hipMemcpyDeviceToHost, stream));
        PYHEA_HIP(hipStreamSynchronize(stream));
        st.evaluations += n;
        std::vector<int> order(n);
        for (int i = 0; i < n; ++i) order[i] = i;
        std::stable_sort(order.begin(), order.end(),
                         [&](int a, int b) { return sf[2 * a + 1] < sf[2 * b + 1]; });
        // local search of the n_refine best, in rank order
        std::vector<ChainJob> jobs(T, proto);
        for (int r = 0; r < T; ++r) {
            PYHEA_HIP(hipMemcpyAsync(refine + (int64_t)r * N, pool + (int64_t)order[r] * N, N,
                                     hipMemcpyDeviceToDevice, stream));
            jobs[r].species_dev = refine + (int64_t)r * N;
            jobs[r].params.chain_id = (uint32_t)(t * n + order[r]);
        }
        s = run_chains(jobs, ms.data(), nullptr, stream, forced_variant());
        if (s != PYHEA_OK) return s;
        std::vector<int> rank(T);
        for (int r = 0; r < T; ++r) {
            rank[r] = r;
            st.trials += ms[r].trials;
            st.commits += ms[r].commits;
        }
        std::stable_sort(rank.begin(), rank.end(), [&](int a, int b) { return ms[a].F < ms[b].F; });
        if (ms[rank[0]].F < st.F) {
            st.F = ms[rank[0]].F;
            st.S = ms[rank[0]].S;
            PYHEA_HIP(hipMemcpyAsync(best_dev, refine + (int64_t)rank[0] * N, N, hipMemcpyDeviceToDevice, stream));
        }
        if (history_host) history_host[t] = st.F;
        // the best R refined solutions seed the next iteration
        for (int i = 0; i < R; ++i)
            PYHEA_HIP(hipMemcpyAsync(pool + (int64_t)i * N, refine + (int64_t)rank[i] * N, N,
                                     hipMemcpyDeviceToDevice, stream));
        kept = R;
    }
    PYHEA_HIP(hipStreamSynchronize(stream));
    *stats_host = st;
    return guard(PYHEA_OK);
}

pyhea_status pyhea_philox4x32_10(const uint32_t *ctr_dev, uint64_t seed, int64_t n, uint32_t *out_dev,
                                 void *stream) {
    if (n < 0 || (n > 0 && (!ctr_dev || !out_dev))) {
        set_error("n must be >= 0 and pointers non-NULL");
        return PYHEA_EINVAL;
    }
    PYHEA_HIP(launch_philox(ctr_dev, seed, n, out_dev, as_stream(stream)));
    return guard(PYHEA_OK);
}

pyhea_status pyhea_tune_force_eval(int32_t kernel) {
    if (kernel < -1 || kernel > 4) {
        set_error("kernel must be -1 (automatic), 0 (gather), 1 (bit-sliced), 2 (bit-sliced, no z split), 3 "
                  "(bit-sliced, four workgroups per CU) or 4 (streaming)");
        return PYHEA_EINVAL;
    }
    set_forced_eval_kernel(kernel);
    return guard(PYHEA_OK);
}

pyhea_status pyhea_tune_force_stream(int32_t layers_per_group, int32_t threads) {
    if (layers_per_group < 0 || layers_per_group > 8 || (threads != 0 && threads != 256 && threads != 512)) {
        set_error("layers_per_group must be 0 (automatic) or 1..8 and threads 0 (automatic), 256 or 512");
        return PYHEA_EINVAL;
    }
    set_forced_stream_shape(layers_per_group, threads);
    return guard(PYHEA_OK);
}

pyhea_status pyhea_tune_measure(int32_t on) {
    if (on != 0 && on != 1) {
        set_error("on must be 0 or 1");
        return PYHEA_EINVAL;
    }
    set_measure_enabled(on != 0);
    return guard(PYHEA_OK);
}

pyhea_status pyhea_tune_graphs(int32_t on) {
    if (on != 0 && on != 1) {
        set_error("on must be 0 or 1");
        return PYHEA_EINVAL;
    }
    set_graphs_enabled(on != 0);
    return guard(PYHEA_OK);
}

pyhea_status pyhea_tune_force_lookahead(int32_t steps) {
    if (steps < 0 || steps > kMaxLookahead) {
        set_error("steps per pass must be 0 (automatic) or 1..8");
        return PYHEA_EINVAL;
    }
    set_forced_lookahead(steps);
    return guard(PYHEA_OK);
}

pyhea_status pyhea_tune_force(int32_t variant) {
    if (variant < -1 || variant >= kNumStoreVariants) {
        set_error("variant out of range");
        return PYHEA_EINVAL;
    }
    set_forced_variant(variant);
    return guard(PYHEA_OK);
}

}  // extern "C"
