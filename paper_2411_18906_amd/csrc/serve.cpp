// Serving API (continuous batching of MC jobs).
#include "pyhea.h"
#include "runtime.h"

using namespace pyhea;

extern "C" {

pyhea_status pyhea_serve_open(int64_t, int32_t, int32_t, void **) {
    set_error("serving is not built yet");
    return PYHEA_ENOSYS;
}
pyhea_status pyhea_serve_submit(void *, uint64_t, const pyhea_lattice *, const pyhea_objective *,
                                const pyhea_mc_params *, const int8_t *) {
    return PYHEA_ENOSYS;
}
pyhea_status pyhea_serve_poll(void *, uint64_t, int8_t *, pyhea_mc_stats *, int64_t *, int32_t) {
    return PYHEA_ENOSYS;
}
pyhea_status pyhea_serve_cancel(void *, uint64_t) { return PYHEA_ENOSYS; }
pyhea_status pyhea_serve_counters(void *, int64_t *) { return PYHEA_ENOSYS; }
pyhea_status pyhea_serve_close(void *) { return PYHEA_ENOSYS; }

}
