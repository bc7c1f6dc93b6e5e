// batch.hip -- many Glasma events evolved together (cpic_batch_* in cpic.h).
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/cpic.h"
#include "internal.h"

struct cpic_batch {
    std::vector<cpic_ctx*> ev;
    hipStream_t st = nullptr;
    bool own_stream = false;
    std::string err;
};

static std::string g_batch_error = "no error";

static cpic_status bfail(cpic_batch* b, cpic_status code, const std::string& m)
{
    if (b) b->err = m; else g_batch_error = m;
    return code;
}

extern "C" cpic_status cpic_batch_create(int32_t n_events, const cpic_glasma_params* gp,
                                         const cpic_particle_params* pp, void* hip_stream, cpic_batch** out)
{
    if (!out || !gp || n_events <= 0) return bfail(nullptr, CPIC_E_INVALID, "cpic_batch_create: bad arguments");
    *out = nullptr;
    cpic_batch* b = new cpic_batch();
    if (hip_stream) {
        b->st = (hipStream_t)hip_stream;
    } else if (hipStreamCreateWithFlags(&b->st, hipStreamNonBlocking) == hipSuccess) {
        b->own_stream = true;
    } else {
        delete b;
        return bfail(nullptr, CPIC_E_HIP, "cpic_batch_create: stream");
    }
    for (int e = 0; e < n_events; e++) {
        cpic_ctx* c = nullptr;
        cpic_status s = cpic_create(gp + e, pp ? pp + e : nullptr, b->st, &c);
        if (s) {
            std::string m = "event " + std::to_string(e) + ": " + cpic_last_error(nullptr);
            cpic_batch_destroy(b);
            return bfail(nullptr, s, m);
        }
        b->ev.push_back(c);
    }
    *out = b;
    return CPIC_OK;
}

extern "C" cpic_status cpic_batch_init_mv(cpic_batch* b)
{
    if (!b) return bfail(nullptr, CPIC_E_INVALID, "cpic_batch_init_mv: NULL");
    for (size_t e = 0; e < b->ev.size(); e++) {
        cpic_status s = cpic_init_mv(b->ev[e]);
        if (s) return bfail(b, s, "event " + std::to_string(e) + ": " + cpic_last_error(b->ev[e]));
    }
    return CPIC_OK;
}

extern "C" cpic_status cpic_batch_run(cpic_batch* b)
{
    if (!b) return bfail(nullptr, CPIC_E_INVALID, "cpic_batch_run: NULL");
    for (size_t e = 0; e < b->ev.size(); e++) {
        cpic_status s = cpic_evolve(b->ev[e], 1e300);
        if (s) return bfail(b, s, "event " + std::to_string(e) + ": " + cpic_last_error(b->ev[e]));
    }
    return CPIC_OK;
}

extern "C" cpic_status cpic_batch_sync(cpic_batch* b)
{
    if (!b) return bfail(nullptr, CPIC_E_INVALID, "cpic_batch_sync: NULL");
    for (size_t e = 0; e < b->ev.size(); e++) {
        cpic_status s = cpic_sync(b->ev[e]);
        if (s) return bfail(b, s, "event " + std::to_string(e) + ": " + cpic_last_error(b->ev[e]));
    }
    return CPIC_OK;
}

extern "C" cpic_status cpic_batch_observables(cpic_batch* b, int32_t event, double* out, int32_t cap,
                                              int32_t* n_samples)
{
    if (!b || event < 0 || event >= (int)b->ev.size()) return bfail(b, CPIC_E_INVALID, "cpic_batch_observables: bad event");
    int32_t ns = 0;
    cpic_num_samples(b->ev[event], &ns);
    if (n_samples) *n_samples = ns;
    cpic_status s = cpic_observables_full(b->ev[event], out, cap);
    if (s) return bfail(b, s, cpic_last_error(b->ev[event]));
    return CPIC_OK;
}

extern "C" cpic_status cpic_batch_get_state(cpic_batch* b, int32_t event, int32_t which, void* dst, size_t bytes)
{
    if (!b || event < 0 || event >= (int)b->ev.size()) return bfail(b, CPIC_E_INVALID, "cpic_batch_get_state: bad event");
    cpic_status s = cpic_get_state(b->ev[event], which, dst, bytes);
    if (s) return bfail(b, s, cpic_last_error(b->ev[event]));
    return CPIC_OK;
}

extern "C" const char* cpic_batch_last_error(const cpic_batch* b) { return b ? b->err.c_str() : g_batch_error.c_str(); }

extern "C" void cpic_batch_destroy(cpic_batch* b)
{
    if (!b) return;
    for (auto c : b->ev) cpic_destroy(c);
    if (b->own_stream) hipStreamDestroy(b->st);
    delete b;
}
