// batch.hip -- many Glasma events evolved together (cpic_batch_* in cpic.h).
//
// Every event keeps its own context (buffers, step counter, samples); the
// batch adds a device table of event descriptors and, for each set of still
// active events, a plan: the active list and the prefix sums of their field
// tiles and push blocks.  One step of the whole batch is three launches --
// batched field update, batched push, batched step end -- whose workgroups
// find their (event, tile) item by binary search in the prefix table.
// Runs of steps between particle reorderings are replayed from HIP graphs
// captured per plan; each event reads its step number, and so its buffer
// parity, kick/formation/recording decisions, from its own device counter.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <map>
#include <string>
#include <vector>

#include "../../include/cpic.h"
#include "ctx.h"
#include "internal.h"

using namespace cpic;

namespace {

constexpr int kBatchGraphSteps = 16;

// Consecutive active events act[first .. first + count) launched together.
struct Group {
    int first = 0, count = 0;
    int total_tiles = 0, total_blocks = 0;
    size_t tiles_off = 0, blocks_off = 0;  // offsets (ints) of the prefix tables in d_idx
};

struct Plan {
    std::vector<int> act;
    std::vector<Group> groups;
    int* d_idx = nullptr;  // act[nact], then per group tile_start[count + 1], blk_start[count + 1]
    hipGraphExec_t graph = nullptr;
};

}  // namespace

struct cpic_batch {
    std::vector<cpic_ctx*> ev;
    hipStream_t st = nullptr;
    bool own_stream = false;
    int prec = CPIC_FP64;
    LaunchCfg cfg{};
    // four wavefronts per particle group: the push is bound by the latency of
    // its gathers, and splitting the field contractions over four waves
    // shortens each wave's chain of dependent loads (measured fastest from
    // 5e4 to 3.5e6 particles per launch)
    int tpp = 4;
    size_t group_bytes = 0;  // working-set budget of a launch group; 0: all active events in one launch
    EventDesc* d_desc = nullptr;
    std::vector<EventDesc> desc;  // host copy (kept alive for the asynchronous upload)
    std::map<std::vector<int>, Plan> plans;
    std::string err;
};

static std::string g_batch_error = "no error";

static cpic_status bfail(cpic_batch* b, cpic_status code, const std::string& m)
{
    if (b) b->err = m; else g_batch_error = m;
    return code;
}
static cpic_status bhip(cpic_batch* b, hipError_t e, const char* where)
{
    return bfail(b, CPIC_E_HIP, std::string(where) + ": " + hipGetErrorString(e));
}
#define BHIP(b, x, where)                                   \
    do {                                                    \
        hipError_t e_ = (x);                                \
        if (e_ != hipSuccess) return bhip(b, e_, where);    \
    } while (0)

static void drop_plans(cpic_batch* b)
{
    for (auto& kv : b->plans) {
        if (kv.second.graph) hipGraphExecDestroy(kv.second.graph);
        hipFree(kv.second.d_idx);
    }
    b->plans.clear();
}

// Descriptors are rebuilt when a run starts: the buffer parity relation
// flip = cur ^ (n & 1) is invariant under steps, so one table serves every step.
static cpic_status upload_desc(cpic_batch* b)
{
    const size_t ne = b->ev.size();
    b->desc.assign(ne, EventDesc{});
    for (size_t e = 0; e < ne; e++) {
        const cpic_ctx* c = b->ev[e];
        EventDesc& d = b->desc[e];
        d.f[0] = c->fbuf[0];
        d.f[1] = c->fbuf[1];
        d.flip = c->cur ^ (c->n & 1);
        d.pr = c->pr;
        d.cell = c->pcell;
        d.N = c->N;
        d.pa = push_args(c, b->tpp);
        d.d_step = c->d_step;
        d.d_err = c->d_err;
        d.partials = c->partials;
        d.obs = c->obs;
    }
    if (!b->d_desc) BHIP(b, hipMalloc(&b->d_desc, sizeof(EventDesc) * ne), "descriptor table");
    BHIP(b, hipMemcpyAsync(b->d_desc, b->desc.data(), sizeof(EventDesc) * ne, hipMemcpyHostToDevice, b->st),
         "descriptor table");
    BHIP(b, hipStreamSynchronize(b->st), "descriptor table");
    return CPIC_OK;
}

static int field_tiles_host(int N, const LaunchCfg& cfg)
{
    return ((N + cfg.bx - 1) / cfg.bx) * ((N + cfg.by - 1) / cfg.by);
}

static size_t working_set(const cpic_ctx* c)
{
    return 2 * (size_t)kRealsPerSite * c->V * c->tsz + (size_t)c->np * (kPartReals * c->tsz + 2 * sizeof(int));
}

// split the active list into launch groups of at most group_bytes working set
static std::vector<std::pair<int, int>> group_ranges(const cpic_batch* b, const std::vector<int>& act)
{
    std::vector<std::pair<int, int>> r;
    size_t acc = 0;
    for (int k = 0; k < (int)act.size(); k++) {
        const size_t w = working_set(b->ev[act[k]]);
        if (r.empty() || (b->group_bytes && acc + w > b->group_bytes)) {
            r.push_back({k, 0});
            acc = 0;
        }
        r.back().second++;
        acc += w;
    }
    return r;
}

static cpic_status get_plan(cpic_batch* b, const std::vector<int>& act, Plan** out)
{
    auto it = b->plans.find(act);
    if (it != b->plans.end()) {
        *out = &it->second;
        return CPIC_OK;
    }
    Plan p;
    p.act = act;
    std::vector<int> idx(act.begin(), act.end());
    for (const auto& gr : group_ranges(b, act)) {
        Group g;
        g.first = gr.first;
        g.count = gr.second;
        g.tiles_off = idx.size();
        idx.push_back(0);
        for (int k = 0; k < g.count; k++)
            idx.push_back(idx.back() + field_tiles_host(b->ev[act[g.first + k]]->N, b->cfg));
        g.total_tiles = idx.back();
        g.blocks_off = idx.size();
        idx.push_back(0);
        for (int k = 0; k < g.count; k++) {
            const cpic_ctx* c = b->ev[act[g.first + k]];
            idx.push_back(idx.back() + (c->np > 0 ? push_blocks((int)c->np, b->tpp) : 0));
        }
        g.total_blocks = idx.back();
        p.groups.push_back(g);
    }
    BHIP(b, hipMalloc(&p.d_idx, sizeof(int) * idx.size()), "plan");
    BHIP(b, hipMemcpy(p.d_idx, idx.data(), sizeof(int) * idx.size(), hipMemcpyHostToDevice), "plan");
    auto ins = b->plans.emplace(act, p);
    *out = &ins.first->second;
    return CPIC_OK;
}

// one step of every active event: per group the field update, then the push
// while the group's fields are cache-resident; then every event's step end
template <typename T> static cpic_status launch_batch_step(cpic_batch* b, const Plan& p)
{
    for (const Group& g : p.groups) {
        const int* act = p.d_idx + g.first;
        BHIP(b, launch_batch_field<T>(b->d_desc, act, p.d_idx + g.tiles_off, g.count, g.total_tiles, b->cfg, b->st),
             "batch field");
        BHIP(b, launch_batch_push<T>(b->d_desc, act, p.d_idx + g.blocks_off, g.count, g.total_blocks, b->tpp, b->st),
             "batch push");
    }
    BHIP(b, launch_batch_step_end(b->d_desc, p.d_idx, (int)p.act.size(), b->st), "batch step end");
    return CPIC_OK;
}
static cpic_status batch_step(cpic_batch* b, const Plan& p)
{
    return b->prec == CPIC_FP64 ? launch_batch_step<double>(b, p) : launch_batch_step<float>(b, p);
}

static cpic_status capture(cpic_batch* b, Plan& p)
{
    hipGraph_t g = nullptr;
    BHIP(b, hipStreamBeginCapture(b->st, hipStreamCaptureModeThreadLocal), "capture");
    cpic_status s = CPIC_OK;
    for (int j = 0; j < kBatchGraphSteps && s == CPIC_OK; j++) s = batch_step(b, p);
    hipError_t e = hipStreamEndCapture(b->st, &g);
    if (s) {
        if (g) hipGraphDestroy(g);
        return s;
    }
    if (e != hipSuccess) return bhip(b, e, "end capture");
    e = hipGraphInstantiate(&p.graph, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e != hipSuccess) return bhip(b, e, "graph instantiate");
    return CPIC_OK;
}

static void advance(cpic_batch* b, const std::vector<int>& act, int k)
{
    for (int e : act) host_advance(b->ev[e], k);
}

extern "C" cpic_status cpic_batch_create(int32_t n_events, const cpic_glasma_params* gp,
                                         const cpic_particle_params* pp, void* hip_stream, cpic_batch** out)
{
    if (!out || !gp || n_events <= 0) return bfail(nullptr, CPIC_E_INVALID, "cpic_batch_create: bad arguments");
    *out = nullptr;
    for (int e = 1; e < n_events; e++)
        if (gp[e].precision != gp[0].precision)
            return bfail(nullptr, CPIC_E_INVALID, "cpic_batch_create: all events must share one precision");
    cpic_batch* b = new cpic_batch();
    b->prec = gp[0].precision;
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
    // FP32 site kernel: 64 x 4 tiles; FP64: 128 x 1 (cpic_batch_tune refines both)
    if (b->prec == CPIC_FP64) { b->cfg.bx = 128; b->cfg.by = 1; }
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

// Advance every active event by up to max_steps batch steps (all when
// max_steps < 0).  Segments end where an event reaches n_max or a particle
// reordering point; inside a segment whole graphs are replayed and the rest
// is launched step by step.
static cpic_status run_steps(cpic_batch* b, int64_t max_steps)
{
    for (size_t e = 0; e < b->ev.size(); e++)
        if (!b->ev[e]->initialised)
            return bfail(b, CPIC_E_INVALID, "cpic_batch_run: event " + std::to_string(e) + " has no state");
    cpic_status s = upload_desc(b);
    if (s) return s;
    int64_t budget = max_steps < 0 ? (int64_t)1 << 40 : max_steps;
    while (budget > 0) {
        std::vector<int> act;
        for (size_t e = 0; e < b->ev.size(); e++)
            if (b->ev[e]->n < b->ev[e]->sc.n_max) act.push_back((int)e);
        if (act.empty()) break;
        int64_t len = budget;
        for (int e : act) {
            cpic_ctx* c = b->ev[e];
            s = maybe_sort(c);
            if (s) return bfail(b, s, "event " + std::to_string(e) + ": " + c->err);
            len = std::min<int64_t>(len, c->sc.n_max - c->n);
            len = std::min<int64_t>(len, next_sort_point(c, c->n) - c->n);
        }
        Plan* p = nullptr;
        s = get_plan(b, act, &p);
        if (s) return s;
        int64_t left = len;
        if (left >= kBatchGraphSteps && !p->graph) {
            s = capture(b, *p);
            if (s) return s;
        }
        while (left >= kBatchGraphSteps) {
            BHIP(b, hipGraphLaunch(p->graph, b->st), "graph launch");
            advance(b, act, kBatchGraphSteps);
            left -= kBatchGraphSteps;
        }
        for (; left > 0; left--) {
            s = batch_step(b, *p);
            if (s) return s;
            advance(b, act, 1);
        }
        budget -= len;
    }
    return CPIC_OK;
}

extern "C" cpic_status cpic_batch_run(cpic_batch* b)
{
    if (!b) return bfail(nullptr, CPIC_E_INVALID, "cpic_batch_run: NULL");
    return run_steps(b, -1);
}

extern "C" cpic_status cpic_batch_step(cpic_batch* b, int32_t k)
{
    if (!b) return bfail(nullptr, CPIC_E_INVALID, "cpic_batch_step: NULL");
    if (k < 0) return bfail(b, CPIC_E_INVALID, "cpic_batch_step: negative step count");
    return run_steps(b, k);
}

extern "C" cpic_status cpic_batch_sync(cpic_batch* b)
{
    if (!b) return bfail(nullptr, CPIC_E_INVALID, "cpic_batch_sync: NULL");
    BHIP(b, hipStreamSynchronize(b->st), "cpic_batch_sync");
    for (size_t e = 0; e < b->ev.size(); e++) {
        cpic_status s = cpic_sync(b->ev[e]);
        if (s) return bfail(b, s, "event " + std::to_string(e) + ": " + cpic_last_error(b->ev[e]));
    }
    return CPIC_OK;
}

// Field-tile tuner: the batched field launch only reads the current buffers
// and writes the other ones, which the next step overwrites anyway, so it can
// be repeated without changing the state.
template <typename T> static cpic_status tune_batch(cpic_batch* b, int reps, std::string& rep)
{
    std::vector<int> act;
    for (size_t e = 0; e < b->ev.size(); e++)
        if (b->ev[e]->n < b->ev[e]->sc.n_max) act.push_back((int)e);
    if (act.empty()) return CPIC_OK;
    cpic_status s = upload_desc(b);
    if (s) return s;
    static const int shapes[][2] = {{64, 1}, {128, 1}, {256, 1}, {32, 2}, {64, 2}, {128, 2},
                                    {16, 4}, {32, 4}, {64, 4}, {32, 8}, {16, 16}};
    hipEvent_t e0, e1;
    BHIP(b, hipEventCreate(&e0), "tune");
    BHIP(b, hipEventCreate(&e1), "tune");
    const LaunchCfg keep = b->cfg;
    LaunchCfg best = keep;
    float best_ms = 1e30f;
    std::vector<int> idx;
    int* d_idx = nullptr;
    BHIP(b, hipMalloc(&d_idx, sizeof(int) * (3 * act.size() + 2)), "tune");
    char line[160];
    for (const auto& sh : shapes)
        for (int remap = 0; remap < 2; remap++) {
            LaunchCfg cfg{};
            cfg.bx = sh[0];
            cfg.by = sh[1];
            cfg.xcd_remap = remap;
            const int na = (int)act.size();
            idx.assign(3 * (size_t)na + 2, 0);
            int* tiles = idx.data() + na;
            for (int k = 0; k < na; k++) {
                idx[k] = act[k];
                tiles[k + 1] = tiles[k] + field_tiles_host(b->ev[act[k]]->N, cfg);
            }
            hipError_t e = hipMemcpy(d_idx, idx.data(), sizeof(int) * idx.size(), hipMemcpyHostToDevice);
            for (int r = 0; r < 2 && e == hipSuccess; r++)  // warm-up
                e = launch_batch_field<T>(b->d_desc, d_idx, d_idx + na, na, tiles[na], cfg, b->st);
            if (e == hipSuccess) e = hipEventRecord(e0, b->st);
            for (int r = 0; r < reps && e == hipSuccess; r++)
                e = launch_batch_field<T>(b->d_desc, d_idx, d_idx + na, na, tiles[na], cfg, b->st);
            if (e == hipSuccess) e = hipEventRecord(e1, b->st);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) {
                hipFree(d_idx);
                hipEventDestroy(e0);
                hipEventDestroy(e1);
                return bhip(b, e, "tune");
            }
            ms /= reps;
            std::snprintf(line, sizeof line, "batch field %3dx%-3d remap %d : %9.2f us\n", cfg.bx, cfg.by, remap,
                          ms * 1e3);
            rep += line;
            if (ms < best_ms) {
                best_ms = ms;
                best = cfg;
            }
        }
    hipFree(d_idx);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    std::snprintf(line, sizeof line, "chosen: %dx%d remap %d (%.2f us)\n", best.bx, best.by, best.xcd_remap,
                  best_ms * 1e3);
    rep += line;
    if (best.bx != keep.bx || best.by != keep.by || best.xcd_remap != keep.xcd_remap) {
        b->cfg = best;
        drop_plans(b);  // tile prefix tables and graphs depend on the tile shape
    }
    return CPIC_OK;
}

extern "C" cpic_status cpic_batch_tune(cpic_batch* b, int32_t reps, char* report, size_t cap)
{
    if (!b) return bfail(nullptr, CPIC_E_INVALID, "cpic_batch_tune: NULL");
    if (reps < 1) return bfail(b, CPIC_E_INVALID, "cpic_batch_tune: reps must be positive");
    std::string rep;
    cpic_status s = b->prec == CPIC_FP64 ? tune_batch<double>(b, reps, rep) : tune_batch<float>(b, reps, rep);
    if (s) return s;
    if (report && cap) {
        const size_t n = std::min(cap - 1, rep.size());
        std::copy(rep.begin(), rep.begin() + n, report);
        report[n] = 0;
    }
    return CPIC_OK;
}

extern "C" cpic_status cpic_batch_set_launch(cpic_batch* b, int32_t bx, int32_t by, int32_t xcd_remap, int32_t tpp)
{
    if (!b) return bfail(nullptr, CPIC_E_INVALID, "cpic_batch_set_launch: NULL");
    if (bx < 1 || by < 1 || bx * by > 256 || (bx * by) % 64 != 0 || (tpp != 1 && tpp != 2 && tpp != 4))
        return bfail(b, CPIC_E_INVALID, "cpic_batch_set_launch: bx*by must be 64, 128, 192 or 256; tpp 1, 2 or 4");
    b->cfg.bx = bx;
    b->cfg.by = by;
    b->cfg.xcd_remap = xcd_remap ? 1 : 0;
    b->tpp = tpp;
    drop_plans(b);
    return CPIC_OK;
}

extern "C" cpic_status cpic_batch_set_group_bytes(cpic_batch* b, int64_t bytes)
{
    if (!b) return bfail(nullptr, CPIC_E_INVALID, "cpic_batch_set_group_bytes: NULL");
    if (bytes < 0) return bfail(b, CPIC_E_INVALID, "cpic_batch_set_group_bytes: negative budget");
    b->group_bytes = (size_t)bytes;
    drop_plans(b);
    return CPIC_OK;
}

extern "C" cpic_status cpic_batch_get_launch(const cpic_batch* b, int32_t out[4])
{
    if (!b || !out) return CPIC_E_INVALID;
    out[0] = b->cfg.bx;
    out[1] = b->cfg.by;
    out[2] = b->cfg.xcd_remap;
    out[3] = b->tpp;
    return CPIC_OK;
}

extern "C" cpic_status cpic_batch_num_events(const cpic_batch* b, int32_t* n)
{
    if (!b || !n) return CPIC_E_INVALID;
    *n = (int32_t)b->ev.size();
    return CPIC_OK;
}

extern "C" cpic_status cpic_batch_current_step(const cpic_batch* b, int32_t event, int64_t* n)
{
    if (!b || !n || event < 0 || event >= (int)b->ev.size()) return CPIC_E_INVALID;
    *n = b->ev[event]->n;
    return CPIC_OK;
}

extern "C" cpic_status cpic_batch_observables(cpic_batch* b, int32_t event, double* out, int32_t cap,
                                              int32_t* n_samples)
{
    if (!b || event < 0 || event >= (int)b->ev.size())
        return bfail(b, CPIC_E_INVALID, "cpic_batch_observables: bad event");
    int32_t ns = 0;
    cpic_num_samples(b->ev[event], &ns);
    if (n_samples) *n_samples = ns;
    cpic_status s = cpic_observables_full(b->ev[event], out, cap);
    if (s) return bfail(b, s, cpic_last_error(b->ev[event]));
    return CPIC_OK;
}

extern "C" cpic_status cpic_batch_get_state(cpic_batch* b, int32_t event, int32_t which, void* dst, size_t bytes)
{
    if (!b || event < 0 || event >= (int)b->ev.size())
        return bfail(b, CPIC_E_INVALID, "cpic_batch_get_state: bad event");
    cpic_status s = cpic_get_state(b->ev[event], which, dst, bytes);
    if (s) return bfail(b, s, cpic_last_error(b->ev[event]));
    return CPIC_OK;
}

extern "C" const char* cpic_batch_last_error(const cpic_batch* b) { return b ? b->err.c_str() : g_batch_error.c_str(); }

extern "C" void cpic_batch_destroy(cpic_batch* b)
{
    if (!b) return;
    if (b->st) hipStreamSynchronize(b->st);
    drop_plans(b);
    hipFree(b->d_desc);
    for (auto c : b->ev) cpic_destroy(c);
    if (b->own_stream) hipStreamDestroy(b->st);
    delete b;
}
