// batch.hip -- many Glasma events evolved together (cpic_batch_* in cpic.h).
//
// Every event keeps its own context (buffers, step counter, samples); the
// batch adds a device table of event descriptors.  Events are split into
// launch groups whose working set fits the last-level cache; the groups are
// dealt to one or two launch lanes (streams), and each lane runs its groups
// one after the other, each to the end of its events.  For every set of
// still active events of a group there is a plan: the active list and the
// work maps (event, tile) and (event, particle block), one entry per
// workgroup.  One step of a group is two launches: the batched field update
// and the batched push, which also advances the events' step counters.  Runs
// of steps between particle reorderings are replayed from HIP graphs captured
// per plan; each event reads its step number, and so its buffer parity and
// its kick/formation/recording decisions, from its own device counter.
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
// Events are run in groups whose working set (both field buffer sets and the
// particle records) stays within about this much, so that from one step to
// the next (and from a group's field update to its push) the data of the
// groups the lanes run side by side is served from the 256 MB last-level
// cache (96 MiB measured best of 64, 96 and 128 with two lanes).
constexpr size_t kDefaultGroupBytes = (size_t)96 << 20;
constexpr int kMaxLanes = 4, kDefaultLanes = 2;

struct Plan {
    std::vector<int> act;          // active events (descriptor indices)
    int* d_act = nullptr;          // [nact]
    int2* d_tiles = nullptr;       // (event, tile) per field workgroup
    int2* d_blocks = nullptr;      // (event, particle block) per push workgroup
    std::vector<int2> tiles, blocks;  // host copies of the work maps (sources of their uploads)
    int total_tiles = 0, total_blocks = 0;
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
    size_t group_bytes = kDefaultGroupBytes;  // working-set budget of a launch group; 0: one group
    // Launch lanes: the groups are dealt to `lanes` streams that run
    // concurrently, so that groups of small events (whose launches leave most
    // of the chip idle) run beside groups of large ones.
    int lanes = kDefaultLanes;
    hipStream_t lane_st[kMaxLanes] = {};      // lane 0 is the batch stream; the others the library's own
    hipEvent_t ev_fork = nullptr, ev_join[kMaxLanes] = {};
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
        if (kv.second.graph) (void)hipGraphExecDestroy(kv.second.graph);
        (void)hipFree(kv.second.d_act);
        (void)hipFree(kv.second.d_tiles);
        (void)hipFree(kv.second.d_blocks);
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
        d.gpl = c->gpl;
        d.cell = c->pcell;
        d.N = c->N;
        d.pa = push_args(c, b->tpp);
        d.d_step = c->d_step;
        d.d_err = c->d_err;
        d.partials = c->partials;
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
    return (2 * (size_t)kRealsPerSite + (c->gpl ? kPlaqReals : 0)) * c->V * c->tsz +
           (size_t)c->np * (kPartReals * c->tsz + 2 * sizeof(int));
}

// Launch groups: events by decreasing working set, packed greedily up to
// group_bytes (an event larger than the budget forms a group of its own);
// group_bytes = 0 puts every event in one group.
static std::vector<std::vector<int>> launch_groups(const cpic_batch* b)
{
    std::vector<int> order(b->ev.size());
    for (size_t e = 0; e < order.size(); e++) order[e] = (int)e;
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return working_set(b->ev[x]) > working_set(b->ev[y]); });
    std::vector<std::vector<int>> groups;
    size_t acc = 0;
    for (int e : order) {
        const size_t w = working_set(b->ev[e]);
        if (groups.empty() || (b->group_bytes && acc + w > b->group_bytes)) {
            groups.emplace_back();
            acc = 0;
        }
        groups.back().push_back(e);
        acc += w;
    }
    for (auto& g : groups) std::sort(g.begin(), g.end());
    return groups;
}

static cpic_status get_plan(cpic_batch* b, const std::vector<int>& act, Plan** out, hipStream_t st)
{
    auto it = b->plans.find(act);
    if (it != b->plans.end()) {
        *out = &it->second;
        return CPIC_OK;
    }
    Plan p;
    p.act = act;
    for (int e : act) {
        const cpic_ctx* c = b->ev[e];
        // an event without particles keeps one push workgroup, which advances its step counter
        const int nt = field_tiles_host(c->N, b->cfg), nb = c->np > 0 ? push_blocks((int)c->np, b->tpp) : 1;
        for (int k = 0; k < nt; k++) p.tiles.push_back(make_int2(e, k));
        for (int k = 0; k < nb; k++) p.blocks.push_back(make_int2(e, k));
    }
    p.total_tiles = (int)p.tiles.size();
    p.total_blocks = (int)p.blocks.size();
    hipError_t e = hipMalloc(&p.d_act, sizeof(int) * act.size());
    if (e == hipSuccess) e = hipMalloc(&p.d_tiles, sizeof(int2) * std::max<size_t>(p.tiles.size(), 1));
    if (e == hipSuccess) e = hipMalloc(&p.d_blocks, sizeof(int2) * std::max<size_t>(p.blocks.size(), 1));
    if (e != hipSuccess) {
        (void)hipFree(p.d_act);
        (void)hipFree(p.d_tiles);
        (void)hipFree(p.d_blocks);
        return bhip(b, e, "plan");
    }
    auto ins = b->plans.emplace(act, std::move(p));
    Plan& q = ins.first->second;
    // uploaded in stream order from the plan's own host copies, so that
    // making a plan does not wait for the work already queued
    BHIP(b, hipMemcpyAsync(q.d_act, q.act.data(), sizeof(int) * q.act.size(), hipMemcpyHostToDevice, st), "plan");
    BHIP(b, hipMemcpyAsync(q.d_tiles, q.tiles.data(), sizeof(int2) * q.tiles.size(), hipMemcpyHostToDevice, st),
         "plan");
    if (!q.blocks.empty())
        BHIP(b, hipMemcpyAsync(q.d_blocks, q.blocks.data(), sizeof(int2) * q.blocks.size(), hipMemcpyHostToDevice, st),
             "plan");
    *out = &q;
    return CPIC_OK;
}

// one step of every active event of a plan (the push also advances the step counters)
template <typename T> static cpic_status launch_batch_step(cpic_batch* b, const Plan& p, hipStream_t st)
{
    BHIP(b, launch_batch_field<T>(b->d_desc, p.d_tiles, p.total_tiles, b->cfg, st), "batch field");
    BHIP(b, launch_batch_push<T>(b->d_desc, p.d_blocks, p.total_blocks, b->tpp, st), "batch push");
    return CPIC_OK;
}
static cpic_status batch_step(cpic_batch* b, const Plan& p, hipStream_t st)
{
    return b->prec == CPIC_FP64 ? launch_batch_step<double>(b, p, st) : launch_batch_step<float>(b, p, st);
}

static cpic_status capture(cpic_batch* b, Plan& p, hipStream_t st)
{
    hipGraph_t g = nullptr;
    BHIP(b, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal), "capture");
    cpic_status s = CPIC_OK;
    for (int j = 0; j < kBatchGraphSteps && s == CPIC_OK; j++) s = batch_step(b, p, st);
    hipError_t e = hipStreamEndCapture(st, &g);
    if (s) {
        if (g) (void)hipGraphDestroy(g);
        return s;
    }
    if (e != hipSuccess) return bhip(b, e, "end capture");
    e = hipGraphInstantiate(&p.graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
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
    for (int e = 0; e < n_events; e++)
        if (gp[e].n_colors == 2)
            return bfail(nullptr, CPIC_E_INVALID, "cpic_batch_create: batches hold SU(3) events only");
    for (int e = 0; pp && e < n_events; e++)
        if (pp[e].n > 0 && pp[e].color_update != CPIC_COLOR_ROTATE)
            return bfail(nullptr, CPIC_E_INVALID,
                         "cpic_batch_create: the colour update by matrix logarithm runs on single events only");
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
        // the batch launches its own kernels over all events: the events'
        // records keep the gather push's order
        if (c->cfg.split == 4) c->cfg.split = 3;
        b->ev.push_back(c);
    }
    // compressed-link LDS tiles of 64 x 4 sites (cpic_batch_tune picks among the shapes)
    b->cfg.split = 3;
    b->cfg.bx = 64;
    b->cfg.by = 4;
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

// Estimated work of one step of an event, in site-updates (a particle push
// costs about as much as two).
static double step_cost(const cpic_ctx* c) { return (double)c->V + 2.0 * (double)c->np; }

// A launch lane: its stream and the launch groups it runs one after the other.
struct Lane {
    hipStream_t st = nullptr;
    std::vector<std::vector<int>> groups;
    size_t gi = 0;        // current group
    int64_t budget = 0;   // steps the current group may still take
    double queued = 0;    // estimated work enqueued so far
    bool done() const { return gi >= groups.size(); }
};

// One segment of a lane's current group: its active events advance to the
// next particle reordering or to the end of an event, whole graphs replayed
// and the rest launched step by step.  A group that has finished (or used
// its step budget) hands over to the lane's next group.
static cpic_status lane_segment(cpic_batch* b, Lane& L, int64_t max_steps)
{
    std::vector<int> act;
    if (L.budget > 0)
        for (int e : L.groups[L.gi])
            if (b->ev[e]->n < b->ev[e]->sc.n_max) act.push_back(e);
    if (act.empty()) {
        L.gi++;
        L.budget = max_steps < 0 ? (int64_t)1 << 40 : max_steps;
        return CPIC_OK;
    }
    int64_t len = L.budget;
    double cost = 0;
    for (int e : act) {
        cpic_ctx* c = b->ev[e];
        cpic_status s = watch_prepare(c);
        if (s) return bfail(b, s, "event " + std::to_string(e) + ": " + c->err);
        s = maybe_sort(c);
        if (s) return bfail(b, s, "event " + std::to_string(e) + ": " + c->err);
        len = std::min<int64_t>(len, c->sc.n_max - c->n);
        len = std::min<int64_t>(len, next_sort_point(c, c->n) - c->n);
        cost += step_cost(c);
    }
    Plan* p = nullptr;
    cpic_status s = get_plan(b, act, &p, L.st);
    if (s) return s;
    int64_t left = len;
    if (left >= kBatchGraphSteps && !p->graph) {
        s = capture(b, *p, L.st);
        if (s) return s;
    }
    while (left >= kBatchGraphSteps) {
        BHIP(b, hipGraphLaunch(p->graph, L.st), "graph launch");
        advance(b, act, kBatchGraphSteps);
        left -= kBatchGraphSteps;
    }
    for (; left > 0; left--) {
        s = batch_step(b, *p, L.st);
        if (s) return s;
        advance(b, act, 1);
    }
    L.budget -= len;
    L.queued += cost * (double)len;
    return CPIC_OK;
}

// Advance every event by up to max_steps steps (to its end when max_steps <
// 0).  The launch groups are dealt to the lanes by their remaining work,
// largest first, each to the lane with less work so far; the host then feeds
// the lanes segment by segment, always the one with less work enqueued, so
// both streams stay busy.  Every event's work goes to its lane's stream (the
// events run on the batch stream again afterwards, which waits for the second
// lane).
static cpic_status run_steps(cpic_batch* b, int64_t max_steps)
{
    for (size_t e = 0; e < b->ev.size(); e++)
        if (!b->ev[e]->initialised)
            return bfail(b, CPIC_E_INVALID, "cpic_batch_run: event " + std::to_string(e) + " has no state");
    cpic_status s = upload_desc(b);
    if (s) return s;
    const std::vector<std::vector<int>> groups = launch_groups(b);
    const int nl = std::max(1, std::min<int>(b->lanes, (int)groups.size()));
    for (int l = 1; l < nl; l++) {
        if (!b->lane_st[l]) BHIP(b, hipStreamCreateWithFlags(&b->lane_st[l], hipStreamNonBlocking), "lane stream");
        if (!b->ev_join[l]) BHIP(b, hipEventCreateWithFlags(&b->ev_join[l], hipEventDisableTiming), "lane event");
    }
    if (nl > 1 && !b->ev_fork) BHIP(b, hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming), "lane event");
    Lane lane[kMaxLanes];
    lane[0].st = b->st;
    for (int l = 1; l < nl; l++) lane[l].st = b->lane_st[l];
    std::vector<std::pair<double, int>> work;
    for (size_t g = 0; g < groups.size(); g++) {
        double w = 0;
        for (int e : groups[g]) {
            const cpic_ctx* c = b->ev[e];
            int64_t steps = std::max<int64_t>(c->sc.n_max - c->n, 0);
            if (max_steps >= 0) steps = std::min<int64_t>(steps, max_steps);
            w += step_cost(c) * (double)steps;
        }
        work.emplace_back(w, (int)g);
    }
    std::stable_sort(work.begin(), work.end(), [](const std::pair<double, int>& x, const std::pair<double, int>& y) {
        return x.first > y.first;
    });
    double total[kMaxLanes] = {};
    for (const auto& wg : work) {
        int l = 0;
        for (int k = 1; k < nl; k++)
            if (total[k] < total[l]) l = k;
        lane[l].groups.push_back(groups[wg.second]);
        total[l] += wg.first;
    }
    // odd lanes take their groups smallest first, so that large groups run
    // beside small ones rather than beside each other
    for (int l = 1; l < nl; l += 2) std::reverse(lane[l].groups.begin(), lane[l].groups.end());
    for (int l = 0; l < nl; l++) {
        lane[l].budget = max_steps < 0 ? (int64_t)1 << 40 : max_steps;
        for (const auto& g : lane[l].groups)
            for (int e : g) b->ev[e]->st = lane[l].st;
    }
    if (nl > 1) {
        BHIP(b, hipEventRecord(b->ev_fork, b->st), "lane fork");
        for (int l = 1; l < nl; l++) BHIP(b, hipStreamWaitEvent(lane[l].st, b->ev_fork, 0), "lane fork");
    }
    while (s == CPIC_OK) {
        int l = -1;
        for (int k = 0; k < nl; k++)
            if (!lane[k].done() && (l < 0 || lane[k].queued < lane[l].queued)) l = k;
        if (l < 0) break;
        s = lane_segment(b, lane[l], max_steps);
    }
    for (cpic_ctx* c : b->ev) c->st = b->st;
    for (int l = 1; l < nl; l++) {
        hipError_t e = hipEventRecord(b->ev_join[l], lane[l].st);
        if (e == hipSuccess) e = hipStreamWaitEvent(b->st, b->ev_join[l], 0);
        if (e != hipSuccess && s == CPIC_OK) s = bhip(b, e, "lane join");
    }
    return s;
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
// A candidate's time is the sum over the launch groups of one step.
template <typename T> static cpic_status tune_batch(cpic_batch* b, int reps, std::string& rep)
{
    std::vector<std::vector<int>> groups;
    for (const auto& g : launch_groups(b)) {
        std::vector<int> act;
        for (int e : g)
            if (b->ev[e]->n < b->ev[e]->sc.n_max) act.push_back(e);
        if (!act.empty()) groups.push_back(act);
    }
    if (groups.empty()) return CPIC_OK;
    cpic_status s = upload_desc(b);
    if (s) return s;
    static const int shapes[][2] = {{64, 4}, {32, 8}, {16, 16}, {32, 4}};
    size_t most = 1;  // largest work map over shapes and groups
    for (const auto& sh : shapes)
        for (const auto& g : groups) {
            LaunchCfg cfg{};
            cfg.split = 3;
            cfg.bx = sh[0];
            cfg.by = sh[1];
            size_t n = 0;
            for (int ev : g) n += (size_t)field_tiles_host(b->ev[ev]->N, cfg);
            most = std::max(most, n);
        }
    int2* d_map = nullptr;
    BHIP(b, hipMalloc(&d_map, sizeof(int2) * most), "tune");
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    const LaunchCfg keep = b->cfg;
    LaunchCfg best = keep;
    float best_ms = 1e30f;
    char line[160];
    std::vector<int2> map;
    for (const auto& sh : shapes)
        for (int remap = 0; remap < 2 && e == hipSuccess; remap++) {
            LaunchCfg cfg{};
            cfg.split = 3;
            cfg.bx = sh[0];
            cfg.by = sh[1];
            cfg.xcd_remap = remap;
            float total = 0;
            for (const auto& g : groups) {
                map.clear();
                for (int ev : g)
                    for (int k = 0, nt = field_tiles_host(b->ev[ev]->N, cfg); k < nt; k++) map.push_back(make_int2(ev, k));
                const int nt = (int)map.size();
                if (e == hipSuccess) e = hipMemcpy(d_map, map.data(), sizeof(int2) * map.size(), hipMemcpyHostToDevice);
                if (e == hipSuccess) e = launch_batch_field<T>(b->d_desc, d_map, nt, cfg, b->st);  // warm-up
                if (e == hipSuccess) e = hipEventRecord(e0, b->st);
                for (int r = 0; r < reps && e == hipSuccess; r++) e = launch_batch_field<T>(b->d_desc, d_map, nt, cfg, b->st);
                if (e == hipSuccess) e = hipEventRecord(e1, b->st);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                total += ms / reps;
            }
            if (e != hipSuccess) break;
            std::snprintf(line, sizeof line, "batch field %3dx%-3d remap %d : %9.2f us per step (%zu groups)\n",
                          cfg.bx, cfg.by, remap, total * 1e3, groups.size());
            rep += line;
            if (total < best_ms) {
                best_ms = total;
                best = cfg;
            }
        }
    (void)hipFree(d_map);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return bhip(b, e, "tune");
    std::snprintf(line, sizeof line, "chosen: %dx%d remap %d (%.2f us)\n", best.bx, best.by, best.xcd_remap,
                  best_ms * 1e3);
    rep += line;
    if (best.bx != keep.bx || best.by != keep.by || best.xcd_remap != keep.xcd_remap) {
        b->cfg = best;
        drop_plans(b);  // work maps and graphs depend on the tile shape
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
    const bool shape = (bx == 64 && by == 4) || (bx == 32 && by == 8) || (bx == 16 && by == 16) || (bx == 32 && by == 4);
    if (!shape || (tpp != 1 && tpp != 2 && tpp != 4))
        return bfail(b, CPIC_E_INVALID, "cpic_batch_set_launch: tiles 64x4, 32x8, 16x16 or 32x4; tpp 1, 2 or 4");
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

extern "C" cpic_status cpic_batch_set_lanes(cpic_batch* b, int32_t lanes)
{
    if (!b) return bfail(nullptr, CPIC_E_INVALID, "cpic_batch_set_lanes: NULL");
    if (lanes < 1 || lanes > kMaxLanes) return bfail(b, CPIC_E_INVALID, "cpic_batch_set_lanes: 1 to 4");
    b->lanes = lanes;
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
    if (b->st) (void)hipStreamSynchronize(b->st);
    for (int l = 1; l < kMaxLanes; l++)
        if (b->lane_st[l]) (void)hipStreamSynchronize(b->lane_st[l]);
    drop_plans(b);
    (void)hipFree(b->d_desc);
    for (int l = 1; l < kMaxLanes; l++) {
        if (b->lane_st[l]) (void)hipStreamDestroy(b->lane_st[l]);
        if (b->ev_join[l]) (void)hipEventDestroy(b->ev_join[l]);
    }
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    for (auto c : b->ev) cpic_destroy(c);
    if (b->own_stream) (void)hipStreamDestroy(b->st);
    delete b;
}
