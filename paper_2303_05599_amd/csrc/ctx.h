// ctx.h -- the per-event context behind cpic_ctx, shared by the single-event
// API (capi.hip) and the batched driver (batch.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <utility>
#include <vector>

#include "../../include/cpic.h"
#include "internal.h"

namespace cpic {
constexpr int kGraphSteps = 16;  // steps per captured graph (even: buffers return to their parity)
}

struct cpic_ctx {
    cpic_glasma_params gp{};
    cpic_particle_params pp{};
    hipStream_t st = nullptr;
    bool own_stream = false;
    int N = 0, V = 0, prec = 0;
    int nc = 3;     // SU(N_c): 3, or 2 for the SU(2) variant
    int rps = 68;   // reals per site of a field buffer set (68 for SU(3), 20 for SU(2))
    size_t tsz = 8;
    double a_fm = 0, a_gev = 0;
    cpic::Schedule sc{};
    int n = 0;    // host mirror of the device step counter
    int cur = 0;  // buffer holding the state at step n
    int64_t np = 0;
    bool is_static = false;
    double mhat = 0;
    double q0[8]{}, q0eig[3]{}, q2ref = 0, q3ref = 0;
    void* fbuf[2] = {nullptr, nullptr};
    void* pr = nullptr;   // particle reals [19][np]
    void* gpl = nullptr;  // plaquette field G = Proj U_12 [8][V] for the push, force table and light-like paths
    int* pcell = nullptr;  // [2][np]
    int pblocks = 0, nslots = 0;
    double* partials = nullptr;  // [nslots][particle groups of 64][4]
    double* obs = nullptr;       // [nslots][4], summed from partials when samples are read
    int obs_reduced = 0;         // samples[0 .. obs_reduced) are summed into obs
    std::vector<std::pair<int, int>> samples;  // (slot, step n after which it was taken)
    std::vector<int> sample_groups;            // groups of partials each sample was written as
    int* pid = nullptr;    // original index of each particle record
    cpic::SortBufs sb{};
    bool static_sorted = false;
    int sorted_at = -1;   // step before which the records were last reordered
    int sort_tx = 0, sort_ty = 0;  // cell tiles of the current record order (0: not ordered)
    // fused step (field variant 4): record range and stragglers of every tile
    int* tile_start = nullptr;    // [tiles + 1]
    int* strag = nullptr;         // [np]
    int* strag_count = nullptr;   // [tiles]
    unsigned long long* d_strag_total = nullptr;  // stragglers pushed while kernel timing is on
    int* d_step = nullptr;
    int* d_err = nullptr;
    int* d_fails = nullptr;
    double* dpart = nullptr;  // diagnostics partials
    double* dout = nullptr;   // diagnostics results [8 + 2]
    int dcap = 0;
    cpic::LaunchCfg cfg{};
    int tpp = 1;          // wavefronts per particle group in the gather push (1, 2, 4, 8)
    int push_table = 0;   // 1: fields from a per-site force table (dense ensembles)
    void* ftab = nullptr; // [48][V] force table (table push, light-like paths)
    bool initialised = false;
    // graphs: [sorted][parity][k] -> executable graph of k steps starting from
    // buffer `parity` (k = kGraphSteps between reordering points, shorter ones
    // up to the next reordering point or the end of an evolve); sorted = 1:
    // the graph starts with the reordering of the records (moving particles
    // at a reordering point)
    hipGraphExec_t gexec[2][2][cpic::kGraphSteps + 1] = {};
    // light-like paths (cpic_jets_enable)
    bool jets = false;
    cpic::JetArgs ja{};
    double jet_q2 = 0;             // q2 of the representation the broadening is quoted for
    void* jW = nullptr;            // [18][V] Wilson lines
    void* jF = nullptr;            // [24][V] integrated transported forces
    int jslots = 0;
    double* jpartials = nullptr;   // [jslots][path groups of 64][4]
    double* jobs = nullptr;        // [jslots][4]
    int jobs_reduced = 0;
    std::vector<std::pair<int, int>> jsamples;  // (slot, step n after which it was taken)
    // timing
    bool timing = false;
    std::vector<hipEvent_t> ev_field, ev_push, ev_jets, ev_table;
    double t_field = 0, t_push = 0, t_jets = 0;
    int64_t k_field = 0, k_push = 0, k_jets = 0;
    // drift watchdog: every watch_every steps (0: off) the diagnostics are
    // compared on the device with thresholds and with a baseline taken when
    // the state was installed; cpic_sync reports a breach
    int watch_every = 64;
    double watch_thr[3] = {1e-8, 1e-8, 1e-8};  // unitarity, Gauss drift, Casimir drift
    bool watch_base_due = true;
    int* d_watch = nullptr;        // [2] flags, step of the first breach (d_err + 1)
    // pinned host staging: d_err[0..3], then the summed samples obs [nslots][4]
    // (copied with the stream's last work, read after one synchronisation)
    void* h_stage = nullptr;
    double* d_watchv = nullptr;    // [4] its values
    double* d_watchbase = nullptr; // [10] baseline diagnostics
    std::string err;
};

namespace cpic {
cpic_status fail(cpic_ctx* c, cpic_status code, const std::string& msg);
cpic_status hip_fail(cpic_ctx* c, hipError_t e, const char* where);
// reorder the particle records by cell if step c->n is a reordering point
cpic_status maybe_sort(cpic_ctx* c);
// first reordering point after step n (1 << 30 if none)
int next_sort_point(const cpic_ctx* c, int n);
// host bookkeeping of k launched steps (sample list, step counter, buffer parity)
cpic_status host_advance(cpic_ctx* c, int k);
PushArgs push_args(const cpic_ctx* c, int tpp);
// the drift watchdog's baseline of a newly installed state, before its first step
cpic_status watch_prepare(cpic_ctx* c);
// the fused step can serve this context: SU(3), particles, the rotation
// colour update, no light-like paths
bool fused_ok(const cpic_ctx* c);
// the fused step is the current launch
bool fused_active(const cpic_ctx* c);
// device address of the allocation-free entry point's scratch array on the
// current device (resolved once per device; noalloc.hip)
cpic_status noalloc_scratch(double** out);
}  // namespace cpic
