// capi.hip -- the C ABI of libcpic (include/cpic.h): context lifecycle,
// initial condition, stepping (eager or replayed HIP graphs), observables,
// diagnostics, state exchange and checkpoints for one Glasma event.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/cpic.h"
#include "ctx.h"
#include "internal.h"

using namespace cpic;

namespace {

constexpr double kHbarC = 0.1973269804;  // GeV fm

// Initial colour vectors with the classical Casimirs of Sec. IV ([eq:q23_main]):
// fundamental q2 = 4, q3 = 10/3 from Q^5 and Q^8 alone (as in [eq:initq0]),
// Q8 the root of Q8^3 - 12 Q8 - 20/sqrt(3) = 0 closest to -1.062; adjoint Q^1 = sqrt(24).
void initial_colour(int rep, double q0[8], double eig[3], double* q2, double* q3)
{
    for (int a = 0; a < 8; a++) q0[a] = 0;
    if (rep == CPIC_REP_ADJ) {
        q0[0] = std::sqrt(24.0);
        eig[0] = -std::sqrt(6.0); eig[1] = 0; eig[2] = std::sqrt(6.0);
        *q2 = 24; *q3 = 0;
        return;
    }
    // Newton on f(q) = q^3 - 12 q - 20/sqrt(3) from -1
    double q = -1.0;
    for (int it = 0; it < 60; it++) {
        const double f = q * q * q - 12 * q - 20 / std::sqrt(3.0), df = 3 * q * q - 12;
        const double nq = q - f / df;
        if (nq == q) break;
        q = nq;
    }
    q0[7] = q;
    q0[4] = -std::sqrt(4 - q * q);
    // Q = Q5 T5 + Q8 T8: eigenvalues Q8/sqrt(3)/... from the 1-3 block and the 2-2 entry
    const double s3 = std::sqrt(3.0);
    const double d11 = q / (2 * s3);            // (T8)_22 Q8
    const double a = q / (2 * s3), c = -q / s3; // 1-3 block diagonal
    const double b = std::fabs(q0[4]) / 2;      // |off-diagonal|
    const double m = 0.5 * (a + c), r = std::sqrt(0.25 * (a - c) * (a - c) + b * b);
    double e[3] = {m - r, d11, m + r};
    std::sort(e, e + 3);
    for (int k = 0; k < 3; k++) eig[k] = e[k];
    *q2 = 4;
    *q3 = 10.0 / 3.0;
}

std::string g_static_error = "no error";

}  // namespace

cpic_status cpic::fail(cpic_ctx* c, cpic_status code, const std::string& msg)
{
    if (c) c->err = msg; else g_static_error = msg;
    return code;
}
cpic_status cpic::hip_fail(cpic_ctx* c, hipError_t e, const char* where)
{
    return fail(c, CPIC_E_HIP, std::string(where) + ": " + hipGetErrorString(e));
}
#define HIPCHK(c, x, where)                            \
    do {                                               \
        hipError_t e_ = (x);                           \
        if (e_ != hipSuccess) return hip_fail(c, e_, where); \
    } while (0)

template <typename T> static Fields<T> F(cpic_ctx* c, int b) { return fields_at<T>(c->fbuf[b], c->V); }
template <typename T> static Fields2<T> F2(cpic_ctx* c, int b) { return fields2_at<T>(c->fbuf[b], c->V); }
template <typename T> static Parts<T> P(cpic_ctx* c) { return {static_cast<T*>(c->pr), c->pcell}; }

static bool valid_N(int N)
{
    if (N < 4 || N > 1024) return false;
    while (N % 2 == 0) N /= 2;
    while (N % 3 == 0) N /= 3;
    return N == 1;
}

static void free_all(cpic_ctx* c)
{
    for (auto& byp : c->gexec)
        for (auto& byk : byp)
            for (auto& g : byk)
                if (g) (void)hipGraphExecDestroy(g);
    for (auto e : c->ev_field) (void)hipEventDestroy(e);
    for (auto e : c->ev_push) (void)hipEventDestroy(e);
    for (auto e : c->ev_jets) (void)hipEventDestroy(e);
    for (auto e : c->ev_table) (void)hipEventDestroy(e);
    (void)hipFree(c->ftab);
    (void)hipFree(c->jW); (void)hipFree(c->jF); (void)hipFree(c->jpartials); (void)hipFree(c->jobs);
    (void)hipFree(c->fbuf[0]); (void)hipFree(c->fbuf[1]); (void)hipFree(c->pr); (void)hipFree(c->pcell); (void)hipFree(c->gpl);
    (void)hipFree(c->partials); (void)hipFree(c->obs); (void)hipFree(c->d_step); (void)hipFree(c->d_err); (void)hipFree(c->d_fails);
    (void)hipFree(c->d_watchv); (void)hipFree(c->d_watchbase);
    if (c->h_stage) (void)hipHostFree(c->h_stage);
    (void)hipFree(c->dpart); (void)hipFree(c->dout);
    (void)hipFree(c->pid); (void)hipFree(c->sb.keys); (void)hipFree(c->sb.keys2); (void)hipFree(c->sb.perm);
    (void)hipFree(c->sb.temp); (void)hipFree(c->sb.r2); (void)hipFree(c->sb.cell2); (void)hipFree(c->sb.pid2);
    (void)hipFree(c->sb.count); (void)hipFree(c->sb.offs);
    (void)hipFree(c->tile_start); (void)hipFree(c->strag); (void)hipFree(c->strag_count);
    (void)hipFree(c->d_strag_total);
    if (c->own_stream && c->st) (void)hipStreamDestroy(c->st);
}

// Store policy of the field update.  After the field update a step reads the
// old state and the new E and pi (push, force table), the particle records
// and the light-like paths; where these, the new links and phi and the force
// table together exceed the 256 MB last-level cache (FP64 at 512^2 with 1e5
// particles: 300 MB), the new state is stored non-temporal so that it does not
// displace the old state the push reads next.  cpic_tune times both.
static void set_store_policy(cpic_ctx* c)
{
    double reals = 2.0 * c->rps * (double)c->V + (double)kPartReals * (double)c->np;
    if (c->push_table || c->jets) reals += 48.0 * (double)c->V;
    if (c->jets) reals += 42.0 * (double)c->V;
    c->cfg.nt_store = (c->np > 0 || c->jets) && reals * (double)c->tsz > 256.0 * 1024 * 1024;
}

extern "C" cpic_status cpic_create(const cpic_glasma_params* gp, const cpic_particle_params* pp, void* hip_stream,
                                   cpic_ctx** out)
{
    if (!gp || !out) return fail(nullptr, CPIC_E_INVALID, "cpic_create: NULL argument");
    *out = nullptr;
    if (!valid_N(gp->N)) return fail(nullptr, CPIC_E_INVALID, "cpic_create: N must be 2^p 3^q in [4, 1024]");
    if (!(gp->L_fm > 0) || !(gp->dtau_over_a > 0) || !(gp->tau_max_fm > 0) || gp->n_sheets < 1 ||
        !(gp->g2mu_GeV >= 0) || !(gp->m_ir_GeV >= 0))
        return fail(nullptr, CPIC_E_INVALID, "cpic_create: L, dtau, tau_max, n_sheets must be positive");
    if (gp->precision != CPIC_FP64 && gp->precision != CPIC_FP32)
        return fail(nullptr, CPIC_E_INVALID, "cpic_create: precision must be CPIC_FP64 or CPIC_FP32");
    if (gp->n_colors != 0 && gp->n_colors != 2 && gp->n_colors != 3)
        return fail(nullptr, CPIC_E_INVALID, "cpic_create: n_colors must be 2 or 3 (0: 3)");
    cpic_particle_params none{};
    if (!pp) pp = &none;
    if (gp->n_colors == 2 && pp->n > 0 && pp->color_update != CPIC_COLOR_ROTATE)
        return fail(nullptr, CPIC_E_INVALID, "cpic_create: the SU(2) variant rotates the charges with the links");
    // particle records are addressed through 32-bit buffer offsets: a
    // component array and the whole record set must stay below 2 GiB
    const int64_t tsz_p = gp->precision == CPIC_FP64 ? 8 : 4;
    if (pp->n < 0 || pp->n > (int64_t)INT32_MAX / (kPartReals * tsz_p))
        return fail(nullptr, CPIC_E_INVALID,
                    "cpic_create: particle count out of range (records must stay below 2 GiB: at most " +
                        std::to_string((int64_t)INT32_MAX / (kPartReals * tsz_p)) + " in this precision)");
    if (pp->n > 0 && (!(pp->mass_GeV > 0) || pp->pT_min_GeV < 0 || pp->pT_max_GeV < pp->pT_min_GeV ||
                      pp->tau_form_fm < 0 || (pp->rep != CPIC_REP_FUND && pp->rep != CPIC_REP_ADJ) ||
                      (pp->color_update != CPIC_COLOR_ROTATE && pp->color_update != CPIC_COLOR_LOG)))
        return fail(nullptr, CPIC_E_INVALID, "cpic_create: bad particle parameters");

    {
        const double steps = gp->tau_max_fm / (gp->dtau_over_a * gp->L_fm / gp->N);
        const double form = pp->n > 0 ? pp->tau_form_fm / (gp->dtau_over_a * gp->L_fm / gp->N) : 0.0;
        if (!(steps < 1e8) || !(form < 1e8))
            return fail(nullptr, CPIC_E_INVALID, "cpic_create: tau_max / dtau or tau_form / dtau above 1e8 steps");
    }
    cpic_ctx* c = new cpic_ctx();
    c->gp = *gp;
    c->pp = *pp;
    c->N = gp->N;
    c->V = gp->N * gp->N;
    c->prec = gp->precision;
    c->tsz = c->prec == CPIC_FP64 ? 8 : 4;
    c->nc = gp->n_colors == 2 ? 2 : 3;
    c->rps = c->nc == 2 ? kRealsPerSite2 : kRealsPerSite;
    c->a_fm = gp->L_fm / gp->N;
    c->a_gev = c->a_fm / kHbarC;
    const double dtau_fm = gp->dtau_over_a * c->a_fm;
    const double steps = gp->tau_max_fm / dtau_fm;
    c->sc.dt = gp->dtau_over_a;
    c->sc.n_max = (int)std::ceil(steps - 1e-9 * steps);
    c->np = pp->n;
    c->is_static = std::isinf(pp->mass_GeV);
    c->mhat = c->is_static ? 0.0 : pp->mass_GeV * c->a_gev;
    if (pp->n > 0) {
        const double f = pp->tau_form_fm / dtau_fm;
        c->sc.n_form = (int)std::ceil(f - 1e-9 * f);
    } else {
        c->sc.n_form = c->sc.n_max;
    }
    c->sc.n_plaq = c->sc.n_form;
    c->sc.record_every = gp->record_every > 0 ? gp->record_every : (1 << 30);
    c->sc.reunit_every = c->prec == CPIC_FP32 ? std::max(0, gp->reunit_every) : 0;
    initial_colour(pp->rep, c->q0, c->q0eig, &c->q2ref, &c->q3ref);
    if (c->nc == 2) {  // [eq:q23c23] for N_c = 2: q2 = D_R C_2(R) = 3/2 (F), 6 (A); q3 = 0
        c->q2ref = pp->rep == CPIC_REP_ADJ ? 6.0 : 1.5;
        c->q3ref = 0;
    }

    hipError_t e = hipSuccess;
    if (hip_stream) {
        c->st = (hipStream_t)hip_stream;
    } else {
        e = hipStreamCreateWithFlags(&c->st, hipStreamNonBlocking);
        c->own_stream = e == hipSuccess;
    }
    const size_t fbytes = (size_t)c->rps * c->V * c->tsz;
    for (int b = 0; b < 2 && e == hipSuccess; b++) e = hipMalloc(&c->fbuf[b], fbytes);
    if (e == hipSuccess && c->np > 0) {
        const size_t np = c->np;
        e = hipMalloc(&c->pr, (size_t)kPartReals * np * c->tsz);
        if (e == hipSuccess) e = hipMalloc(&c->pcell, sizeof(int) * 2 * np);
        if (e == hipSuccess && c->nc == 3) e = hipMalloc(&c->gpl, (size_t)kPlaqReals * c->V * c->tsz);
        if (e == hipSuccess) e = hipMalloc(&c->pid, sizeof(int) * np);
        if (e == hipSuccess) e = hipMalloc(&c->sb.keys, sizeof(unsigned) * np);
        if (e == hipSuccess) e = hipMalloc(&c->sb.keys2, sizeof(unsigned) * np);
        if (e == hipSuccess) e = hipMalloc(&c->sb.perm, sizeof(int) * np);
        if (e == hipSuccess) e = hipMalloc(&c->sb.r2, (size_t)kPartReals * np * c->tsz);
        if (e == hipSuccess) e = hipMalloc(&c->sb.cell2, sizeof(int) * 2 * np);
        if (e == hipSuccess) e = hipMalloc(&c->sb.pid2, sizeof(int) * np);
        c->sb.key_cap = key_capacity(c->N);
        if (e == hipSuccess) e = hipMalloc(&c->sb.count, sizeof(int) * (size_t)c->sb.key_cap);
        if (e == hipSuccess) e = hipMalloc(&c->sb.offs, sizeof(int) * (size_t)c->sb.key_cap);
        // the reordering keeps the key counts zero between its calls
        if (e == hipSuccess) e = hipMemsetAsync(c->sb.count, 0, sizeof(int) * (size_t)c->sb.key_cap, c->st);
        c->sb.temp_bytes = std::max<size_t>(sort_temp_bytes(c->N), 16);
        if (e == hipSuccess) e = hipMalloc(&c->sb.temp, c->sb.temp_bytes);
        if (c->nc == 3) {
            const int nt = fused_tiles(c->N, 8, 8);  // the most tiles of any fused shape
            if (e == hipSuccess) e = hipMalloc(&c->tile_start, sizeof(int) * (nt + 1));
            if (e == hipSuccess) e = hipMalloc(&c->strag, sizeof(int) * np);
            if (e == hipSuccess) e = hipMalloc(&c->strag_count, sizeof(int) * nt);
            if (e == hipSuccess) e = hipMalloc(&c->d_strag_total, sizeof(unsigned long long));
            if (e == hipSuccess) e = hipMemsetAsync(c->d_strag_total, 0, sizeof(unsigned long long), c->st);
        }
    }
    // few particles: several wavefronts share each particle group so that the
    // push still fills the 1024 SIMDs (tunable with cpic_tune)
    c->tpp = c->nc == 2 ? 1 : (c->np <= (1 << 18) ? 4 : (c->np <= (1 << 20) ? 2 : 1));
    // more particles than sites: evaluate the fields once per site (force table)
    c->push_table = c->nc == 3 && c->np > c->V && c->pp.color_update == CPIC_COLOR_ROTATE;
    if (e == hipSuccess && c->push_table) e = hipMalloc(&c->ftab, (size_t)48 * c->V * c->tsz);
    // field update: compressed-link LDS tiles of 64 x 8 sites (the tuner's pick
    // at 512^2, 1-2 % per step ahead of 64 x 4).  The fused step (variant 4)
    // is chosen explicitly: at 512^2 with 1e5 particles it computes the
    // fields at every site of a tile, more FP64 work than the gather push's
    // evaluation at the particles' cells (0.145 against 0.127 ms per step)
    c->cfg.split = 3;
    c->cfg.bx = 64;
    c->cfg.by = 8;
    set_store_policy(c);
    c->pblocks = c->np > 0 ? push_blocks((int)c->np, c->tpp) : 0;
    c->nslots = c->np > 0 ? num_slots(c->sc) : 0;
    if (e == hipSuccess && c->nslots > 0) {
        const int groups = std::max(obs_groups((int)c->np), c->nc == 3 ? fused_groups_max(c->N) : 0);
        e = hipMalloc(&c->partials, sizeof(double) * 4 * (size_t)groups * c->nslots);
        if (e == hipSuccess) e = hipMalloc(&c->obs, sizeof(double) * 4 * c->nslots);
    }
    if (e == hipSuccess) e = hipMalloc(&c->d_step, 2 * sizeof(int));
    // d_err[0]: cell jumps; d_err[1..2]: the watchdog's flags and step (read
    // together by cpic_sync)
    if (e == hipSuccess) e = hipMalloc(&c->d_err, 4 * sizeof(int));
    c->d_watch = c->d_err + 1;
    if (e == hipSuccess) e = hipMalloc(&c->d_watchv, 4 * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&c->d_watchbase, 10 * sizeof(double));
    if (e == hipSuccess) e = hipHostMalloc(&c->h_stage, 4 * sizeof(int) + sizeof(double) * 4 * (size_t)c->nslots);
    if (c->prec == CPIC_FP32) c->watch_thr[0] = c->watch_thr[1] = c->watch_thr[2] = 1e-2;
    if (e == hipSuccess) e = hipMalloc(&c->d_fails, sizeof(int));
    c->dcap = std::max((c->V + 255) / 256, std::max(c->np > 0 ? push_blocks((int)c->np, 1) : 0, 1));
    if (e == hipSuccess) e = hipMalloc(&c->dpart, sizeof(double) * 8 * c->dcap);
    if (e == hipSuccess) e = hipMalloc(&c->dout, sizeof(double) * 16);
    // the allocation-free entry point's scratch array: its device address on
    // this device is resolved here, at set-up, rather than inside that call
    double* scratch_dev = nullptr;
    if (e == hipSuccess && noalloc_scratch(&scratch_dev) != CPIC_OK) e = hipErrorInvalidSymbol;
    if (e == hipSuccess) e = hipMemsetAsync(c->d_step, 0, 2 * sizeof(int), c->st);
    if (e == hipSuccess) e = hipMemsetAsync(c->d_err, 0, 4 * sizeof(int), c->st);
    if (e == hipSuccess && c->obs) e = hipMemsetAsync(c->obs, 0, sizeof(double) * 4 * c->nslots, c->st);
    if (e == hipSuccess) e = hipStreamSynchronize(c->st);
    if (e != hipSuccess) {
        const bool oom = e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation;
        free_all(c);
        delete c;
        return fail(nullptr, oom ? CPIC_E_NOMEM : CPIC_E_HIP, std::string("cpic_create: ") + hipGetErrorString(e));
    }
    *out = c;
    return CPIC_OK;
}

extern "C" void cpic_destroy(cpic_ctx* c)
{
    if (!c) return;
    if (c->st) (void)hipStreamSynchronize(c->st);
    free_all(c);
    delete c;
}

extern "C" const char* cpic_last_error(const cpic_ctx* c) { return c ? c->err.c_str() : g_static_error.c_str(); }

static cpic_status reset_pid(cpic_ctx* c)
{
    if (c->np <= 0) return CPIC_OK;
    std::vector<int> iota(c->np);
    for (int64_t p = 0; p < c->np; p++) iota[p] = (int)p;
    HIPCHK(c, hipMemcpy(c->pid, iota.data(), sizeof(int) * iota.size(), hipMemcpyHostToDevice), "pid");
    c->static_sorted = false;
    c->sorted_at = -1;
    c->sort_tx = c->sort_ty = 0;
    return CPIC_OK;
}

bool cpic::fused_ok(const cpic_ctx* c)
{
    return c->nc == 3 && c->np > 0 && c->pp.color_update == CPIC_COLOR_ROTATE && !c->jets && c->tile_start;
}
bool cpic::fused_active(const cpic_ctx* c) { return c->cfg.split == 4 && fused_ok(c); }
// the cell tiles the records are ordered by for the current launch
static void sort_tiles(const cpic_ctx* c, int* tx, int* ty)
{
    *tx = fused_active(c) ? c->cfg.bx : kGatherSortTileX;
    *ty = fused_active(c) ? c->cfg.by : kGatherSortTileY;
}

// Particle records are reordered by cell before step n when n is the first
// push step or a multiple of kSortEvery (moving particles); static particles
// never change cell and are ordered once.  The fused step needs the records
// ordered by its own tiles: any push step finds them so.
static bool is_sort_point(const cpic_ctx* c, int n)
{
    if (c->np < 1 || n < c->sc.n_form || n >= c->sc.n_max) return false;
    if (fused_active(c) && (c->sort_tx != c->cfg.bx || c->sort_ty != c->cfg.by)) return true;
    if (c->np == 1) return false;
    if (c->is_static) return !c->static_sorted;
    return n == c->sc.n_form || n % kSortEvery == 0;
}
int cpic::next_sort_point(const cpic_ctx* c, int n)
{
    if (c->np <= 1 || n + 1 > c->sc.n_max) return 1 << 30;
    if (c->is_static) return (!c->static_sorted && n + 1 <= c->sc.n_form) ? c->sc.n_form : 1 << 30;
    int m = n + 1;
    if (m <= c->sc.n_form) return c->sc.n_form;
    m = ((m + kSortEvery - 1) / kSortEvery) * kSortEvery;
    return m;
}
// whether the records are due for a reordering before step n, and by which tiles
static bool sort_due(const cpic_ctx* c, int* tx, int* ty)
{
    sort_tiles(c, tx, ty);
    return is_sort_point(c, c->n) && !(c->sorted_at == c->n && c->sort_tx == *tx && c->sort_ty == *ty);
}
// enqueue the reordering (also under graph capture: no memset, no synchronisation)
static hipError_t enqueue_sort(cpic_ctx* c, int tx, int ty)
{
    // the tile ranges wherever the order is one a fused step can use
    int* ts = c->tile_start && fused_shape(tx, ty) ? c->tile_start : nullptr;
    const bool pos = !c->is_static;
    return c->prec == CPIC_FP64
               ? sort_particles<double>(c->sb, (double*)c->pr, c->pcell, c->pid, (int)c->np, c->N, tx, ty, pos, ts,
                                        c->st)
               : sort_particles<float>(c->sb, (float*)c->pr, c->pcell, c->pid, (int)c->np, c->N, tx, ty, pos, ts,
                                       c->st);
}
static void mark_sorted(cpic_ctx* c, int tx, int ty)
{
    c->sorted_at = c->n;
    c->sort_tx = tx;
    c->sort_ty = ty;
    if (c->is_static) c->static_sorted = true;
}
cpic_status cpic::maybe_sort(cpic_ctx* c)
{
    int tx, ty;
    if (!sort_due(c, &tx, &ty)) return CPIC_OK;
    c->sorted_at = c->n;
    const hipError_t e = enqueue_sort(c, tx, ty);
    if (e != hipSuccess) return hip_fail(c, e, "particle sort");
    mark_sorted(c, tx, ty);
    return CPIC_OK;
}

static void drop_graphs(cpic_ctx* c)
{
    for (auto& byp : c->gexec)
        for (auto& byk : byp)
            for (auto& g : byk)
                if (g) {
                    (void)hipGraphExecDestroy(g);
                    g = nullptr;
                }
}

static cpic_status reset_counters(cpic_ctx* c, int n)
{
    c->n = n;
    c->watch_base_due = true;
    c->samples.clear();
    c->sample_groups.clear();
    c->obs_reduced = 0;
    c->jsamples.clear();
    c->jobs_reduced = 0;
    HIPCHK(c, hipMemcpyAsync(c->d_step, &c->n, sizeof(int), hipMemcpyHostToDevice, c->st), "step counter");
    if (c->obs) HIPCHK(c, hipMemsetAsync(c->obs, 0, sizeof(double) * 4 * c->nslots, c->st), "obs reset");
    if (c->jobs) HIPCHK(c, hipMemsetAsync(c->jobs, 0, sizeof(double) * 4 * c->jslots, c->st), "obs reset");
    HIPCHK(c, hipStreamSynchronize(c->st), "reset");
    return CPIC_OK;
}

extern "C" cpic_status cpic_init_mv(cpic_ctx* c)
{
    if (!c) return fail(nullptr, CPIC_E_INVALID, "cpic_init_mv: NULL context");
    ICArgs a{};
    a.N = c->N;
    a.n_sheets = c->gp.n_sheets;
    a.seed = c->gp.seed;
    a.g2mua = c->gp.g2mu_GeV * c->a_gev;
    a.mhat = c->gp.m_ir_GeV * c->a_gev;
    a.uvhat = c->gp.uv_GeV > 0 ? c->gp.uv_GeV * c->a_gev : 0.0;
    a.tol = 1e-14;
    a.maxit = 50;
    void* dbl = c->fbuf[0];
    void* stage = nullptr;
    if (c->prec == CPIC_FP32) {
        HIPCHK(c, hipMalloc(&stage, sizeof(double) * c->rps * c->V), "IC staging");
        dbl = stage;
    }
    HIPCHK(c, hipMemsetAsync(c->d_fails, 0, sizeof(int), c->st), "IC");
    hipError_t e = c->nc == 2 ? ic_glasma2(a, fields2_at<double>(dbl, c->V), c->st)
                              : ic_glasma(a, fields_at<double>(dbl, c->V), c->d_fails, c->st);
    if (e == hipSuccess && c->prec == CPIC_FP32)
        e = convert_to_float((const double*)stage, (float*)c->fbuf[0], (size_t)c->rps * c->V, c->st);
    if (e == hipSuccess && c->np > 0) {
        PartICArgs pa{};
        pa.N = c->N;
        pa.np = (int)c->np;
        pa.azimuth_uniform = c->pp.azimuth_uniform;
        pa.seed = c->pp.seed;
        pa.pt_min = c->pp.pT_min_GeV * c->a_gev;
        pa.pt_max = c->pp.pT_max_GeV * c->a_gev;
        for (int k = 0; k < 8; k++) pa.q0[k] = c->q0[k];
        double* pdst = (double*)c->pr;
        void* pstage = nullptr;
        if (c->prec == CPIC_FP32) {
            e = hipMalloc(&pstage, sizeof(double) * kPartReals * c->np);
            pdst = (double*)pstage;
        }
        if (e == hipSuccess)
            e = c->nc == 2 ? ic_particles2(pa, c->q2ref, pdst, c->pcell, c->st) : ic_particles(pa, pdst, c->pcell, c->st);
        if (e == hipSuccess && c->prec == CPIC_FP32)
            e = convert_to_float(pdst, (float*)c->pr, (size_t)kPartReals * c->np, c->st);
        if (e == hipSuccess) e = hipStreamSynchronize(c->st);
        (void)hipFree(pstage);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(c->st);
    (void)hipFree(stage);
    if (e != hipSuccess) return hip_fail(c, e, "cpic_init_mv");
    int fails = 0;
    HIPCHK(c, hipMemcpy(&fails, c->d_fails, sizeof(int), hipMemcpyDeviceToHost), "IC");
    c->cur = 0;
    c->initialised = true;
    cpic_status s = reset_counters(c, 0);
    if (s) return s;
    s = reset_pid(c);
    if (s) return s;
    if (fails) return fail(c, CPIC_E_IC_NEWTON, "cpic_init_mv: initial-link Newton solve failed on " +
                                                    std::to_string(fails) + " links");
    return CPIC_OK;
}

PushArgs cpic::push_args(const cpic_ctx* c, int tpp)
{
    PushArgs pa{};
    pa.N = c->N;
    pa.np = (int)c->np;
    pa.is_static = c->is_static;
    pa.tpp = tpp;
    pa.color_log = !c->is_static && c->pp.color_update == CPIC_COLOR_LOG;
    pa.mhat = c->mhat;
    for (int k = 0; k < 3; k++) pa.q0eig[k] = c->q0eig[k];
    pa.sc = c->sc;
    return pa;
}

// one step: field update (cur -> cur^1), push (advances the step counter),
// light-like paths
// SU(2) step: field update, push (or the step advance without particles)
template <typename T> static cpic_status launch_one_su2(cpic_ctx* c, int parity, bool with_events)
{
    const Fields2<T> A = F2<T>(c, parity), B = F2<T>(c, parity ^ 1);
    KTimer tf, tp;
    if (with_events) {
        HIPCHK(c, hipEventCreate(&tf.start), "event"); HIPCHK(c, hipEventCreate(&tf.stop), "event");
        c->ev_field.push_back(tf.start); c->ev_field.push_back(tf.stop);
    }
    HIPCHK(c, launch_su2_field<T>(A, B, c->N, c->sc, c->d_step, c->st, tf), "SU(2) field step");
    if (c->np > 0) {
        if (with_events) {
            HIPCHK(c, hipEventCreate(&tp.start), "event"); HIPCHK(c, hipEventCreate(&tp.stop), "event");
            c->ev_push.push_back(tp.start); c->ev_push.push_back(tp.stop);
        }
        HIPCHK(c, launch_su2_push<T>(A, B, P<T>(c), push_args(c, 1), c->d_step, c->partials, c->d_err, c->st, tp),
               "SU(2) push");
    } else {
        HIPCHK(c, launch_step_advance(c->d_step, c->st), "step advance");
    }
    return CPIC_OK;
}

// The force table serves the table push and the light-like paths: it is
// evaluated from the first step either of them needs, with the magnetic
// fields unless only static particles read it.
static bool uses_table(const cpic_ctx* c) { return c->ftab && ((c->np > 0 && c->push_table) || c->jets); }
static Schedule table_schedule(const cpic_ctx* c)
{
    Schedule s = c->sc;
    s.n_form = c->sc.n_max;
    if (c->np > 0 && c->push_table) s.n_form = std::min(s.n_form, c->sc.n_form);
    if (c->jets) s.n_form = std::min(s.n_form, c->ja.sc.n_form);
    return s;
}

template <typename T> static cpic_status launch_one(cpic_ctx* c, int parity, bool with_events)
{
    if (c->nc == 2) return launch_one_su2<T>(c, parity, with_events);
    const Fields<T> A = F<T>(c, parity), B = F<T>(c, parity ^ 1);
    auto timer = [&](std::vector<hipEvent_t>& evs, KTimer& tm) -> hipError_t {
        if (!with_events) return hipSuccess;
        hipError_t e = hipEventCreate(&tm.start);
        if (e == hipSuccess) e = hipEventCreate(&tm.stop);
        if (e == hipSuccess) { evs.push_back(tm.start); evs.push_back(tm.stop); }
        return e;
    };
    KTimer tf, tt, tp, tj;
    HIPCHK(c, timer(c->ev_field, tf), "event");
    if (fused_active(c)) {
        // the field update with the tile push (timed as the field kernel),
        // then the stragglers (timed as the push)
        HIPCHK(c, timer(c->ev_push, tp), "event");
        const TileParts tpa{c->tile_start, c->strag, c->strag_count, c->timing ? c->d_strag_total : nullptr};
        HIPCHK(c, launch_fused<T>(A, B, c->cfg, P<T>(c), push_args(c, 8), tpa,
                                  c->d_step, c->partials, c->d_err, c->st, tf, tp),
               "fused step");
        return CPIC_OK;
    }
    HIPCHK(c, launch_field_step<T>(A, B, static_cast<T*>(c->gpl), c->N, c->sc, c->d_step, c->cfg, c->st, tf),
           "field step");
    if (uses_table(c)) {
        HIPCHK(c, timer(c->ev_table, tt), "event");
        HIPCHK(c, launch_force_table<T>(A, B, static_cast<const T*>(c->gpl), static_cast<T*>(c->ftab), c->N,
                                        table_schedule(c), c->is_static && !c->jets, c->d_step, c->st, tt),
               "force table");
    }
    if (c->np > 0) {
        HIPCHK(c, timer(c->ev_push, tp), "event");
        if (c->push_table)
            HIPCHK(c, launch_push_table<T>(A, B, static_cast<const T*>(c->ftab), P<T>(c), push_args(c, 1), c->d_step,
                                           c->partials, c->d_err, c->st, tp), "table push");
        else
            HIPCHK(c, launch_push<T>(A, B, static_cast<const T*>(c->gpl), P<T>(c), push_args(c, c->tpp), c->d_step,
                                     c->partials, c->d_err, c->st, tp), "push");
    } else {
        // the push advances the step counter; without particles a one-thread kernel does
        HIPCHK(c, launch_step_advance(c->d_step, c->st), "step advance");
    }
    if (c->jets) {
        // reads the step from d_step[1], which only the next field update changes
        HIPCHK(c, timer(c->ev_jets, tj), "event");
        HIPCHK(c, launch_jets<T>(A, static_cast<const T*>(c->ftab), static_cast<T*>(c->jW), static_cast<T*>(c->jF),
                                 c->ja, c->d_step, c->jpartials, c->st, tj), "light-like paths");
    }
    return CPIC_OK;
}

static cpic_status enqueue_watch(cpic_ctx* c, bool take_base);

// groups of 4 partial sums a sample of the current launch writes
static int sample_groups_now(const cpic_ctx* c)
{
    return fused_active(c) ? fused_groups(c->N, c->cfg.bx, c->cfg.by) : obs_groups((int)c->np);
}

cpic_status cpic::host_advance(cpic_ctx* c, int k)
{
    const int n0 = c->n;
    for (int j = 0; j < k; j++) {
        if (c->np > 0 && is_record_step(c->sc, c->n)) {
            c->samples.push_back({record_slot_of(c->sc, c->n), c->n});
            c->sample_groups.push_back(sample_groups_now(c));
        }
        if (c->jets && is_record_step(c->ja.sc, c->n))
            c->jsamples.push_back({record_slot_of(c->ja.sc, c->n), c->n});
        c->n++;
        c->cur ^= 1;
    }
    // the drift watchdog after every multiple of watch_every steps
    if (c->watch_every > 0 && c->n / c->watch_every > n0 / c->watch_every) return enqueue_watch(c, false);
    return CPIC_OK;
}

static cpic_status eager_steps(cpic_ctx* c, int k)
{
    cpic_status ws = watch_prepare(c);
    if (ws) return ws;
    for (int j = 0; j < k; j++) {
        cpic_status so = maybe_sort(c);
        if (so) return so;
        const bool ev = c->timing;
        cpic_status s = c->prec == CPIC_FP64 ? launch_one<double>(c, c->cur, ev) : launch_one<float>(c, c->cur, ev);
        if (s) return s;
        host_advance(c, 1);
    }
    return CPIC_OK;
}

// a graph of k steps from buffer `parity`
// sorted: the graph starts with the reordering of the records by tx x ty tiles
static cpic_status build_graph(cpic_ctx* c, int parity, int k, bool sorted, int tx, int ty)
{
    hipGraph_t g = nullptr;
    HIPCHK(c, hipStreamBeginCapture(c->st, hipStreamCaptureModeThreadLocal), "capture");
    cpic_status s = CPIC_OK;
    if (sorted) {
        const hipError_t e = enqueue_sort(c, tx, ty);
        if (e != hipSuccess) s = hip_fail(c, e, "particle sort");
    }
    for (int j = 0; j < k && s == CPIC_OK; j++)
        s = c->prec == CPIC_FP64 ? launch_one<double>(c, parity ^ (j & 1), false)
                                 : launch_one<float>(c, parity ^ (j & 1), false);
    hipError_t e = hipStreamEndCapture(c->st, &g);
    if (s) { if (g) (void)hipGraphDestroy(g); return s; }
    if (e != hipSuccess) return hip_fail(c, e, "end capture");
    e = hipGraphInstantiate(&c->gexec[sorted ? 1 : 0][parity][k], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(c, e, "graph instantiate");
    return CPIC_OK;
}

extern "C" cpic_status cpic_step(cpic_ctx* c, int32_t k)
{
    if (!c) return fail(nullptr, CPIC_E_INVALID, "cpic_step: NULL context");
    if (!c->initialised) return fail(c, CPIC_E_INVALID, "cpic_step: no state (call cpic_init_mv or cpic_set_state)");
    if (k < 0 || c->n + (int64_t)k > c->sc.n_max)
        return fail(c, CPIC_E_INVALID, "cpic_step: would pass n_max = " + std::to_string(c->sc.n_max));
    return eager_steps(c, k);
}

extern "C" cpic_status cpic_evolve(cpic_ctx* c, double tau_target_fm)
{
    if (!c) return fail(nullptr, CPIC_E_INVALID, "cpic_evolve: NULL context");
    if (!c->initialised) return fail(c, CPIC_E_INVALID, "cpic_evolve: no state");
    const double dtau_fm = c->sc.dt * c->a_fm;
    const double f = tau_target_fm / dtau_fm;
    int target;
    if (!(f < (double)c->sc.n_max)) target = c->sc.n_max;  // also catches NaN and huge values
    else target = std::max(0, (int)std::ceil(f - 1e-9 * std::fabs(f)));
    if (target <= c->n) return CPIC_OK;
    int left = target - c->n;
    if (c->timing) return eager_steps(c, left);
    cpic_status ws = watch_prepare(c);
    if (ws) return ws;
    while (left > 0) {
        // a reordering of moving particles is the start of the stretch's graph;
        // static particles are ordered once, outside the graphs
        int tx, ty;
        const bool due = sort_due(c, &tx, &ty), in_graph = due && !c->is_static;
        if (due && !in_graph) {
            cpic_status so = maybe_sort(c);
            if (so) return so;
        }
        // one graph up to the next reordering point, at most kGraphSteps steps
        // (graphs of each length are captured once per buffer parity)
        const int k = std::min(std::min(left, kGraphSteps), std::max(1, next_sort_point(c, c->n) - c->n));
        const int parity = c->cur, sg = in_graph ? 1 : 0;
        if (!c->gexec[sg][parity][k]) {
            cpic_status s = build_graph(c, parity, k, in_graph, tx, ty);
            if (s) return s;
        }
        HIPCHK(c, hipGraphLaunch(c->gexec[sg][parity][k], c->st), "graph launch");
        if (in_graph) mark_sorted(c, tx, ty);
        host_advance(c, k);
        left -= k;
    }
    return CPIC_OK;
}

static cpic_status collect_timing(cpic_ctx* c)
{
    for (size_t i = 0; i + 1 < c->ev_field.size(); i += 2) {
        float ms = 0;
        HIPCHK(c, hipEventElapsedTime(&ms, c->ev_field[i], c->ev_field[i + 1]), "timing");
        c->t_field += ms;
        c->k_field++;
        (void)hipEventDestroy(c->ev_field[i]); (void)hipEventDestroy(c->ev_field[i + 1]);
    }
    for (size_t i = 0; i + 1 < c->ev_push.size(); i += 2) {
        float ms = 0;
        HIPCHK(c, hipEventElapsedTime(&ms, c->ev_push[i], c->ev_push[i + 1]), "timing");
        c->t_push += ms;
        c->k_push++;
        (void)hipEventDestroy(c->ev_push[i]); (void)hipEventDestroy(c->ev_push[i + 1]);
    }
    for (size_t i = 0; i + 1 < c->ev_table.size(); i += 2) {
        // the table kernel counts as push time (table push), else as light-like path time
        float ms = 0;
        HIPCHK(c, hipEventElapsedTime(&ms, c->ev_table[i], c->ev_table[i + 1]), "timing");
        (c->np > 0 && c->push_table ? c->t_push : c->t_jets) += ms;
        (void)hipEventDestroy(c->ev_table[i]); (void)hipEventDestroy(c->ev_table[i + 1]);
    }
    c->ev_table.clear();
    for (size_t i = 0; i + 1 < c->ev_jets.size(); i += 2) {
        float ms = 0;
        HIPCHK(c, hipEventElapsedTime(&ms, c->ev_jets[i], c->ev_jets[i + 1]), "timing");
        c->t_jets += ms;
        c->k_jets++;
        (void)hipEventDestroy(c->ev_jets[i]); (void)hipEventDestroy(c->ev_jets[i + 1]);
    }
    c->ev_field.clear();
    c->ev_push.clear();
    c->ev_jets.clear();
    return CPIC_OK;
}

extern "C" cpic_status cpic_sync(cpic_ctx* c)
{
    if (!c) return fail(nullptr, CPIC_E_INVALID, "cpic_sync: NULL context");
    // the error words come back with the stream's last work: one synchronisation
    int* err = static_cast<int*>(c->h_stage);
    HIPCHK(c, hipMemcpyAsync(err, c->d_err, 3 * sizeof(int), hipMemcpyDeviceToHost, c->st), "cpic_sync");
    HIPCHK(c, hipStreamSynchronize(c->st), "cpic_sync");
    if (c->timing) {
        cpic_status s = collect_timing(c);
        if (s) return s;
    }
    if (err[0]) {
        HIPCHK(c, hipMemset(c->d_err, 0, sizeof(int)), "cpic_sync");
        return fail(c, CPIC_E_CELL_JUMP, std::to_string(err[0]) + " particle moves of more than one cell");
    }
    if (err[1]) {
        double v[4];
        HIPCHK(c, hipMemcpy(v, c->d_watchv, sizeof v, hipMemcpyDeviceToHost), "cpic_sync");
        HIPCHK(c, hipMemset(c->d_watch, 0, 2 * sizeof(int)), "cpic_sync");
        std::string m = "watchdog after step " + std::to_string(err[2]) + ":";
        char b[160];
        if (err[1] & 1) m += " non-finite diagnostics;";
        if (err[1] & 2) { std::snprintf(b, sizeof b, " unitarity max|UU^+-1| = %.3e > %.1e;", v[0], c->watch_thr[0]); m += b; }
        if (err[1] & 4) { std::snprintf(b, sizeof b, " Gauss-law drift %.3e > %.1e;", v[1], c->watch_thr[1]); m += b; }
        if (err[1] & 8) {
            std::snprintf(b, sizeof b, " Casimir drift q2 %.3e, q3 %.3e > %.1e;", v[2], v[3], c->watch_thr[2]);
            m += b;
        }
        return fail(c, (err[1] & 1) ? CPIC_E_NAN : CPIC_E_DRIFT, m);
    }
    return CPIC_OK;
}

// Sum the per-group partials of every sample taken since the last call into
// obs[slot] (groups in order, fixed-order block reduction).
static cpic_status reduce_samples(cpic_ctx* c)
{
    // runs of samples in consecutive slots with one group count: one launch each
    for (size_t k = (size_t)c->obs_reduced; k < c->samples.size();) {
        const int slot = c->samples[k].first, groups = c->sample_groups[k];
        size_t j = k + 1;
        while (j < c->samples.size() && c->samples[j].first == slot + (int)(j - k) && c->sample_groups[j] == groups) j++;
        HIPCHK(c, launch_reduce_samples(c->partials, groups, slot, (int)(j - k), c->obs, c->st), "observables");
        k = j;
    }
    c->obs_reduced = (int)c->samples.size();
    // the light-like paths' samples likewise (the same [slot][group][4] layout)
    const int jg = jet_groups(c->V);
    for (size_t k = (size_t)c->jobs_reduced; k < c->jsamples.size();) {
        const int slot = c->jsamples[k].first;
        size_t j = k + 1;
        while (j < c->jsamples.size() && c->jsamples[j].first == slot + (int)(j - k)) j++;
        HIPCHK(c, launch_reduce_samples(c->jpartials, jg, slot, (int)(j - k), c->jobs, c->st), "light-like observables");
        k = j;
    }
    c->jobs_reduced = (int)c->jsamples.size();
    return CPIC_OK;
}

extern "C" cpic_status cpic_current_step(const cpic_ctx* c, int64_t* n)
{
    if (!c || !n) return CPIC_E_INVALID;
    *n = c->n;
    return CPIC_OK;
}
extern "C" cpic_status cpic_num_samples(const cpic_ctx* c, int32_t* n)
{
    if (!c || !n) return CPIC_E_INVALID;
    *n = (int32_t)c->samples.size();
    return CPIC_OK;
}

extern "C" cpic_status cpic_observables_full(cpic_ctx* c, double* out, int32_t cap)
{
    if (!c) return fail(nullptr, CPIC_E_INVALID, "cpic_observables: NULL context");
    const int ns = (int)c->samples.size();
    if (cap < ns) return fail(c, CPIC_E_CAPACITY, "cpic_observables: capacity " + std::to_string(cap) + " < " +
                                                      std::to_string(ns) + " samples");
    cpic_status s = reduce_samples(c);
    if (s) return s;
    const double* h = reinterpret_cast<const double*>(static_cast<char*>(c->h_stage) + 4 * sizeof(int));
    if (ns && out)
        HIPCHK(c, hipMemcpyAsync(const_cast<double*>(h), c->obs, sizeof(double) * 4 * (size_t)c->nslots,
                                 hipMemcpyDeviceToHost, c->st), "observables");
    s = cpic_sync(c);
    if (s) return s;
    if (!ns || !out) return CPIC_OK;
    const double inv = 1.0 / ((double)c->np * c->a_gev * c->a_gev);
    for (int k = 0; k < ns; k++) {
        const int slot = c->samples[k].first;
        out[6 * k + 0] = (c->samples[k].second + 1) * c->sc.dt * c->a_fm;
        for (int j = 0; j < 4; j++) out[6 * k + 1 + j] = h[4 * (size_t)slot + j] * inv;
        out[6 * k + 5] = (double)c->np;
    }
    return CPIC_OK;
}

// Central differences of a broadening series that opens with zeros at the
// formation time: rows (tau_mid, d/dtau of the four means, tau_k, the two
// ratios of columns 1/0 and 1/3), as documented at cpic_transport.
static void transport_rows(double tau_form, int ns, const double* tau, const double* b, int stride, double* out)
{
    double t0 = tau_form, v0[4] = {0, 0, 0, 0};
    for (int k = 0; k < ns; k++) {
        const double t1 = tau[(size_t)k * stride], *v1 = b + (size_t)k * stride;
        double* o = out + 8 * (size_t)k;
        o[0] = 0.5 * (t0 + t1);
        for (int j = 0; j < 4; j++) o[1 + j] = (v1[j] - v0[j]) / (t1 - t0);
        o[5] = t1;
        o[6] = v1[1] / v1[0];
        o[7] = v1[1] / v1[3];
        t0 = t1;
        for (int j = 0; j < 4; j++) v0[j] = v1[j];
    }
}

extern "C" cpic_status cpic_transport(cpic_ctx* c, double* out, int32_t cap, int32_t* n_samples)
{
    if (!c) return fail(nullptr, CPIC_E_INVALID, "cpic_transport: NULL context");
    const int ns = (int)c->samples.size();
    if (n_samples) *n_samples = ns;
    if (cap < ns) return fail(c, CPIC_E_CAPACITY, "cpic_transport: capacity " + std::to_string(cap) + " < " +
                                                     std::to_string(ns) + " samples");
    std::vector<double> full(6 * (size_t)std::max(ns, 1));
    cpic_status s = cpic_observables_full(c, full.data(), ns);
    if (s) return s;
    if (!ns || !out) return CPIC_OK;
    transport_rows(c->sc.n_form * c->sc.dt * c->a_fm, ns, full.data(), full.data() + 1, 6, out);
    return CPIC_OK;
}

extern "C" cpic_status cpic_observables(cpic_ctx* c, double* tau_fm, double* dpT2, double* dpL2, int32_t cap)
{
    if (!c) return fail(nullptr, CPIC_E_INVALID, "cpic_observables: NULL context");
    const int ns = (int)c->samples.size();
    std::vector<double> full(6 * (size_t)std::max(ns, 1));
    cpic_status s = cpic_observables_full(c, full.data(), cap < ns ? cap : ns);
    if (s) return s;
    for (int k = 0; k < ns; k++) {
        if (tau_fm) tau_fm[k] = full[6 * k];
        if (dpT2) dpT2[k] = full[6 * k + 1];
        if (dpL2) dpL2[k] = full[6 * k + 2];
    }
    return CPIC_OK;
}

// the diagnostics columns of the current state into dout[0..9] (asynchronous;
// columns 8, 9 only with particles; without energies columns 2..5 stay 0)
static cpic_status enqueue_diagnostics(cpic_ctx* c, bool energies = true)
{
    int nb = 0;
    hipError_t e;
    if (c->nc == 2)
        e = c->prec == CPIC_FP64
                ? launch_su2_diag<double>(F2<double>(c, c->cur), c->N, c->sc.dt, c->n, c->dpart, c->dcap, &nb, c->st)
                : launch_su2_diag<float>(F2<float>(c, c->cur), c->N, c->sc.dt, c->n, c->dpart, c->dcap, &nb, c->st);
    else
        e = c->prec == CPIC_FP64
                ? launch_field_diag<double>(F<double>(c, c->cur), c->N, c->sc.dt, c->n, c->dpart, c->dcap, &nb, c->st,
                                            energies)
                : launch_field_diag<float>(F<float>(c, c->cur), c->N, c->sc.dt, c->n, c->dpart, c->dcap, &nb, c->st,
                                           energies);
    HIPCHK(c, e, "field diagnostics");
    HIPCHK(c, launch_reduce_rows(c->dpart, nb, 8, c->dout, c->st), "reduce");
    if (c->np > 0) {
        e = c->prec == CPIC_FP64 ? launch_part_diag<double>(P<double>(c), (int)c->np, c->q2ref, c->q3ref, c->dpart, c->st)
                                 : launch_part_diag<float>(P<float>(c), (int)c->np, c->q2ref, c->q3ref, c->dpart, c->st);
        HIPCHK(c, e, "particle diagnostics");
        HIPCHK(c, launch_reduce_rows(c->dpart, push_blocks((int)c->np, 1), 2, c->dout + 8, c->st), "reduce");
    }
    return CPIC_OK;
}

// the watchdog's check of the current state, or its baseline (asynchronous)
static cpic_status enqueue_watch(cpic_ctx* c, bool take_base)
{
    // the checks read the Gauss and unitarity columns and test every column
    // for a non-finite value: the energies are not needed
    cpic_status s = enqueue_diagnostics(c, false);
    if (s) return s;
    // the charges' Casimirs are kept by the rotation update (SU(3)); the
    // logarithm update lets them drift by design
    const bool casimir = c->np > 0 && c->nc == 3 && c->pp.color_update == CPIC_COLOR_ROTATE;
    HIPCHK(c, launch_watchdog(c->dout, c->d_watchbase, take_base, casimir, c->watch_thr, c->q2ref, c->n, c->d_watch,
                              c->d_watchv, c->st), "watchdog");
    return CPIC_OK;
}
cpic_status cpic::watch_prepare(cpic_ctx* c)
{
    if (c->watch_every <= 0 || !c->watch_base_due) return CPIC_OK;
    c->watch_base_due = false;
    return enqueue_watch(c, true);
}

extern "C" cpic_status cpic_set_watchdog(cpic_ctx* c, int32_t every, double max_unitarity, double max_gauss_drift,
                                         double max_casimir_drift)
{
    if (!c) return fail(nullptr, CPIC_E_INVALID, "cpic_set_watchdog: NULL context");
    if (every < 0 || !(max_unitarity > 0) || !(max_gauss_drift > 0) || !(max_casimir_drift > 0))
        return fail(c, CPIC_E_INVALID, "cpic_set_watchdog: every >= 0 and positive thresholds");
    c->watch_every = every;
    c->watch_thr[0] = max_unitarity;
    c->watch_thr[1] = max_gauss_drift;
    c->watch_thr[2] = max_casimir_drift;
    c->watch_base_due = true;
    return CPIC_OK;
}

extern "C" cpic_status cpic_diagnostics(cpic_ctx* c, double out[10])
{
    if (!c || !out) return fail(c, CPIC_E_INVALID, "cpic_diagnostics: NULL argument");
    if (!c->initialised) return fail(c, CPIC_E_INVALID, "cpic_diagnostics: no state");
    cpic_status s = enqueue_diagnostics(c);
    if (s) return s;
    double h[10] = {0};
    HIPCHK(c, hipStreamSynchronize(c->st), "diagnostics");
    HIPCHK(c, hipMemcpy(h, c->dout, sizeof(double) * (c->np > 0 ? 10 : 8), hipMemcpyDeviceToHost), "diagnostics");
    std::memcpy(out, h, sizeof(h));
    for (int k = 0; k < 10; k++)
        if (!std::isfinite(h[k])) return fail(c, CPIC_E_NAN, "cpic_diagnostics: non-finite value in column " + std::to_string(k));
    return CPIC_OK;
}

extern "C" cpic_status cpic_diagnostics_summary(cpic_ctx* c, double* gauss_l2, double* energy_lat,
                                                double* unitarity_max, double* casimir_max)
{
    double d[10];
    const cpic_status s = cpic_diagnostics(c, d);
    if (s) return s;
    if (gauss_l2) *gauss_l2 = std::sqrt(d[0]);
    if (energy_lat) *energy_lat = d[2] + d[3] + d[4] + d[5];
    if (unitarity_max) *unitarity_max = d[6];
    if (casimir_max) *casimir_max = c->np > 0 ? std::max(d[8], d[9]) : 0.0;
    return CPIC_OK;
}

// ------------------------------------------------------------------ state exchange
// algebra components and complex link entries per site and direction
static int ncomp(const cpic_ctx* c) { return c->nc == 2 ? 3 : 8; }
static int nlink(const cpic_ctx* c) { return c->nc == 2 ? 4 : 9; }
static size_t state_bytes(const cpic_ctx* c, int which)
{
    switch (which) {
    case CPIC_STATE_U: return sizeof(double) * 2 * 2 * nlink(c) * (size_t)c->V;
    case CPIC_STATE_PHI: case CPIC_STATE_PI: return sizeof(double) * ncomp(c) * (size_t)c->V;
    case CPIC_STATE_E: return sizeof(double) * 2 * ncomp(c) * (size_t)c->V;
    case CPIC_STATE_PARTICLES: return sizeof(double) * 20 * (size_t)c->np;
    case CPIC_STATE_PTAU: return c->nc == 3 && !c->is_static ? sizeof(double) * 2 * (size_t)c->np : 0;
    case CPIC_STATE_STEP: return sizeof(int64_t);
    case CPIC_STATE_JET_W: return c->jets ? sizeof(double) * 18 * (size_t)c->V : 0;
    case CPIC_STATE_JET_F: return c->jets ? sizeof(double) * 24 * (size_t)c->V : 0;
    default: return 0;
    }
}

// device SoA (type T) <-> host interchange (double, site-major)
template <typename T> static void soa_to_host(const std::vector<T>& d, double* h, int which, int V)
{
    if (which == CPIC_STATE_U) {
        // the device keeps the first two rows of each link; the third is their
        // conjugate cross product, formed here as the kernels form it
        for (int i = 0; i < 2; i++)
            for (int s = 0; s < V; s++) {
                double* m = h + ((size_t)i * V + s) * 18;
                for (int c = 0; c < 12; c++) m[c] = (double)d[((size_t)i * 18 + c) * V + s];
                for (int j = 0; j < 3; j++) {
                    const int j1 = (j + 1) % 3, j2 = (j + 2) % 3;
                    const double* a = m + 2 * j1; const double* b = m + 6 + 2 * j2;  // r1[j1], r2[j2]
                    const double* e = m + 2 * j2; const double* f = m + 6 + 2 * j1;  // r1[j2], r2[j1]
                    const double pre = a[0] * b[0] - a[1] * b[1], pim = a[0] * b[1] + a[1] * b[0];
                    const double qre = e[0] * f[0] - e[1] * f[1], qim = e[0] * f[1] + e[1] * f[0];
                    m[12 + 2 * j] = pre - qre;
                    m[13 + 2 * j] = qim - pim;
                }
            }
    } else {
        const int blocks = which == CPIC_STATE_E ? 2 : 1;
        for (int i = 0; i < blocks; i++)
            for (int s = 0; s < V; s++)
                for (int a = 0; a < 8; a++) h[((size_t)i * V + s) * 8 + a] = (double)d[((size_t)i * 8 + a) * V + s];
    }
}
template <typename T> static void host_to_soa(const double* h, std::vector<T>& d, int which, int V)
{
    if (which == CPIC_STATE_U) {
        for (int i = 0; i < 2; i++)
            for (int s = 0; s < V; s++)
                for (int c = 0; c < 18; c++) d[((size_t)i * 18 + c) * V + s] = (T)h[((size_t)i * V + s) * 18 + c];
    } else {
        const int blocks = which == CPIC_STATE_E ? 2 : 1;
        for (int i = 0; i < blocks; i++)
            for (int s = 0; s < V; s++)
                for (int a = 0; a < 8; a++) d[((size_t)i * 8 + a) * V + s] = (T)h[((size_t)i * V + s) * 8 + a];
    }
}
static size_t field_offset(int which, int V)
{
    switch (which) {
    case CPIC_STATE_U: return 0;
    case CPIC_STATE_PHI: return 36 * (size_t)V;
    case CPIC_STATE_E: return 44 * (size_t)V;
    default: return 60 * (size_t)V;  // PI
    }
}
// SU(2) buffer set: U [2][4][V] quaternions (w, a1, a2, a3) for
// U = w + i a.sigma = [[w + i a3, a2 + i a1], [-a2 + i a1, w - i a3]];
// phi [3][V], E [2][3][V], pi [3][V]
static size_t field_offset2(int which, int V)
{
    switch (which) {
    case CPIC_STATE_U: return 0;
    case CPIC_STATE_PHI: return 8 * (size_t)V;
    case CPIC_STATE_E: return 11 * (size_t)V;
    default: return 17 * (size_t)V;
    }
}
template <typename T> static void su2_to_host(const std::vector<T>& d, double* h, int which, int V)
{
    if (which == CPIC_STATE_U) {
        for (int i = 0; i < 2; i++)
            for (int s = 0; s < V; s++) {
                const double w = d[((size_t)i * 4 + 0) * V + s], a1 = d[((size_t)i * 4 + 1) * V + s],
                             a2 = d[((size_t)i * 4 + 2) * V + s], a3 = d[((size_t)i * 4 + 3) * V + s];
                double* m = h + ((size_t)i * V + s) * 8;  // 2x2 complex, row-major, re/im
                m[0] = w;   m[1] = a3;
                m[2] = a2;  m[3] = a1;
                m[4] = -a2; m[5] = a1;
                m[6] = w;   m[7] = -a3;
            }
    } else {
        const int blocks = which == CPIC_STATE_E ? 2 : 1;
        for (int i = 0; i < blocks; i++)
            for (int s = 0; s < V; s++)
                for (int a = 0; a < 3; a++) h[((size_t)i * V + s) * 3 + a] = (double)d[((size_t)i * 3 + a) * V + s];
    }
}
template <typename T> static void host_to_su2(const double* h, std::vector<T>& d, int which, int V)
{
    if (which == CPIC_STATE_U) {
        for (int i = 0; i < 2; i++)
            for (int s = 0; s < V; s++) {
                const double* m = h + ((size_t)i * V + s) * 8;
                d[((size_t)i * 4 + 0) * V + s] = (T)m[0];
                d[((size_t)i * 4 + 1) * V + s] = (T)m[3];
                d[((size_t)i * 4 + 2) * V + s] = (T)m[2];
                d[((size_t)i * 4 + 3) * V + s] = (T)m[1];
            }
    } else {
        const int blocks = which == CPIC_STATE_E ? 2 : 1;
        for (int i = 0; i < blocks; i++)
            for (int s = 0; s < V; s++)
                for (int a = 0; a < 3; a++) d[((size_t)i * 3 + a) * V + s] = (T)h[((size_t)i * V + s) * 3 + a];
    }
}
// interchange particle columns: x y eta px py peta Q1..Q8 cx cy deta ux0 uy0 pt0
static const int kXchgToDev[20] = {PX_, PY_, PETA_, PPX, PPY, PPETA, PQ0, PQ0 + 1, PQ0 + 2, PQ0 + 3, PQ0 + 4,
                                   PQ0 + 5, PQ0 + 6, PQ0 + 7, -1, -2, PDETA, PUX0, PUY0, PPT0};

template <typename T> static cpic_status get_t(cpic_ctx* c, int which, double* h)
{
    if (which == CPIC_STATE_JET_W || which == CPIC_STATE_JET_F) {
        const int nc = which == CPIC_STATE_JET_W ? 18 : 24;
        std::vector<T> d((size_t)nc * c->V);
        HIPCHK(c, hipMemcpy(d.data(), which == CPIC_STATE_JET_W ? c->jW : c->jF, sizeof(T) * d.size(),
                            hipMemcpyDeviceToHost), "get paths");
        for (int s = 0; s < c->V; s++)
            for (int k = 0; k < nc; k++) h[(size_t)s * nc + k] = (double)d[(size_t)k * c->V + s];
        return CPIC_OK;
    }
    if (which == CPIC_STATE_PTAU) {
        // p^tau from the constraint at step n beside the integrated value
        const size_t np = c->np;
        std::vector<T> r(kPartReals * np);
        std::vector<int> pid(np);
        HIPCHK(c, hipMemcpy(r.data(), c->pr, sizeof(T) * r.size(), hipMemcpyDeviceToHost), "get p^tau");
        HIPCHK(c, hipMemcpy(pid.data(), c->pid, sizeof(int) * np, hipMemcpyDeviceToHost), "get p^tau");
        const double t = c->n * c->sc.dt;
        for (size_t p = 0; p < np; p++) {
            const size_t row = (size_t)pid[p];
            if (row >= np) return fail(c, CPIC_E_INVALID, "get_state: corrupt particle index");
            const double px = r[PPX * np + p], py = r[PPY * np + p], pe = r[PPETA * np + p];
            h[2 * row] = std::sqrt(px * px + py * py + (t * pe) * (t * pe) + c->mhat * c->mhat);
            h[2 * row + 1] = (double)r[(size_t)PPTAU * np + p];
        }
        return CPIC_OK;
    }
    if (which == CPIC_STATE_PARTICLES) {
        const size_t np = c->np;
        std::vector<T> r(kPartReals * np);
        std::vector<int> cell(2 * np), pid(np);
        HIPCHK(c, hipMemcpy(r.data(), c->pr, sizeof(T) * r.size(), hipMemcpyDeviceToHost), "get particles");
        HIPCHK(c, hipMemcpy(cell.data(), c->pcell, sizeof(int) * cell.size(), hipMemcpyDeviceToHost), "get particles");
        HIPCHK(c, hipMemcpy(pid.data(), c->pid, sizeof(int) * np, hipMemcpyDeviceToHost), "get particles");
        for (size_t p = 0; p < np; p++) {
            const size_t row = (size_t)pid[p];
            if (row >= np) return fail(c, CPIC_E_INVALID, "get_state: corrupt particle index");
            for (int k = 0; k < 20; k++) {
                const int d = kXchgToDev[k];
                h[row * 20 + k] = d >= 0 ? (double)r[(size_t)d * np + p] : (double)cell[(size_t)(-d - 1) * np + p];
            }
        }
        return CPIC_OK;
    }
    if (c->nc == 2) {
        const size_t cnt = which == CPIC_STATE_U ? 8 : (which == CPIC_STATE_E ? 6 : 3);
        std::vector<T> d(cnt * c->V);
        const T* src = static_cast<const T*>(c->fbuf[c->cur]) + field_offset2(which, c->V);
        HIPCHK(c, hipMemcpy(d.data(), src, sizeof(T) * d.size(), hipMemcpyDeviceToHost), "get state");
        su2_to_host(d, h, which, c->V);
        return CPIC_OK;
    }
    const size_t cnt = which == CPIC_STATE_U ? 36 : (which == CPIC_STATE_E ? 16 : 8);
    std::vector<T> d(cnt * c->V);
    const T* src = static_cast<const T*>(c->fbuf[c->cur]) + field_offset(which, c->V);
    HIPCHK(c, hipMemcpy(d.data(), src, sizeof(T) * d.size(), hipMemcpyDeviceToHost), "get state");
    soa_to_host(d, h, which, c->V);
    return CPIC_OK;
}
template <typename T> static cpic_status set_t(cpic_ctx* c, int which, const double* h)
{
    if (which == CPIC_STATE_PARTICLES) {
        const size_t np = c->np;
        std::vector<T> r(kPartReals * np);
        std::vector<int> cell(2 * np);
        for (size_t p = 0; p < np; p++)
            for (int k = 0; k < 20; k++) {
                const int d = kXchgToDev[k];
                if (d >= 0) r[(size_t)d * np + p] = (T)h[p * 20 + k];
                else cell[(size_t)(-d - 1) * np + p] = (int)h[p * 20 + k];
            }
        // the integrated p^tau restarts from the constraint at the current step
        const double t = c->n * c->sc.dt;
        for (size_t p = 0; p < np; p++) {
            const double px = h[p * 20 + 3], py = h[p * 20 + 4], pe = h[p * 20 + 5];
            r[(size_t)PPTAU * np + p] = (T)std::sqrt(px * px + py * py + (t * pe) * (t * pe) + c->mhat * c->mhat);
        }
        HIPCHK(c, hipMemcpy(c->pr, r.data(), sizeof(T) * r.size(), hipMemcpyHostToDevice), "set particles");
        HIPCHK(c, hipMemcpy(c->pcell, cell.data(), sizeof(int) * cell.size(), hipMemcpyHostToDevice), "set particles");
        return reset_pid(c);
    }
    if (c->nc == 2) {
        const size_t cnt = which == CPIC_STATE_U ? 8 : (which == CPIC_STATE_E ? 6 : 3);
        std::vector<T> d(cnt * c->V);
        host_to_su2(h, d, which, c->V);
        T* dst = static_cast<T*>(c->fbuf[c->cur]) + field_offset2(which, c->V);
        HIPCHK(c, hipMemcpy(dst, d.data(), sizeof(T) * d.size(), hipMemcpyHostToDevice), "set state");
        return CPIC_OK;
    }
    const size_t cnt = which == CPIC_STATE_U ? 36 : (which == CPIC_STATE_E ? 16 : 8);
    std::vector<T> d(cnt * c->V);
    host_to_soa(h, d, which, c->V);
    T* dst = static_cast<T*>(c->fbuf[c->cur]) + field_offset(which, c->V);
    HIPCHK(c, hipMemcpy(dst, d.data(), sizeof(T) * d.size(), hipMemcpyHostToDevice), "set state");
    return CPIC_OK;
}

extern "C" cpic_status cpic_get_state(cpic_ctx* c, int32_t which, void* dst, size_t bytes)
{
    if (!c || !dst) return fail(c, CPIC_E_INVALID, "cpic_get_state: NULL argument");
    const size_t need = state_bytes(c, which);
    if (!need && which != CPIC_STATE_PARTICLES)
        return fail(c, CPIC_E_INVALID,
                    "cpic_get_state: unknown part (light-like paths not enabled, or p^tau without moving SU(3) particles)");
    if (bytes != need) return fail(c, CPIC_E_CAPACITY, "cpic_get_state: expected " + std::to_string(need) + " bytes");
    HIPCHK(c, hipStreamSynchronize(c->st), "get state");
    if (which == CPIC_STATE_STEP) {
        const int64_t n = c->n;
        std::memcpy(dst, &n, sizeof n);
        return CPIC_OK;
    }
    if (which == CPIC_STATE_PARTICLES && c->np == 0) return CPIC_OK;
    return c->prec == CPIC_FP64 ? get_t<double>(c, which, (double*)dst) : get_t<float>(c, which, (double*)dst);
}

extern "C" cpic_status cpic_set_state(cpic_ctx* c, int32_t which, const void* src, size_t bytes)
{
    if (!c || !src) return fail(c, CPIC_E_INVALID, "cpic_set_state: NULL argument");
    if (which == CPIC_STATE_JET_W || which == CPIC_STATE_JET_F || which == CPIC_STATE_PTAU)
        return fail(c, CPIC_E_INVALID, "cpic_set_state: the light-like paths and p^tau are read-only");
    const size_t need = state_bytes(c, which);
    if (!need && which != CPIC_STATE_PARTICLES) return fail(c, CPIC_E_INVALID, "cpic_set_state: unknown part");
    if (bytes != need) return fail(c, CPIC_E_CAPACITY, "cpic_set_state: expected " + std::to_string(need) + " bytes");
    HIPCHK(c, hipStreamSynchronize(c->st), "set state");
    if (which == CPIC_STATE_STEP) {
        int64_t n;
        std::memcpy(&n, src, sizeof n);
        if (n < 0 || n > c->sc.n_max) return fail(c, CPIC_E_INVALID, "cpic_set_state: step out of range");
        c->initialised = true;
        return reset_counters(c, (int)n);
    }
    if (which == CPIC_STATE_PARTICLES && c->np == 0) return CPIC_OK;
    if (which == CPIC_STATE_PARTICLES) {
        const double* h = (const double*)src;
        for (int64_t p = 0; p < c->np; p++) {
            const double cx = h[p * 20 + 14], cy = h[p * 20 + 15];
            if (!(cx >= 0 && cx < c->N && cy >= 0 && cy < c->N) || cx != std::floor(cx) || cy != std::floor(cy))
                return fail(c, CPIC_E_INVALID, "cpic_set_state: particle cell out of range");
            const double x = h[p * 20], y = h[p * 20 + 1];
            if (!(x >= 0 && x < c->N && y >= 0 && y < c->N))
                return fail(c, CPIC_E_INVALID, "cpic_set_state: particle position out of [0, N)");
        }
    }
    c->watch_base_due = true;  // the watchdog's baseline is the installed state
    return c->prec == CPIC_FP64 ? set_t<double>(c, which, (const double*)src) : set_t<float>(c, which, (const double*)src);
}

// ------------------------------------------------------------------ checkpoints
namespace {
struct CkptHeader {
    char magic[8];
    int32_t version, N, prec, n, cur_unused, nsamples;
    int64_t np;
    int32_t nslots, jets;  // jets: 1 if the light-like path section follows the particle section
    cpic_glasma_params gp;
    cpic_particle_params pp;
};
}

extern "C" cpic_status cpic_save(cpic_ctx* c, const char* path)
{
    if (!c || !path) return fail(c, CPIC_E_INVALID, "cpic_save: NULL argument");
    cpic_status rs = reduce_samples(c);
    if (rs) return rs;
    HIPCHK(c, hipStreamSynchronize(c->st), "save");
    CkptHeader h{};
    std::memcpy(h.magic, "CPICKPT1", 8);
    h.version = 2; h.N = c->N; h.prec = c->prec; h.n = c->n; h.nsamples = (int)c->samples.size();
    h.np = c->np; h.nslots = c->nslots; h.gp = c->gp; h.pp = c->pp; h.jets = c->jets;
    const size_t fb = (size_t)c->rps * c->V * c->tsz, pb = (size_t)kPartReals * c->np * c->tsz;
    std::vector<char> f(fb), p(pb);
    std::vector<int> cell(2 * c->np), pid(c->np);
    std::vector<unsigned> keys;
    std::vector<double> obs(4 * (size_t)c->nslots);
    HIPCHK(c, hipMemcpy(f.data(), c->fbuf[c->cur], fb, hipMemcpyDeviceToHost), "save");
    if (pb) {
        HIPCHK(c, hipMemcpy(p.data(), c->pr, pb, hipMemcpyDeviceToHost), "save");
        HIPCHK(c, hipMemcpy(cell.data(), c->pcell, sizeof(int) * cell.size(), hipMemcpyDeviceToHost), "save");
        HIPCHK(c, hipMemcpy(pid.data(), c->pid, sizeof(int) * pid.size(), hipMemcpyDeviceToHost), "save");
        if (fused_shape(c->sort_tx, c->sort_ty)) {
            keys.resize(c->np);
            HIPCHK(c, hipMemcpy(keys.data(), c->sb.keys2, sizeof(unsigned) * keys.size(), hipMemcpyDeviceToHost), "save");
        }
    }
    if (!obs.empty()) HIPCHK(c, hipMemcpy(obs.data(), c->obs, sizeof(double) * obs.size(), hipMemcpyDeviceToHost), "save");
    const size_t jwb = c->jets ? (size_t)18 * c->V * c->tsz : 0, jfb = c->jets ? (size_t)24 * c->V * c->tsz : 0;
    std::vector<char> jw(jwb), jf(jfb);
    std::vector<double> jobs(c->jets ? 4 * (size_t)c->jslots : 0);
    if (c->jets) {
        HIPCHK(c, hipMemcpy(jw.data(), c->jW, jwb, hipMemcpyDeviceToHost), "save");
        HIPCHK(c, hipMemcpy(jf.data(), c->jF, jfb, hipMemcpyDeviceToHost), "save");
        if (!jobs.empty())
            HIPCHK(c, hipMemcpy(jobs.data(), c->jobs, sizeof(double) * jobs.size(), hipMemcpyDeviceToHost), "save");
    }
    FILE* fp = std::fopen(path, "wb");
    if (!fp) return fail(c, CPIC_E_IO, std::string("cpic_save: cannot open ") + path);
    bool ok = std::fwrite(&h, sizeof h, 1, fp) == 1;
    for (auto& sm : c->samples) {
        const int32_t v[2] = {sm.first, sm.second};
        ok = ok && std::fwrite(v, sizeof v, 1, fp) == 1;
    }
    ok = ok && std::fwrite(f.data(), 1, fb, fp) == fb;
    if (pb) {
        ok = ok && std::fwrite(p.data(), 1, pb, fp) == pb;
        ok = ok && std::fwrite(cell.data(), sizeof(int), cell.size(), fp) == cell.size();
        ok = ok && std::fwrite(pid.data(), sizeof(int), pid.size(), fp) == pid.size();
        const int32_t ss = c->static_sorted;
        ok = ok && std::fwrite(&ss, sizeof ss, 1, fp) == 1;
        const int32_t order[2] = {fused_shape(c->sort_tx, c->sort_ty) ? c->sort_tx : 0, c->sort_ty};
        ok = ok && std::fwrite(order, sizeof order, 1, fp) == 1;
        if (order[0] > 0) ok = ok && std::fwrite(keys.data(), sizeof(unsigned), keys.size(), fp) == keys.size();
    }
    if (!obs.empty()) ok = ok && std::fwrite(obs.data(), sizeof(double), obs.size(), fp) == obs.size();
    if (c->jets) {
        const double xo = c->ja.x_off;
        const int32_t jh[4] = {c->ja.stride, c->ja.sc.n_form, c->jslots, (int32_t)c->jsamples.size()};
        ok = ok && std::fwrite(&xo, sizeof xo, 1, fp) == 1 && std::fwrite(jh, sizeof jh, 1, fp) == 1;
        for (auto& sm : c->jsamples) {
            const int32_t v[2] = {sm.first, sm.second};
            ok = ok && std::fwrite(v, sizeof v, 1, fp) == 1;
        }
        ok = ok && std::fwrite(jw.data(), 1, jwb, fp) == jwb && std::fwrite(jf.data(), 1, jfb, fp) == jfb;
        if (!jobs.empty()) ok = ok && std::fwrite(jobs.data(), sizeof(double), jobs.size(), fp) == jobs.size();
    }
    ok = (std::fclose(fp) == 0) && ok;
    if (!ok) return fail(c, CPIC_E_IO, std::string("cpic_save: write failed for ") + path);
    return CPIC_OK;
}

extern "C" cpic_status cpic_load(cpic_ctx* c, const char* path)
{
    if (!c || !path) return fail(c, CPIC_E_INVALID, "cpic_load: NULL argument");
    FILE* fp = std::fopen(path, "rb");
    if (!fp) return fail(c, CPIC_E_IO, std::string("cpic_load: cannot open ") + path);
    CkptHeader h{};
    bool ok = std::fread(&h, sizeof h, 1, fp) == 1 && std::memcmp(h.magic, "CPICKPT1", 8) == 0 &&
              (h.version == 1 || h.version == 2);
    if (ok && (h.N != c->N || h.prec != c->prec || h.np != c->np || h.nslots != c->nslots || h.nsamples < 0 ||
               h.nsamples > c->nslots || h.n < 0 || h.n > c->sc.n_max || (h.jets != 0) != c->jets ||
               (h.gp.n_colors == 2 ? 2 : 3) != c->nc)) {
        std::fclose(fp);
        return fail(c, CPIC_E_INVALID, "cpic_load: checkpoint does not match this context");
    }
    std::vector<std::pair<int, int>> samples;
    for (int k = 0; ok && k < h.nsamples; k++) {
        int32_t v[2];
        ok = std::fread(v, sizeof v, 1, fp) == 1 && v[0] >= 0 && v[0] < c->nslots;
        samples.push_back({v[0], v[1]});
    }
    const size_t fb = (size_t)c->rps * c->V * c->tsz, pb = (size_t)kPartReals * c->np * c->tsz;
    std::vector<char> f(fb), p(pb);
    std::vector<int> cell(2 * c->np), pid(c->np);
    std::vector<double> obs(4 * (size_t)c->nslots);
    int32_t ss = 0, order[2] = {0, 0};
    std::vector<unsigned> keys;
    ok = ok && std::fread(f.data(), 1, fb, fp) == fb;
    if (pb) {
        ok = ok && std::fread(p.data(), 1, pb, fp) == pb;
        ok = ok && std::fread(cell.data(), sizeof(int), cell.size(), fp) == cell.size();
        ok = ok && std::fread(pid.data(), sizeof(int), pid.size(), fp) == pid.size();
        ok = ok && std::fread(&ss, sizeof ss, 1, fp) == 1;
        // version 2: the cell tiles of the record order and, for a fused-step
        // order, the sorted keys (from which the tile ranges follow)
        if (ok && h.version >= 2) {
            ok = std::fread(order, sizeof order, 1, fp) == 1;
            if (ok && order[0] > 0) {
                ok = fused_shape(order[0], order[1]);
                keys.resize(c->np);
                ok = ok && std::fread(keys.data(), sizeof(unsigned), keys.size(), fp) == keys.size();
                const unsigned bound = (unsigned)fused_tiles(c->N, order[0], order[1]) * (unsigned)(order[0] * order[1]);
                for (size_t k = 0; ok && k < keys.size(); k++) ok = keys[k] < bound && (k == 0 || keys[k - 1] <= keys[k]);
            }
        }
    }
    if (!obs.empty()) ok = ok && std::fread(obs.data(), sizeof(double), obs.size(), fp) == obs.size();
    const size_t jwb = c->jets ? (size_t)18 * c->V * c->tsz : 0, jfb = c->jets ? (size_t)24 * c->V * c->tsz : 0;
    std::vector<char> jw(jwb), jf(jfb);
    std::vector<double> jobs(c->jets ? 4 * (size_t)c->jslots : 0);
    std::vector<std::pair<int, int>> jsamples;
    bool jmatch = true;
    if (ok && c->jets) {
        double xo = 0;
        int32_t jh[4] = {0, 0, 0, 0};
        ok = std::fread(&xo, sizeof xo, 1, fp) == 1 && std::fread(jh, sizeof jh, 1, fp) == 1;
        jmatch = xo == c->ja.x_off && jh[0] == c->ja.stride && jh[1] == c->ja.sc.n_form && jh[2] == c->jslots &&
                 jh[3] >= 0 && jh[3] <= c->jslots;
        for (int k = 0; ok && jmatch && k < jh[3]; k++) {
            int32_t v[2];
            ok = std::fread(v, sizeof v, 1, fp) == 1 && v[0] >= 0 && v[0] < c->jslots;
            jsamples.push_back({v[0], v[1]});
        }
        if (jmatch) {
            ok = ok && std::fread(jw.data(), 1, jwb, fp) == jwb && std::fread(jf.data(), 1, jfb, fp) == jfb;
            if (!jobs.empty()) ok = ok && std::fread(jobs.data(), sizeof(double), jobs.size(), fp) == jobs.size();
        }
    }
    std::fclose(fp);
    if (!jmatch) return fail(c, CPIC_E_INVALID, "cpic_load: light-like path parameters differ from the checkpoint's");
    if (!ok) return fail(c, CPIC_E_IO, std::string("cpic_load: truncated or corrupt checkpoint ") + path);
    for (int v : cell)
        if (v < 0 || v >= c->N) return fail(c, CPIC_E_IO, "cpic_load: corrupt particle cells");
    {
        std::vector<char> seen(c->np, 0);
        for (int v : pid) {
            if (v < 0 || v >= c->np || seen[v]) return fail(c, CPIC_E_IO, "cpic_load: corrupt particle indices");
            seen[v] = 1;
        }
    }
    HIPCHK(c, hipStreamSynchronize(c->st), "load");
    c->cur = 0;
    HIPCHK(c, hipMemcpy(c->fbuf[0], f.data(), fb, hipMemcpyHostToDevice), "load");
    if (pb) {
        HIPCHK(c, hipMemcpy(c->pr, p.data(), pb, hipMemcpyHostToDevice), "load");
        HIPCHK(c, hipMemcpy(c->pcell, cell.data(), sizeof(int) * cell.size(), hipMemcpyHostToDevice), "load");
        HIPCHK(c, hipMemcpy(c->pid, pid.data(), sizeof(int) * pid.size(), hipMemcpyHostToDevice), "load");
        c->static_sorted = ss != 0;
        c->sorted_at = -1;
        c->sort_tx = c->sort_ty = 0;
        if (order[0] > 0 && c->tile_start) {
            // the fused step's tile order of the records: its ranges again
            HIPCHK(c, hipMemcpy(c->sb.keys2, keys.data(), sizeof(unsigned) * keys.size(), hipMemcpyHostToDevice), "load");
            HIPCHK(c, launch_tile_start(c->sb.keys2, (int)c->np, c->N, order[0], order[1], c->tile_start, c->st), "load");
            c->sort_tx = order[0];
            c->sort_ty = order[1];
        }
    }
    c->n = h.n;
    c->watch_base_due = true;
    HIPCHK(c, hipMemcpy(c->d_step, &c->n, sizeof(int), hipMemcpyHostToDevice), "load");
    if (!obs.empty()) HIPCHK(c, hipMemcpy(c->obs, obs.data(), sizeof(double) * obs.size(), hipMemcpyHostToDevice), "load");
    c->samples = samples;
    c->sample_groups.assign(samples.size(), obs_groups((int)c->np));  // already summed into obs
    c->obs_reduced = (int)samples.size();
    if (c->jets) {
        HIPCHK(c, hipMemcpy(c->jW, jw.data(), jwb, hipMemcpyHostToDevice), "load");
        HIPCHK(c, hipMemcpy(c->jF, jf.data(), jfb, hipMemcpyHostToDevice), "load");
        if (!jobs.empty())
            HIPCHK(c, hipMemcpy(c->jobs, jobs.data(), sizeof(double) * jobs.size(), hipMemcpyHostToDevice), "load");
        c->jsamples = jsamples;
        c->jobs_reduced = (int)jsamples.size();
    }
    c->initialised = true;
    return CPIC_OK;
}

// ------------------------------------------------------------------ tuning and timing
extern "C" cpic_status cpic_set_launch(cpic_ctx* c, int32_t bx, int32_t by, int32_t remap, int32_t waves,
                                       int32_t variant)
{
    if (!c) return fail(nullptr, CPIC_E_INVALID, "cpic_set_launch: NULL context");
    if (c->nc == 2) return fail(c, CPIC_E_INVALID, "cpic_set_launch: the SU(2) variant has one launch shape");
    if (variant == 1) {
        if (bx <= 0 || by <= 0 || bx * by != 128 || bx % 32 != 0)
            return fail(c, CPIC_E_INVALID, "cpic_set_launch: link-parallel tiles hold 128 sites, bx a multiple of 32");
        if (waves < 1 || waves > 3) return fail(c, CPIC_E_INVALID, "cpic_set_launch: waves must be 1..3");
    } else if (variant == 2) {
        const bool shape = (bx == 64 && by == 4) || (bx == 32 && by == 4) || (bx == 64 && by == 2) ||
                           (bx == 32 && by == 8) || (bx == 16 && by == 8);
        if (!shape) return fail(c, CPIC_E_INVALID, "cpic_set_launch: LDS tiles are 64x4, 32x4, 64x2, 32x8 or 16x8");
        if (waves != 1) return fail(c, CPIC_E_INVALID, "cpic_set_launch: LDS tiles take waves = 1");
    } else if (variant == 3) {
        const bool shape = (bx == 64 && by == 4) || (bx == 32 && by == 8) || (bx == 16 && by == 16) ||
                           (bx == 32 && by == 4) || (bx == 64 && by == 8);
        if (!shape)
            return fail(c, CPIC_E_INVALID, "cpic_set_launch: compressed LDS tiles are 64x4, 32x8, 16x16, 32x4 or 64x8");
        if (waves != 1) return fail(c, CPIC_E_INVALID, "cpic_set_launch: LDS tiles take waves = 1");
    } else if (variant == 0) {
        if (bx <= 0 || by <= 0 || bx * by > 256 || (bx * by) % 64 != 0)
            return fail(c, CPIC_E_INVALID, "cpic_set_launch: need bx*by a multiple of 64 and <= 256");
    } else if (variant == 4) {
        if (!fused_ok(c))
            return fail(c, CPIC_E_INVALID,
                        "cpic_set_launch: the fused step needs SU(3) particles with the rotation colour update and no "
                        "light-like paths");
        if (!fused_shape(bx, by))
            return fail(c, CPIC_E_INVALID, "cpic_set_launch: fused tiles are 64x8, 32x8, 16x16 or 8x8");
        if (waves != 1) return fail(c, CPIC_E_INVALID, "cpic_set_launch: LDS tiles take waves = 1");
    } else {
        return fail(c, CPIC_E_INVALID, "cpic_set_launch: variant must be 0 .. 4");
    }
    if (waves < 1 || waves > 4) return fail(c, CPIC_E_INVALID, "cpic_set_launch: waves must be 1..4");
    c->cfg.split = variant;
    c->cfg.bx = bx;
    c->cfg.by = by;
    c->cfg.xcd_remap = remap ? 1 : 0;
    c->cfg.waves = waves;
    drop_graphs(c);
    return CPIC_OK;
}

extern "C" cpic_status cpic_set_store_policy(cpic_ctx* c, int32_t non_temporal)
{
    if (!c) return fail(nullptr, CPIC_E_INVALID, "cpic_set_store_policy: NULL context");
    if (non_temporal != 0 && non_temporal != 1)
        return fail(c, CPIC_E_INVALID, "cpic_set_store_policy: 0 (default stores) or 1 (non-temporal)");
    c->cfg.nt_store = non_temporal;
    drop_graphs(c);
    return CPIC_OK;
}

extern "C" cpic_status cpic_set_timing(cpic_ctx* c, int32_t enable)
{
    if (!c) return fail(nullptr, CPIC_E_INVALID, "cpic_set_timing: NULL context");
    cpic_status s = cpic_sync(c);
    if (s) return s;
    c->timing = enable != 0;
    c->t_field = c->t_push = c->t_jets = 0;
    c->k_field = c->k_push = c->k_jets = 0;
    if (c->d_strag_total) HIPCHK(c, hipMemset(c->d_strag_total, 0, sizeof(unsigned long long)), "timing");
    return CPIC_OK;
}

extern "C" cpic_status cpic_straggler_pushes(cpic_ctx* c, int64_t* n)
{
    if (!c || !n) return fail(c, CPIC_E_INVALID, "cpic_straggler_pushes: NULL argument");
    cpic_status s = cpic_sync(c);
    if (s) return s;
    unsigned long long v = 0;
    if (c->d_strag_total)
        HIPCHK(c, hipMemcpy(&v, c->d_strag_total, sizeof v, hipMemcpyDeviceToHost), "cpic_straggler_pushes");
    *n = (int64_t)v;
    return CPIC_OK;
}

extern "C" cpic_status cpic_timing(cpic_ctx* c, double* field_ms, double* push_ms, int64_t* n_field, int64_t* n_push)
{
    if (!c) return fail(nullptr, CPIC_E_INVALID, "cpic_timing: NULL context");
    cpic_status s = cpic_sync(c);
    if (s) return s;
    if (field_ms) *field_ms = c->t_field;
    if (push_ms) *push_ms = c->t_push;
    if (n_field) *n_field = c->k_field;
    if (n_push) *n_push = c->k_push;
    return CPIC_OK;
}

// ------------------------------------------------------------------ launch tuner
// Times candidate launch configurations in place on the current state: the
// field kernel reads the current buffer and writes the free one (the step is
// not advanced); the push runs on a saved copy of the particle records, which
// is restored after every trial.  The fastest configuration is kept.
static const char* const kVariantName[5] = {"site", "link", "tile", "ctile", "fused"};

template <typename T> static cpic_status tune_t(cpic_ctx* c, int reps, std::string& rep)
{
    // the trial pushes may count cell jumps: the counter is put back afterwards
    int err0 = 0;
    HIPCHK(c, hipMemcpy(&err0, c->d_err, sizeof(int), hipMemcpyDeviceToHost), "tune");
    const LaunchCfg orig = c->cfg;  // the configuration before tuning (default or set by the caller)
    const Fields<T> A = F<T>(c, c->cur), B = F<T>(c, c->cur ^ 1);
    T* const G = static_cast<T*>(c->gpl);
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0), "tune");
    HIPCHK(c, hipEventCreate(&e1), "tune");
    const int shapes[][2] = {{64, 4}, {64, 2}, {64, 1}, {128, 2}, {128, 1}, {256, 1}, {32, 8}, {32, 4}, {16, 16}};
    LaunchCfg best = c->cfg;
    double best_ms = 1e300;
    std::vector<std::pair<double, LaunchCfg>> timed;
    char line[160];
    std::vector<LaunchCfg> cands;
    for (const auto& sh : shapes)
        for (int waves = 1; waves <= 3; waves++)
            for (int remap = 0; remap <= 1; remap++) cands.push_back(LaunchCfg{sh[0], sh[1], remap, waves, 0});
    const int lshapes[][2] = {{128, 1}, {64, 2}, {32, 4}};
    for (const auto& sh : lshapes)
        for (int waves = 1; waves <= 3; waves++)
            for (int remap = 0; remap <= 1; remap++) cands.push_back(LaunchCfg{sh[0], sh[1], remap, waves, 1});
    const int tshapes[][2] = {{64, 4}, {32, 4}, {64, 2}, {32, 8}, {16, 8}};
    for (const auto& sh : tshapes)
        for (int remap = 0; remap <= 1; remap++) cands.push_back(LaunchCfg{sh[0], sh[1], remap, 1, 2});
    const int cshapes[][2] = {{64, 4}, {32, 8}, {16, 16}, {32, 4}, {64, 8}};
    for (const auto& sh : cshapes)
        for (int remap = 0; remap <= 1; remap++) cands.push_back(LaunchCfg{sh[0], sh[1], remap, 1, 3});
    for (LaunchCfg& cfg : cands) cfg.nt_store = c->cfg.nt_store;
    for (const LaunchCfg& cfg : cands) {
                HIPCHK(c, launch_field_step<T>(A, B, G, c->N, c->sc, c->d_step, cfg, c->st), "tune");  // warm-up
                HIPCHK(c, hipEventRecord(e0, c->st), "tune");
                for (int r = 0; r < reps; r++)
                    HIPCHK(c, launch_field_step<T>(A, B, G, c->N, c->sc, c->d_step, cfg, c->st), "tune");
                HIPCHK(c, hipEventRecord(e1, c->st), "tune");
                HIPCHK(c, hipEventSynchronize(e1), "tune");
                float ms = 0;
                HIPCHK(c, hipEventElapsedTime(&ms, e0, e1), "tune");
                const double per = ms / reps;
                std::snprintf(line, sizeof line, "field %s bx=%d by=%d waves=%d remap=%d: %.2f us\n",
                              kVariantName[cfg.split], cfg.bx, cfg.by, cfg.waves, cfg.xcd_remap, per * 1e3);
                rep += line;
                if (per < best_ms) { best_ms = per; best = cfg; }
                timed.push_back({per, cfg});
            }
    c->cfg = best;
    std::snprintf(line, sizeof line, "best field: %s bx=%d by=%d waves=%d remap=%d %.2f us%s\n",
                  kVariantName[best.split], best.bx, best.by, best.waves, best.xcd_remap, best_ms * 1e3,
                  best.split == 3 && best.nt_store ? " (non-temporal stores of the new state)" : "");
    rep += line;
    const int lanes[4] = {1, 2, 4, 8};
    double lane_iso[4] = {1e300, 1e300, 1e300, 1e300};  // isolated push times per lane count
    const int tpp0 = c->tpp;                              // the lane count before tuning
    if (c->np > 0 && c->n >= c->sc.n_form && c->n < c->sc.n_max) {
        const size_t rb = sizeof(T) * kPartReals * (size_t)c->np, cb = sizeof(int) * 2 * (size_t)c->np;
        HIPCHK(c, hipMemcpyAsync(c->sb.r2, c->pr, rb, hipMemcpyDeviceToDevice, c->st), "tune");
        HIPCHK(c, hipMemcpyAsync(c->sb.cell2, c->pcell, cb, hipMemcpyDeviceToDevice, c->st), "tune");
        // the step's new momenta: run the field kernel once into the free buffer
        HIPCHK(c, launch_field_step<T>(A, B, G, c->N, c->sc, c->d_step, c->cfg, c->st), "tune");
        // the lane counts timed in interleaved rounds (the first a warm-up),
        // each by its median; the current count stays unless another is at
        // least 3 % faster (timing noise does not flip between equals)
        std::vector<double> times[4];
        for (int r = 0; r <= 2 * reps; r++)
            for (int k = 0; k < 4; k++) {
                HIPCHK(c, hipEventRecord(e0, c->st), "tune");
                HIPCHK(c, launch_push<T>(A, B, G, P<T>(c), push_args(c, lanes[k]), c->d_step, c->partials, c->d_err,
                                         c->st), "tune");
                HIPCHK(c, hipEventRecord(e1, c->st), "tune");
                HIPCHK(c, hipMemcpyAsync(c->pr, c->sb.r2, rb, hipMemcpyDeviceToDevice, c->st), "tune");
                HIPCHK(c, hipMemcpyAsync(c->pcell, c->sb.cell2, cb, hipMemcpyDeviceToDevice, c->st), "tune");
                HIPCHK(c, hipEventSynchronize(e1), "tune");
                float ms = 0;
                HIPCHK(c, hipEventElapsedTime(&ms, e0, e1), "tune");
                if (r > 0) times[k].push_back(ms);
            }
        int best_tpp = c->tpp;
        double best_p = 1e300, cur_p = 1e300;
        for (int k = 0; k < 4; k++) {
            std::sort(times[k].begin(), times[k].end());
            const double per = times[k][times[k].size() / 2];
            lane_iso[k] = per;
            std::snprintf(line, sizeof line, "push lanes=%d: %.2f us\n", lanes[k], per * 1e3);
            rep += line;
            if (per < best_p) { best_p = per; best_tpp = lanes[k]; }
            if (lanes[k] == c->tpp) cur_p = per;
        }
        if (cur_p <= 1.03 * best_p) { best_tpp = c->tpp; best_p = cur_p; }
        bool table = false;
        if (c->nc == 3 && c->pp.color_update == CPIC_COLOR_ROTATE) {
            if (!c->ftab) HIPCHK(c, hipMalloc(&c->ftab, (size_t)48 * c->V * c->tsz), "tune");
            double tot = 0;
            for (int r = 0; r <= reps; r++) {
                HIPCHK(c, hipEventRecord(e0, c->st), "tune");
                HIPCHK(c, launch_force_table<T>(A, B, G, static_cast<T*>(c->ftab), c->N, c->sc, c->is_static != 0,
                                                c->d_step, c->st), "tune");
                HIPCHK(c, launch_push_table<T>(A, B, static_cast<const T*>(c->ftab), P<T>(c), push_args(c, 1),
                                               c->d_step, c->partials, c->d_err, c->st), "tune");
                HIPCHK(c, hipEventRecord(e1, c->st), "tune");
                HIPCHK(c, hipMemcpyAsync(c->pr, c->sb.r2, rb, hipMemcpyDeviceToDevice, c->st), "tune");
                HIPCHK(c, hipMemcpyAsync(c->pcell, c->sb.cell2, cb, hipMemcpyDeviceToDevice, c->st), "tune");
                HIPCHK(c, hipEventSynchronize(e1), "tune");
                float ms = 0;
                HIPCHK(c, hipEventElapsedTime(&ms, e0, e1), "tune");
                if (r > 0) tot += ms;
            }
            const double per = tot / reps;
            std::snprintf(line, sizeof line, "push with force table: %.2f us\n", per * 1e3);
            rep += line;
            if (per < best_p) { best_p = per; table = true; }
        }
        HIPCHK(c, hipStreamSynchronize(c->st), "tune");
        HIPCHK(c, hipMemcpy(c->d_err, &err0, sizeof(int), hipMemcpyHostToDevice), "tune");
        // the trial pushes advanced the step counter: put it back
        HIPCHK(c, hipMemcpy(c->d_step, &c->n, sizeof(int), hipMemcpyHostToDevice), "tune");
        c->tpp = best_tpp;
        c->pblocks = push_blocks((int)c->np, c->tpp);
        c->push_table = table;
        set_store_policy(c);
        if (table) std::snprintf(line, sizeof line, "best push: force table %.2f us\n", best_p * 1e3);
        else std::snprintf(line, sizeof line, "best push: lanes=%d %.2f us\n", best_tpp, best_p * 1e3);
        rep += line;
    }
    // In the step: the field kernel shares the caches with the push and the
    // light-like paths, which the isolated timings above do not see.  The
    // three fastest field launches, each with both store policies, and the
    // fused step on its tile shapes run two real steps (both buffer
    // parities) from the current state, which is restored after every trial;
    // the fastest step pair decides.  A fused trial first reorders the
    // records by its tiles (a reordering changes no result).
    // (the fused step needs the records in the order of its tiles at every
    // push step: a trial pair must not run into the first push step, before
    // which the records are first ordered)
    const bool order_ok = !fused_ok(c) || c->n >= c->sc.n_form || c->n + 2 <= c->sc.n_form;
    if (!order_ok) rep += "step trials skipped: the first push step falls inside the trial steps\n";
    if (c->n + 2 <= c->sc.n_max && timed.size() > 0 && order_ok) {
        std::sort(timed.begin(), timed.end(),
                  [](const std::pair<double, LaunchCfg>& a, const std::pair<double, LaunchCfg>& b) { return a.first < b.first; });
        const size_t fbytes = (size_t)c->rps * c->V * c->tsz;
        const size_t rb = sizeof(T) * kPartReals * (size_t)c->np, cb = sizeof(int) * 2 * (size_t)c->np;
        const size_t wb = (size_t)18 * c->V * c->tsz, fb = (size_t)24 * c->V * c->tsz;
        void *bk = nullptr, *bw = nullptr, *bf = nullptr, *bp = nullptr, *bc = nullptr;
        hipError_t he = hipMalloc(&bk, fbytes);
        if (he == hipSuccess && c->jets) he = hipMalloc(&bw, wb);
        if (he == hipSuccess && c->jets) he = hipMalloc(&bf, fb);
        if (he == hipSuccess && c->np > 0) he = hipMalloc(&bp, rb);
        if (he == hipSuccess && c->np > 0) he = hipMalloc(&bc, cb);
        auto release = [&]() {
            (void)hipFree(bk); (void)hipFree(bw); (void)hipFree(bf); (void)hipFree(bp); (void)hipFree(bc);
        };
        if (he != hipSuccess) {
            release();
            rep += "step trials skipped: no memory for the state copy\n";
        } else {
            auto copy = [&](void* dst, const void* src, size_t bytes) {
                return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, c->st);
            };
            hipError_t te = copy(bk, c->fbuf[c->cur], fbytes);
            if (te == hipSuccess && c->np > 0) te = copy(bp, c->pr, rb);
            if (te == hipSuccess && c->np > 0) te = copy(bc, c->pcell, cb);
            if (te == hipSuccess && c->jets) te = copy(bw, c->jW, wb);
            if (te == hipSuccess && c->jets) te = copy(bf, c->jF, fb);
            auto restore = [&]() {
                hipError_t r = copy(c->fbuf[c->cur], bk, fbytes);
                if (r == hipSuccess && c->np > 0) r = copy(c->pr, bp, rb);
                if (r == hipSuccess && c->np > 0) r = copy(c->pcell, bc, cb);
                if (r == hipSuccess && c->jets) r = copy(c->jW, bw, wb);
                if (r == hipSuccess && c->jets) r = copy(c->jF, bf, fb);
                if (r == hipSuccess) r = hipStreamSynchronize(c->st);
                if (r == hipSuccess) r = hipMemcpy(c->d_step, &c->n, sizeof(int), hipMemcpyHostToDevice);
                if (r == hipSuccess) r = hipMemcpy(c->d_err, &err0, sizeof(int), hipMemcpyHostToDevice);
                return r;
            };
            const LaunchCfg keep = c->cfg;
            auto same = [](const LaunchCfg& a, const LaunchCfg& b) {
                return a.bx == b.bx && a.by == b.by && a.xcd_remap == b.xcd_remap && a.waves == b.waves &&
                       a.split == b.split && a.nt_store == b.nt_store;
            };
            // the trials: the three fastest in isolation with both store
            // policies, and the configuration before tuning
            std::vector<LaunchCfg> trials;
            const size_t ntop = std::min<size_t>(3, timed.size());
            for (size_t k = 0; k < ntop; k++)
                for (int nt = 0; nt <= 1; nt++) {
                    LaunchCfg cfg = timed[k].second;
                    if (cfg.split != 3 && nt == 1) continue;  // the store policy exists for the compressed tiles
                    cfg.nt_store = cfg.split == 3 ? nt : 0;
                    trials.push_back(cfg);
                }
            if (orig.split == 4 && fused_ok(c) && c->n >= c->sc.n_form) {  // from the tile push mode only
                const int shapes[3][2] = {{64, 8}, {32, 8}, {16, 16}}, small[2][2] = {{16, 16}, {8, 8}};
                const int ns = c->N >= 64 ? 3 : 2;
                for (int k = 0; k < ns; k++)
                    for (int nt = 0; nt <= 1; nt++) {
                        LaunchCfg cfg;
                        cfg.split = 4;
                        cfg.bx = c->N >= 64 ? shapes[k][0] : small[k][0];
                        cfg.by = c->N >= 64 ? shapes[k][1] : small[k][1];
                        cfg.xcd_remap = 1;
                        cfg.waves = 1;
                        cfg.nt_store = nt;
                        trials.push_back(cfg);
                    }
            }
            bool have_orig = false;
            for (const LaunchCfg& t : trials) have_orig = have_orig || same(t, orig);
            if (!have_orig) trials.push_back(orig);
            // two real steps from the saved state, per step (reps pairs after a warm-up pair)
            auto time_pair = [&](double& per) -> cpic_status {
                double tot = 0;
                for (int r = 0; r <= reps && te == hipSuccess; r++) {
                    te = hipEventRecord(e0, c->st);
                    cpic_status ls = CPIC_OK;
                    if (te == hipSuccess) ls = launch_one<T>(c, c->cur, false);
                    if (te == hipSuccess && !ls) ls = launch_one<T>(c, c->cur ^ 1, false);
                    if (ls) return ls;
                    if (te == hipSuccess) te = hipEventRecord(e1, c->st);
                    if (te == hipSuccess) te = hipEventSynchronize(e1);
                    float ms = 0;
                    if (te == hipSuccess) te = hipEventElapsedTime(&ms, e0, e1);
                    if (te == hipSuccess) te = restore();
                    if (r > 0) tot += ms;
                }
                per = tot / reps / 2;
                return CPIC_OK;
            };
            LaunchCfg best_step = keep;
            double best_pair = 1e300, orig_pair = 1e300;
            for (size_t k = 0; k < trials.size() && te == hipSuccess; k++) {
                {
                    const LaunchCfg cfg = trials[k];
                    c->cfg = cfg;
                    if (fused_active(c) && (c->sort_tx != cfg.bx || c->sort_ty != cfg.by)) {
                        // records in this trial's tile order, and the copy the
                        // trials restore taken again
                        cpic_status so = maybe_sort(c);
                        if (so) { c->cfg = keep; (void)restore(); release(); return so; }
                        te = copy(bp, c->pr, rb);
                        if (te == hipSuccess) te = copy(bc, c->pcell, cb);
                    }
                    double per = 0;
                    cpic_status ls = time_pair(per);
                    if (ls) { c->cfg = keep; (void)restore(); release(); return ls; }
                    if (te != hipSuccess) break;
                    std::snprintf(line, sizeof line, "step with field %s bx=%d by=%d waves=%d remap=%d nt=%d: %.2f us\n",
                                  kVariantName[cfg.split], cfg.bx, cfg.by, cfg.waves, cfg.xcd_remap, cfg.nt_store,
                                  per * 1e3);
                    rep += line;
                    if (per < best_pair) { best_pair = per; best_step = cfg; }
                    if (same(cfg, orig)) orig_pair = per;
                }
            }
            if (te != hipSuccess) { c->cfg = keep; release(); return hip_fail(c, te, "tune"); }
            // a change of configuration has to gain at least 2 % per step, so
            // that timing noise does not flip the choice between equals
            if (orig_pair <= 1.02 * best_pair) {
                best_step = orig;
                best_pair = orig_pair;
            }
            c->cfg = best_step;
            // the gather push's lane count in the step too (in isolation the
            // push misses what the field update leaves in the caches): the
            // counts within 10 % of the fastest in isolation and the count
            // before tuning, which stays unless another is at least 2 %
            // faster per step
            if (!fused_active(c) && !c->push_table && c->np > 0 && lane_iso[0] < 1e300) {
                const int cur_tpp = c->tpp;  // the field trials ran with it
                double step_t[4] = {1e300, 1e300, 1e300, 1e300};
                double best_iso = 1e300;
                for (int k = 0; k < 4; k++) {
                    best_iso = std::min(best_iso, lane_iso[k]);
                    if (lanes[k] == cur_tpp) step_t[k] = best_pair;
                }
                for (int k = 0; k < 4 && te == hipSuccess; k++) {
                    if (lanes[k] == cur_tpp || !(lane_iso[k] <= 1.10 * best_iso || lanes[k] == tpp0)) continue;
                    c->tpp = lanes[k];
                    c->pblocks = push_blocks((int)c->np, c->tpp);
                    cpic_status ls = time_pair(step_t[k]);
                    if (ls) { c->tpp = cur_tpp; c->pblocks = push_blocks((int)c->np, cur_tpp); (void)restore(); release(); return ls; }
                    std::snprintf(line, sizeof line, "step with push lanes=%d: %.2f us\n", lanes[k], step_t[k] * 1e3);
                    rep += line;
                }
                int pick = 0;
                for (int k = 1; k < 4; k++)
                    if (step_t[k] < step_t[pick]) pick = k;
                for (int k = 0; k < 4; k++)
                    if (lanes[k] == tpp0 && step_t[k] <= 1.02 * step_t[pick]) pick = k;
                c->tpp = lanes[pick];
                c->pblocks = push_blocks((int)c->np, c->tpp);
                best_pair = step_t[pick];
            }
            release();
            if (te != hipSuccess) { c->cfg = keep; return hip_fail(c, te, "tune"); }
            std::snprintf(line, sizeof line,
                          "chosen: field %s bx=%d by=%d waves=%d remap=%d nt=%d, push lanes=%d, step %.2f us\n",
                          kVariantName[best_step.split], best_step.bx, best_step.by, best_step.waves,
                          best_step.xcd_remap, best_step.nt_store, c->tpp, best_pair * 1e3);
            rep += line;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    drop_graphs(c);
    return CPIC_OK;
}

extern "C" cpic_status cpic_tune(cpic_ctx* c, int32_t reps, char* report, size_t cap)
{
    if (!c) return fail(nullptr, CPIC_E_INVALID, "cpic_tune: NULL context");
    if (!c->initialised) return fail(c, CPIC_E_INVALID, "cpic_tune: no state");
    if (reps < 1) reps = 1;
    if (c->timing) return fail(c, CPIC_E_INVALID, "cpic_tune: disable timing first");
    HIPCHK(c, hipStreamSynchronize(c->st), "tune");
    std::string rep;
    if (c->nc == 2) {
        rep = "SU(2): one launch shape (256 sites or particles per workgroup); nothing to tune\n";
    } else {
        cpic_status s = c->prec == CPIC_FP64 ? tune_t<double>(c, reps, rep) : tune_t<float>(c, reps, rep);
        if (s) return s;
    }
    if (report && cap) {
        std::strncpy(report, rep.c_str(), cap - 1);
        report[cap - 1] = 0;
    }
    return CPIC_OK;
}

extern "C" cpic_status cpic_get_launch(const cpic_ctx* c, int32_t out[7])
{
    if (!c || !out) return CPIC_E_INVALID;
    out[0] = c->cfg.bx; out[1] = c->cfg.by; out[2] = c->cfg.xcd_remap; out[3] = c->cfg.waves; out[4] = c->tpp;
    out[5] = c->cfg.split; out[6] = c->cfg.nt_store;
    return CPIC_OK;
}

extern "C" cpic_status cpic_set_push_lanes(cpic_ctx* c, int32_t lanes)
{
    if (!c) return fail(nullptr, CPIC_E_INVALID, "cpic_set_push_lanes: NULL context");
    if (lanes != 1 && lanes != 2 && lanes != 4 && lanes != 8)
        return fail(c, CPIC_E_INVALID, "cpic_set_push_lanes: 1, 2, 4 or 8");
    if (c->nc == 2 && lanes != 1) return fail(c, CPIC_E_INVALID, "cpic_set_push_lanes: the SU(2) push takes 1");
    HIPCHK(c, hipStreamSynchronize(c->st), "set push lanes");
    c->tpp = lanes;
    c->pblocks = c->np > 0 ? push_blocks((int)c->np, lanes) : 0;
    drop_graphs(c);
    return CPIC_OK;
}

// ------------------------------------------------------------------ light-like jet limit
extern "C" cpic_status cpic_jets_enable(cpic_ctx* c, const cpic_jet_params* jp)
{
    if (!c || !jp) return fail(c, CPIC_E_INVALID, "cpic_jets_enable: NULL argument");
    if (c->jets) return fail(c, CPIC_E_INVALID, "cpic_jets_enable: already enabled");
    if (c->nc == 2) return fail(c, CPIC_E_INVALID, "cpic_jets_enable: SU(3) only");
    if (!(jp->x_offset >= 0 && jp->x_offset < 1) || jp->stride < 1 || !(jp->tau_form_fm >= 0) ||
        (jp->rep != CPIC_REP_FUND && jp->rep != CPIC_REP_ADJ))
        return fail(c, CPIC_E_INVALID, "cpic_jets_enable: need 0 <= x_offset < 1, stride >= 1, tau_form >= 0, a valid rep");
    if (!(c->sc.dt <= 1))
        return fail(c, CPIC_E_INVALID, "cpic_jets_enable: needs dtau <= a (at most one cell per step)");
    const double dtau_fm = c->sc.dt * c->a_fm;
    const double f = jp->tau_form_fm / dtau_fm;
    if (!(f < 1e8)) return fail(c, CPIC_E_INVALID, "cpic_jets_enable: tau_form / dtau above 1e8 steps");
    const int n_form = std::min(c->sc.n_max, (int)std::ceil(f - 1e-9 * f));
    if (c->initialised && c->n > n_form)
        return fail(c, CPIC_E_INVALID, "cpic_jets_enable: the paths would form before the current step");
    HIPCHK(c, hipStreamSynchronize(c->st), "jets");
    JetArgs ja{};
    ja.N = c->N;
    ja.stride = jp->stride;
    ja.x_off = jp->x_offset;
    ja.sc = c->sc;
    ja.sc.n_form = n_form;
    const int jslots = num_slots(ja.sc);
    const size_t V = c->V;
    hipError_t e = hipSuccess;
    void *W = nullptr, *Fp = nullptr, *tab = nullptr;
    double *part = nullptr, *obs = nullptr;
    e = hipMalloc(&W, 18 * V * c->tsz);
    if (e == hipSuccess) e = hipMalloc(&Fp, 24 * V * c->tsz);
    if (e == hipSuccess && !c->ftab) e = hipMalloc(&tab, (size_t)48 * V * c->tsz);
    void* gpl = nullptr;
    if (e == hipSuccess && !c->gpl) e = hipMalloc(&gpl, (size_t)kPlaqReals * V * c->tsz);
    if (e == hipSuccess && jslots > 0) e = hipMalloc(&part, sizeof(double) * 4 * (size_t)jet_groups(c->V) * jslots);
    if (e == hipSuccess && jslots > 0) e = hipMalloc(&obs, sizeof(double) * 4 * (size_t)jslots);
    if (e == hipSuccess && obs) e = hipMemsetAsync(obs, 0, sizeof(double) * 4 * (size_t)jslots, c->st);
    if (e == hipSuccess) e = hipStreamSynchronize(c->st);
    if (e != hipSuccess) {
        (void)hipFree(W); (void)hipFree(Fp); (void)hipFree(tab); (void)hipFree(gpl); (void)hipFree(part);
        (void)hipFree(obs);
        const bool oom = e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation;
        return fail(c, oom ? CPIC_E_NOMEM : CPIC_E_HIP, std::string("cpic_jets_enable: ") + hipGetErrorString(e));
    }
    if (tab) c->ftab = tab;
    if (gpl) c->gpl = gpl;
    c->sc.n_plaq = std::min(c->sc.n_plaq, n_form);
    c->jW = W;
    c->jF = Fp;
    c->jpartials = part;
    c->jobs = obs;
    c->jslots = jslots;
    c->ja = ja;
    double q0[8], eig[3], q3 = 0;
    initial_colour(jp->rep, q0, eig, &c->jet_q2, &q3);
    c->jsamples.clear();
    c->jobs_reduced = 0;
    c->jets = true;
    if (c->cfg.split == 4) c->cfg.split = 3;  // the paths read the force table: a separate push
    set_store_policy(c);
    drop_graphs(c);
    return CPIC_OK;
}

extern "C" cpic_status cpic_jets_observables(cpic_ctx* c, double* out, int32_t cap, int32_t* n_samples)
{
    if (!c) return fail(nullptr, CPIC_E_INVALID, "cpic_jets_observables: NULL context");
    if (!c->jets) return fail(c, CPIC_E_INVALID, "cpic_jets_observables: light-like paths not enabled");
    const int ns = (int)c->jsamples.size();
    if (n_samples) *n_samples = ns;
    if (cap < ns) return fail(c, CPIC_E_CAPACITY, "cpic_jets_observables: capacity " + std::to_string(cap) + " < " +
                                                      std::to_string(ns) + " samples");
    cpic_status s = reduce_samples(c);
    if (s) return s;
    s = cpic_sync(c);
    if (s) return s;
    if (!ns || !out) return CPIC_OK;
    std::vector<double> h(4 * (size_t)c->jslots);
    HIPCHK(c, hipMemcpy(h.data(), c->jobs, sizeof(double) * h.size(), hipMemcpyDeviceToHost), "jets observables");
    const double scale = c->jet_q2 / 8.0 / ((double)c->V * c->a_gev * c->a_gev);
    for (int k = 0; k < ns; k++) {
        const int slot = c->jsamples[k].first;
        out[4 * k] = (c->jsamples[k].second + 1) * c->sc.dt * c->a_fm;
        for (int j = 0; j < 3; j++) out[4 * k + 1 + j] = h[4 * (size_t)slot + j] * scale;
    }
    return CPIC_OK;
}

extern "C" cpic_status cpic_jets_transport(cpic_ctx* c, double* out, int32_t cap, int32_t* n_samples)
{
    if (!c) return fail(nullptr, CPIC_E_INVALID, "cpic_jets_transport: NULL context");
    if (!c->jets) return fail(c, CPIC_E_INVALID, "cpic_jets_transport: light-like paths not enabled");
    const int ns = (int)c->jsamples.size();
    if (n_samples) *n_samples = ns;
    if (cap < ns) return fail(c, CPIC_E_CAPACITY, "cpic_jets_transport: capacity " + std::to_string(cap) + " < " +
                                                     std::to_string(ns) + " samples");
    std::vector<double> obs(4 * (size_t)std::max(ns, 1));
    cpic_status s = cpic_jets_observables(c, obs.data(), ns, nullptr);
    if (s) return s;
    if (!ns || !out) return CPIC_OK;
    // rows of (tau, <dp_x^2>, <dp_y^2>, <dp_z^2>) as (tau, T = x, L = z, par = x, perp = y)
    std::vector<double> series(6 * (size_t)ns);
    for (int k = 0; k < ns; k++) {
        const double* o = obs.data() + 4 * (size_t)k;
        double* r = series.data() + 6 * (size_t)k;
        r[0] = o[0];
        r[1] = o[1];
        r[2] = o[3];
        r[3] = o[1];
        r[4] = o[2];
        r[5] = 0;
    }
    std::vector<double> rows(8 * (size_t)ns);
    transport_rows(c->ja.sc.n_form * c->ja.sc.dt * c->a_fm, ns, series.data(), series.data() + 1, 6, rows.data());
    for (int k = 0; k < ns; k++) {
        const double* r = rows.data() + 8 * (size_t)k;
        double* o = out + 6 * (size_t)k;
        o[0] = r[0];   // tau_mid
        o[1] = r[3];   // qhat_x
        o[2] = r[4];   // qhat_y
        o[3] = r[2];   // qhat_z
        o[4] = r[5];   // tau_k
        o[5] = r[7];   // <dp_z^2>/<dp_y^2>
    }
    return CPIC_OK;
}

extern "C" cpic_status cpic_jets_timing(cpic_ctx* c, double* ms, int64_t* launches)
{
    if (!c) return fail(nullptr, CPIC_E_INVALID, "cpic_jets_timing: NULL context");
    cpic_status s = cpic_sync(c);
    if (s) return s;
    if (ms) *ms = c->t_jets;
    if (launches) *launches = c->k_jets;
    return CPIC_OK;
}

extern "C" cpic_status cpic_set_push_mode(cpic_ctx* c, int32_t mode)
{
    if (!c) return fail(nullptr, CPIC_E_INVALID, "cpic_set_push_mode: NULL context");
    if (mode != CPIC_PUSH_GATHER && mode != CPIC_PUSH_TABLE && mode != CPIC_PUSH_TILE)
        return fail(c, CPIC_E_INVALID, "cpic_set_push_mode: CPIC_PUSH_GATHER, CPIC_PUSH_TABLE or CPIC_PUSH_TILE");
    if (mode == CPIC_PUSH_TABLE && (c->nc != 3 || c->pp.color_update != CPIC_COLOR_ROTATE))
        return fail(c, CPIC_E_INVALID, "cpic_set_push_mode: the force table serves the SU(3) rotation update");
    if (mode == CPIC_PUSH_TILE && !fused_ok(c))
        return fail(c, CPIC_E_INVALID,
                    "cpic_set_push_mode: the tile push needs SU(3) particles with the rotation colour update and no "
                    "light-like paths");
    HIPCHK(c, hipStreamSynchronize(c->st), "set push mode");
    if (mode == CPIC_PUSH_TILE) {
        if (c->cfg.split != 4) {
            c->cfg.split = 4;
            c->cfg.waves = 1;
            if (!fused_shape(c->cfg.bx, c->cfg.by)) {
                c->cfg.bx = c->N < 64 ? (c->N >= 16 ? 16 : 8) : 64;
                c->cfg.by = c->N < 64 ? c->cfg.bx : 8;
            }
        }
        c->push_table = false;
        set_store_policy(c);
        drop_graphs(c);
        return CPIC_OK;
    }
    if (c->cfg.split == 4) c->cfg.split = 3;  // back to the compressed tiles with a separate push
    if (mode == CPIC_PUSH_TABLE && !c->ftab)
        HIPCHK(c, hipMalloc(&c->ftab, (size_t)48 * c->V * c->tsz), "force table");
    c->push_table = mode == CPIC_PUSH_TABLE;
    set_store_policy(c);
    drop_graphs(c);
    return CPIC_OK;
}

extern "C" cpic_status cpic_get_push_mode(const cpic_ctx* c, int32_t* mode)
{
    if (!c || !mode) return CPIC_E_INVALID;
    *mode = fused_active(c) ? CPIC_PUSH_TILE : (c->push_table ? CPIC_PUSH_TABLE : CPIC_PUSH_GATHER);
    return CPIC_OK;
}
