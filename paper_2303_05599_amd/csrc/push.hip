// push.hip -- the Wong / CPIC particle push (Sec. III.B) and the momentum
// broadening sums [eq:mombroad].
//
// One thread owns one test particle (structure-of-arrays records).  At time
// t_n it (1) rotates its colour charge with the links it crossed since t_{n-1}
// and with the rapidity Wilson line, (2) reads the colour-electric and
// -magnetic fields at its nearest grid point from U(n), phi(n), E(n +- 1/2),
// pi(n +- 1/2), (3) takes one explicit Euler step.  On recording steps the
// block writes double-precision partial sums of the broadening; a second
// small kernel adds the block partials in a fixed order.
#include "reduce.h"
#include "wong.h"

namespace cpic {


// Sub-job placement.  The TPP waves that share a group of 64 particles split
// the eight sub-jobs of the colour fields (cellfields.h); the owner wave
// (role 0) meanwhile rotates Q and, after one barrier, contracts the helpers'
// vectors with Q.  Byte k of the table places sub-job k as (wave << 4 | LDS
// slot of that wave); wave 0 is the owner, which evaluates its sub-jobs
// itself.  Sub-jobs share a slot only if they are parts of the same field
// (B_eta).  Each helper takes one memory round trip per sub-job:
//   TPP 1: the owner evaluates everything;
//   TPP 2: wave 1 E_y (slot 0) and B_eta (slot 1), the owner the rest;
//   TPP 4: the helpers split by the link they transport with:
//          1: E_x, B_y and B_eta part 5 (U_x(c-x)); 2: E_y, B_x and part 6
//          (U_y(c-y)); 3: part 7 (U_y(c-x-y) and U_x(c-x)) and E_eta;
//   TPP 8: one sub-job per helper (E_eta beside part 6 in wave 6), in
//          blocks of 512 threads.
// The links are read as two rows (the third rebuilt).
template <int TPP> __device__ __forceinline__ constexpr int subjob_place(int k)
{
    constexpr uint64_t tab = TPP == 8   ? 0x7060503040612010ull
                             : TPP == 4 ? 0x3022121121312010ull
                             : TPP == 2 ? 0x1111110000001000ull
                                        : 0ull;
    return (int)((tab >> (8 * k)) & 0xffu);
}
template <int TPP> constexpr int kSlots = TPP == 4 ? 3 : 2;  // LDS slots per helper wave

// A helper of a four-wave group (the placement of subjob_place<4>), with the
// loads shared between its sub-jobs.  Role 1 (i = x) and 2 (i = y) gather in
// their first phase what other waves of the group also read (U_i(c-i), U_i(c),
// phi at c +- i, the plaquettes), and form D_i and their part of B_eta; in the
// second phase, with U_i(c-i) kept, E_i at c and c-i at both half steps,
// which no other wave reads.  Lines that several waves read are so fetched
// while they are all in flight, before the L2 turns them over.  Role 3 forms
// part 7 and E_eta in one round trip.  The results go to the wave's LDS slots
// (rows r0 + 8 slot).
template <typename T>
__device__ __forceinline__ void helper4(int role, const View<T>& A, const View<T>& B, const View<T>& Gv, const Cell& c,
                                        int n, T t, bool eonly, T (*shF)[64], int r0, int lane, bool live)
{
    const bool on_e = n > 0, on_bt = n > 0 && !eonly, on_be = !eonly;
    auto put = [&](int slot, const a8<T>& F) {
#pragma unroll
        for (int q = 0; q < 8; q++) shF[r0 + 8 * slot + q][lane] = live ? F.v[q] : T(0);
    };
    if (role == 3) {
        a8<T> part = azero<T>();
        if (on_be) part = subjob<T>(7, A, B, Gv, c, n, t);
        put(0, part);
        put(1, cell_Eeta<T>(A, B, c, n));
        return;
    }
    const int i = role - 1;
    const uint32_t sb = i == 0 ? c.s_xm : c.s_ym, ce = kCompE + 8 * (uint32_t)i;
    const m3<T> L = vU(A, sb, i);
    a8<T> bf = azero<T>(), part = azero<T>();
    if (on_bt) {
        // B_y = +(1/2t) D_x (role 1), B_x = -(1/2t) D_y (role 2)
        const a8<T> f = transport(vU(A, c.s, i), vA(A, i == 0 ? c.s_xp : c.s_yp, kCompPhi));
        const a8<T> b = transport_adj(L, vA(A, sb, kCompPhi));
        const T sc = (i == 0 ? T(1) : T(-1)) / (T(2) * t);
#pragma unroll
        for (int q = 0; q < 8; q++) bf.v[q] = sc * (f.v[q] - b.v[q]);
    }
    if (on_be) {
        part = transport_adj(L, vA(Gv, sb, 0));
        if (i == 0) {
            const a8<T> g0 = vA(Gv, c.s, 0);
#pragma unroll
            for (int q = 0; q < 8; q++) part.v[q] += g0.v[q];
        }
#pragma unroll
        for (int q = 0; q < 8; q++) part.v[q] *= T(-0.25);
    }
    put(1, bf);
    put(2, part);
    CPIC_PHASE();
    a8<T> e = azero<T>();
    if (on_e) {
        const a8<T> h0 = vA(A, c.s, ce), h1 = vA(B, c.s, ce), b0 = vA(A, sb, ce), b1 = vA(B, sb, ce);
        a8<T> back;
#pragma unroll
        for (int q = 0; q < 8; q++) back.v[q] = b0.v[q] + b1.v[q];
        const a8<T> tb = transport_adj(L, back);
        const T w = T(1) / (T(4) * t);
#pragma unroll
        for (int q = 0; q < 8; q++) e.v[q] = w * ((h0.v[q] + h1.v[q]) + tb.v[q]);
    }
    put(0, e);
}
__host__ __device__ constexpr int push_block_threads(int tpp) { return tpp == 8 ? 512 : 256; }

// TPP wavefronts per group of 64 particles: a block holds 256 / TPP particles
// (64 for TPP 8).  Wave w works on particle group w / TPP in role w % TPP, so
// every wave follows one uniform path.  The role-0 wave owns the particle
// state: it rotates Q while the helper waves evaluate their field vectors
// into LDS; after one barrier it contracts all of them with Q and takes the
// Euler step.
template <int TPP> constexpr int kPushPPB = push_block_threads(TPP) / TPP;  // particles per block

// Observables: on recording steps the owner wave of each group of 64 writes
// the group's four double-precision sums to partials[slot][group][4]; they
// are added over the groups, in group order, when the samples are read.
//
// LOGQ selects the alternative colour update of Sec. III.B instead of the
// rotation with the links: dQ/dt = i[Q, A_x v_x + A_y v_y + phi v_eta], with
// the gauge fields from the matrix logarithm of the links (A_x on the x link
// whose midpoint is nearest to the particle, (floor(x), NGP row); A_y on
// (NGP column, floor(y)); phi at the grid point; all at t_n), stepped by
// explicit Euler with the state at n like the rest of the particle.  The
// charges are then not renormalised (their Casimir drift is part of the
// method).
//
// TABLE reads the six field vectors at the cell from the per-site force
// table of this step (force_table_kernel) instead of evaluating them: the
// choice for dense ensembles, where several particles share a cell.  GL forms
// the B_eta sub-jobs from the links (no plaquette field; the straggler push
// of the fused step, fused.hip).
//
// push_particle: particle p (live: p is a particle) on the owner lane of its
// group, its broadening terms added to obs on recording steps; every wave of
// the block calls it (one barrier inside with more than one wave per group).
template <typename T, int TPP, bool LOGQ, bool TABLE = false, bool GL = false>
__device__ __forceinline__ void push_particle(const Fields<T>& Af, const Fields<T>& Bf, const T* gpl,
                                              const Parts<T>& P, const PushArgs& a, int n, int* err, int p, bool live,
                                              double (&obs)[4], const T* table = nullptr)
{
    static_assert(!(GL && (TPP == 4 || TABLE)), "B_eta from the links: generic sub-job placements only");
    constexpr int PPB = kPushPPB<TPP>;
    constexpr int NG = PPB / 64;                     // particle groups per block
    constexpr int S = kSlots<TPP>;
    const int wave = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63;
    const int role = wave % TPP, grp = wave / TPP;
    // helper-wave field vectors: row ((grp * (TPP-1) + role-1) * S + slot) * 8 + a
    __shared__ T shF[TPP > 1 ? NG * (TPP - 1) * S * 8 : 1][64];
    const int N = a.N, np = a.np;
    const uint32_t V = (uint32_t)N * N;
    const View<T> A = make_view<T>(Af.U, kRealsPerSite, V), B = make_view<T>(Bf.U, kRealsPerSite, V);
    const View<T> Gv = make_view<T>(gpl, kPlaqReals, V);
    const View<T> R = make_view<T>(P.r, kPartReals, (uint32_t)np);
    const View<int> C = make_view<int>(P.cell, 2, (uint32_t)np);
    const T t = T(n * a.sc.dt);
    const bool record = is_record_step(a.sc, n);
    const bool renorm = is_reunit_step(a.sc, n);
    const bool eonly = a.is_static != 0;
    const uint32_t po = (uint32_t)(live ? p : 0) * sizeof(T), pi = (uint32_t)(live ? p : 0) * sizeof(int);
    Particle<T> s;
    particle_cell(R, C, po, pi, N, a.is_static != 0, s);
    const Cell cell = make_cell<T>(s.nx, s.ny, N);
    T f[6] = {0, 0, 0, 0, 0, 0};
    if (role == 0) {
        particle_load_rotate<T, LOGQ, TPP == 8>(A, R, C, po, pi, cell, a, n, live, renorm, err, s);
        CPIC_PHASE();
        if (TABLE && live) {
            // all six table vectors gathered at once (one memory round trip)
            const View<T> TV = make_view<T>(table, 48, V);
            a8<T> tv[kJobs];
#pragma unroll
            for (int j = 0; j < kJobs; j++) tv[j] = vA(TV, cell.s, 8 * (uint32_t)j);
#pragma unroll
            for (int j = 0; j < kJobs; j++) f[j] += job_active(j, n, eonly) ? dot(s.Q, tv[j]) : T(0);
        } else if constexpr (!TABLE && TPP <= 2) {
            // the owner's own sub-jobs (one or two waves per group)
            if (live) {
#pragma unroll 1
                for (int k = 0; k < kSubJobs; k++) {
                    if ((subjob_place<TPP>(k) >> 4) != 0 || !subjob_active<GL>(k, n, eonly)) continue;
                    CPIC_PHASE();
                    const T dq = dot(s.Q, subjob<T, GL>(k, A, B, Gv, cell, n, t));
                    const int j = subjob_field(k);
#pragma unroll
                    for (int jj = 0; jj < kJobs; jj++) f[jj] += jj == j ? dq : T(0);
                }
            }
        }
    } else if constexpr (TPP == 4) {
        helper4<T>(role, A, B, Gv, cell, n, t, eonly, shF, (grp * (TPP - 1) + role - 1) * S * 8, lane, live);
    } else if (TPP > 1) {
        // a helper wave: its sub-jobs, accumulated into its LDS slots (the
        // loop is unrolled, so each sub-job's code is specialised; with eight
        // waves a helper's one or two sub-jobs share one round trip)
        const int row0 = (grp * (TPP - 1) + role - 1) * S * 8;
#pragma unroll
        for (int r = 0; r < S * 8; r++) shF[row0 + r][lane] = T(0);
#pragma unroll
        for (int k = 0; k < kSubJobs; k++) {
            const int pl = subjob_place<TPP>(k);
            if ((pl >> 4) != role || !subjob_active<GL>(k, n, eonly)) continue;
            if (TPP < 8) CPIC_PHASE();
            const a8<T> F = subjob<T, GL>(k, A, B, Gv, cell, n, t);
            const int r = row0 + (pl & 15) * 8;
#pragma unroll
            for (int q = 0; q < 8; q++) shF[r + q][lane] += live ? F.v[q] : T(0);
        }
    }
    if (TPP > 1) {
        __syncthreads();
        if (role == 0 && live) {
            // Q . (vector of each helper slot), each slot counted once
#pragma unroll
            for (int k = 0; k < kSubJobs; k++) {
                const int pl = subjob_place<TPP>(k);
                bool first = (pl >> 4) != 0 && !(GL && k > 5);
#pragma unroll
                for (int i = 0; i < k; i++)
                    if (subjob_place<TPP>(i) == pl) first = false;
                if (!first) continue;
                const int r = ((grp * (TPP - 1) + (pl >> 4) - 1) * S + (pl & 15)) * 8;
                T dq = s.Q.v[0] * shF[r][lane];
#pragma unroll
                for (int q = 1; q < 8; q++) dq = fmaT(s.Q.v[q], shF[r + q][lane], dq);
                const int j = subjob_field(k);
#pragma unroll
                for (int jj = 0; jj < kJobs; jj++) f[jj] += jj == j ? dq : T(0);
            }
        }
    }
    if (role == 0 && live) particle_update<T, LOGQ>(A, R, C, po, pi, cell, a, n, renorm, record, f, s, obs);
}

// one particle per owner lane, particle blk * PPB + grp * 64 + lane; the
// owner wave of each group of 64 writes the group's sums on recording steps
template <typename T, int TPP, bool LOGQ, bool TABLE = false>
__device__ __forceinline__ void push_body(const Fields<T>& Af, const Fields<T>& Bf, const T* gpl, const Parts<T>& P,
                                          const PushArgs& a, int n, double* partials, int* err, int blk,
                                          const T* table = nullptr)
{
    if (n < a.sc.n_form || n >= a.sc.n_max) return;  // uniform over the event
    constexpr int NG = kPushPPB<TPP> / 64;
    const int wave = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63;
    const int role = wave % TPP, grp = wave / TPP;
    const int p = blk * kPushPPB<TPP> + grp * 64 + lane;
    double obs[4] = {0, 0, 0, 0};
    push_particle<T, TPP, LOGQ, TABLE>(Af, Bf, gpl, P, a, n, err, p, p < a.np, obs, table);
    if (is_record_step(a.sc, n) && role == 0) {
        const int ngroups = (a.np + 63) / 64, group = blk * NG + grp;
        double* dst = partials + ((size_t)record_slot_of(a.sc, n) * ngroups + group) * 4;
#pragma unroll
        for (int c = 0; c < 4; c++) {
            const double v = wave_sum(obs[c]);
            if (lane == 0 && group < ngroups) dst[c] = v;
        }
    }
}

// The field update of step n copies n into d_step[1]; the push reads it there
// and its first block advances d_step[0] to n + 1 (no other kernel of the
// push reads d_step[0], and the next field update starts after the push).
__device__ __forceinline__ int push_step(int* d_step, int blk)
{
    const int n = d_step[1];
    if (blk == 0 && threadIdx.x == 0) d_step[0] = n + 1;
    return n;
}

// At least two waves per SIMD for blocks of 256 threads (FP64: 176 VGPRs,
// two blocks per CU), four (128 VGPRs: two blocks per CU) for the 512-thread
// blocks of eight waves per group.  A third block per CU (168 VGPRs, 12 of
// them spilled) puts more lines in flight than the L2 keeps for the
// wavefronts that share them: the FP64 step was 2.4 % slower.  The logarithm
// variant also takes two (FP64: 254 VGPRs, 8 spilled): with one wave per SIMD
// and no spills its FP64 step took 0.180 ms against 0.132 ms.
template <typename T, int TPP, bool LOGQ = false>
__global__ __launch_bounds__(push_block_threads(TPP), (TPP == 8 && !LOGQ) ? 4 : 2) void push_kernel(
    Fields<T> Af, Fields<T> Bf, const T* gpl, Parts<T> P, PushArgs a, int* d_step, double* partials, int* err)
{
    const int nblocks = (a.np + kPushPPB<TPP> - 1) / kPushPPB<TPP>;
    const int blk = xcd_block(nblocks);
    if (blk >= nblocks) return;
    const int n = push_step(d_step, blk);
    push_body<T, TPP, LOGQ>(Af, Bf, gpl, P, a, n, partials, err, blk);
}

// one wavefront per group of 64 particles, fields from the force table
template <typename T>
__global__ __launch_bounds__(256) void push_table_kernel(Fields<T> Af, Fields<T> Bf, const T* table, Parts<T> P,
                                                         PushArgs a, int* d_step, double* partials, int* err)
{
    const int nblocks = (a.np + 255) / 256;
    const int blk = xcd_block(nblocks);
    if (blk >= nblocks) return;
    const int n = push_step(d_step, blk);
    push_body<T, 1, false, true>(Af, Bf, nullptr, P, a, n, partials, err, blk, table);
}

// The six field vectors (E_x, E_y, E_eta, B_x, B_y, B_eta, 8 components
// each, [48][V]) at every site at t_n, from the same per-site arithmetic
// the push applies at a particle's cell.  Runs between the field update
// (which provides n in d_step[1]) and the table push or the light-like
// paths, which read the table at their cells.
template <typename T>
__global__ __launch_bounds__(256) void force_table_kernel(Fields<T> Af, Fields<T> Bf, const T* gpl, T* table, int N,
                                                          Schedule sc, bool electric_only, const int* d_step)
{
    const int V = N * N, nb = (V + 255) / 256;
    const int blk = xcd_block(nb);
    if (blk >= nb) return;
    const int n = d_step[1];
    if (n < sc.n_form || n >= sc.n_max) return;
    const int s = blk * 256 + (int)threadIdx.x;
    if (s >= V) return;
    const View<T> A = make_view<T>(Af.U, kRealsPerSite, V), B = make_view<T>(Bf.U, kRealsPerSite, V);
    const View<T> TB = make_view<T>(table, 48, V), Gv = make_view<T>(gpl, kPlaqReals, V);
    const Cell cell = make_cell<T>(s % N, s / N, N);
    const T t = T(n * sc.dt);
#pragma unroll 1
    for (int j = 0; j < kJobs; j++) {
        a8<T> F = azero<T>();
        if (job_active(j, n, electric_only)) F = job_field<T>(j, A, B, Gv, cell, n, t);
        vA_st(TB, (uint32_t)s * (uint32_t)sizeof(T), 8 * (uint32_t)j, F);
        CPIC_PHASE();
    }
}

// batched events: logical block g works on particle block map[g].y of event map[g].x
// (at least two waves per SIMD, as push_kernel: the FP64 batch of 64 uneven
// events ran 2.3 % faster than with three and 12 registers spilled)
template <typename T, int TPP>
__global__ __launch_bounds__(256, 2) void batch_push_kernel(const EventDesc* __restrict__ ev, const int2* __restrict__ map,
                                                         int total)
{
    const int g = xcd_block(total);
    if (g >= total) return;
    // the work item is uniform over the workgroup: keep it (and every address
    // derived from it) in scalar registers
    const int2 m = map[g];
    const int e = __builtin_amdgcn_readfirstlane(m.x), blk = __builtin_amdgcn_readfirstlane(m.y);
    const EventDesc& d = ev[e];
    const int n = __builtin_amdgcn_readfirstlane(push_step(d.d_step, blk));
    if (d.pa.np == 0) return;  // an event without particles only advances its step
    const int V = d.N * d.N, parity = (n & 1) ^ d.flip;
    push_body<T, TPP, false>(fields_at<T>(d.f[parity], V), fields_at<T>(d.f[parity ^ 1], V),
                             static_cast<const T*>(d.gpl), Parts<T>{static_cast<T*>(d.pr), d.cell}, d.pa, n,
                             d.partials, d.d_err, blk);
}

template <typename T>
hipError_t launch_batch_push(const EventDesc* ev, const int2* map, int total_blocks, int tpp, hipStream_t st)
{
    if (total_blocks <= 0) return hipSuccess;
    const dim3 g(8 * ((total_blocks + 7) / 8)), b(256);
    switch (tpp) {
    case 2: hipLaunchKernelGGL((batch_push_kernel<T, 2>), g, b, 0, st, ev, map, total_blocks); break;
    case 4: hipLaunchKernelGGL((batch_push_kernel<T, 4>), g, b, 0, st, ev, map, total_blocks); break;
    default: hipLaunchKernelGGL((batch_push_kernel<T, 1>), g, b, 0, st, ev, map, total_blocks);
    }
    return hipGetLastError();
}
template hipError_t launch_batch_push<double>(const EventDesc*, const int2*, int, int, hipStream_t);
template hipError_t launch_batch_push<float>(const EventDesc*, const int2*, int, int, hipStream_t);

int push_blocks(int np, int tpp) { return push_blocks_d(np, tpp); }

template <typename T>
hipError_t launch_force_table(const Fields<T>& A, const Fields<T>& B, const T* gpl, T* table, int N,
                              const Schedule& sc, bool electric_only, const int* d_step, hipStream_t st,
                              const KTimer& tm)
{
    if (!table || !gpl || N <= 0) return hipErrorInvalidValue;
    const int nbt = (N * N + 255) / 256;
    klaunch(tm, force_table_kernel<T>, dim3(8 * ((nbt + 7) / 8)), dim3(256), st, A, B, gpl, table, N, sc,
            electric_only, d_step);
    return hipGetLastError();
}
template hipError_t launch_force_table<double>(const Fields<double>&, const Fields<double>&, const double*, double*,
                                               int, const Schedule&, bool, const int*, hipStream_t, const KTimer&);
template hipError_t launch_force_table<float>(const Fields<float>&, const Fields<float>&, const float*, float*, int,
                                              const Schedule&, bool, const int*, hipStream_t, const KTimer&);

template <typename T>
hipError_t launch_push_table(const Fields<T>& A, const Fields<T>& B, const T* table, const Parts<T>& P,
                             const PushArgs& a, int* d_step, double* partials, int* err, hipStream_t st,
                             const KTimer& tm)
{
    if (a.np <= 0) return hipSuccess;
    if (!table) return hipErrorInvalidValue;
    const int nb = (a.np + 255) / 256;
    klaunch(tm, push_table_kernel<T>, dim3(8 * ((nb + 7) / 8)), dim3(256), st, A, B, table, P, a, d_step, partials,
            err);
    return hipGetLastError();
}
template hipError_t launch_push_table<double>(const Fields<double>&, const Fields<double>&, const double*,
                                              const Parts<double>&, const PushArgs&, int*, double*, int*, hipStream_t,
                                              const KTimer&);
template hipError_t launch_push_table<float>(const Fields<float>&, const Fields<float>&, const float*,
                                             const Parts<float>&, const PushArgs&, int*, double*, int*, hipStream_t,
                                             const KTimer&);

template <typename T, bool LOGQ>
static void launch_push_t(const Fields<T>& A, const Fields<T>& B, const T* gpl, const Parts<T>& P, const PushArgs& a,
                          int* d_step, double* partials, int* err, hipStream_t st, const KTimer& tm)
{
    const int nb = push_blocks(a.np, a.tpp);
    const dim3 g(8 * ((nb + 7) / 8)), b(push_block_threads(a.tpp));
    switch (a.tpp) {
    case 2: klaunch(tm, push_kernel<T, 2, LOGQ>, g, b, st, A, B, gpl, P, a, d_step, partials, err); break;
    case 4: klaunch(tm, push_kernel<T, 4, LOGQ>, g, b, st, A, B, gpl, P, a, d_step, partials, err); break;
    case 8: klaunch(tm, push_kernel<T, 8, LOGQ>, g, b, st, A, B, gpl, P, a, d_step, partials, err); break;
    default: klaunch(tm, push_kernel<T, 1, LOGQ>, g, b, st, A, B, gpl, P, a, d_step, partials, err);
    }
}

template <typename T>
hipError_t launch_push(const Fields<T>& A, const Fields<T>& B, const T* gpl, const Parts<T>& P, const PushArgs& a,
                       int* d_step, double* partials, int* err, hipStream_t st, const KTimer& tm)
{
    if (a.np <= 0) return hipSuccess;
    if (!gpl) return hipErrorInvalidValue;
    if (a.color_log)
        launch_push_t<T, true>(A, B, gpl, P, a, d_step, partials, err, st, tm);
    else
        launch_push_t<T, false>(A, B, gpl, P, a, d_step, partials, err, st, tm);
    return hipGetLastError();
}

// The particles that left their tile since the last reordering: blocks of
// eight waves (one group of 64 particles, one B_eta part or field per wave,
// above) over the stragglers of kStragTiles consecutive tiles, in list
// order.  Advances the step counter like the push.
template <typename T>
__global__ __launch_bounds__(512) void straggler_kernel(Fields<T> Af, Fields<T> Bf, Parts<T> P, PushArgs a,
                                                        TileParts tp, int ntiles, int* d_step, double* partials,
                                                        int ngroups, int* err)
{
    constexpr int TB = kStragTiles;
    const int nb = (ntiles + TB - 1) / TB, blk = (int)blockIdx.x;
    if (blk >= nb) return;
    const int n = push_step(d_step, blk);
    if (n < a.sc.n_form || n >= a.sc.n_max) return;  // uniform
    __shared__ int pre[TB + 1];
    const int t0 = blk * TB;
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int j = 0; j < TB; j++) {
            pre[j] = acc;
            acc += t0 + j < ntiles ? tp.strag_count[t0 + j] : 0;
        }
        pre[TB] = acc;
    }
    __syncthreads();
    const int K = pre[TB], lane = (int)threadIdx.x & 63;
    if (tp.strag_total && threadIdx.x == 0 && K > 0) atomicAdd(tp.strag_total, (unsigned long long)K);
    double obs[4] = {0, 0, 0, 0};
    for (int c0 = 0; c0 < K; c0 += 64) {
        const int i = c0 + lane;
        bool live = i < K;
        int p = 0;
        if (live) {
            int j = 0;
            while (j + 1 < TB && pre[j + 1] <= i) j++;
            const int k = tp.tile_start[t0 + j] + (i - pre[j]);
            p = k >= 0 && k < a.np ? tp.strag[k] : -1;
            live = p >= 0 && p < a.np;
        }
        push_particle<T, 8, false, false, true>(Af, Bf, nullptr, P, a, n, err, p, live, obs);
        __syncthreads();  // the next chunk rewrites the helpers' LDS slots
    }
    if (is_record_step(a.sc, n) && threadIdx.x < 64) {
        double* dst = partials + ((size_t)record_slot_of(a.sc, n) * ngroups + ntiles + blk) * 4;
#pragma unroll
        for (int c = 0; c < 4; c++) {
            const double v = wave_sum(obs[c]);
            if (lane == 0) dst[c] = v;
        }
    }
}

template <typename T>
hipError_t launch_stragglers(const Fields<T>& A, const Fields<T>& B, const Parts<T>& P, const PushArgs& a,
                             const TileParts& tp, int ntiles, int* d_step, double* partials, int ngroups, int* err,
                             hipStream_t st, const KTimer& tm)
{
    const int nb = (ntiles + kStragTiles - 1) / kStragTiles;
    klaunch(tm, straggler_kernel<T>, dim3(nb), dim3(512), st, A, B, P, a, tp, ntiles, d_step, partials, ngroups, err);
    return hipGetLastError();
}
template hipError_t launch_stragglers<double>(const Fields<double>&, const Fields<double>&, const Parts<double>&,
                                              const PushArgs&, const TileParts&, int, int*, double*, int, int*,
                                              hipStream_t, const KTimer&);
template hipError_t launch_stragglers<float>(const Fields<float>&, const Fields<float>&, const Parts<float>&,
                                             const PushArgs&, const TileParts&, int, int*, double*, int, int*,
                                             hipStream_t, const KTimer&);

// step end of an event without particles (no push): advance the step counter
__global__ void step_advance_kernel(int* d_step)
{
    if (threadIdx.x == 0) d_step[0] = d_step[1] + 1;
}
hipError_t launch_step_advance(int* d_step, hipStream_t st)
{
    hipLaunchKernelGGL(step_advance_kernel, dim3(1), dim3(64), 0, st, d_step);
    return hipGetLastError();
}

// out[c] = sum (or max, bit c of mask) over rows of partials[row][c]; one block,
// rows dealt to threads in a fixed pattern, then a fixed-order block reduction
template <int NC>
__global__ __launch_bounds__(256) void reduce_rows_kernel(const double* __restrict__ partials, int nrows,
                                                          unsigned mask, double* out)
{
    double v[NC];
#pragma unroll
    for (int c = 0; c < NC; c++) v[c] = 0;
    for (int r = threadIdx.x; r < nrows; r += blockDim.x)
#pragma unroll
        for (int c = 0; c < NC; c++) {
            const double x = partials[(size_t)r * NC + c];
            v[c] = ((mask >> c) & 1) ? fmax(v[c], x) : v[c] + x;
        }
    block_reduce_store<NC>(v, mask, out);
}

// samples: block b sums the rows of sample slot first + b (4 columns each)
__global__ __launch_bounds__(256) void reduce_samples_kernel(const double* __restrict__ partials, int nrows, int first,
                                                             double* out)
{
    const int slot = first + (int)blockIdx.x;
    double v[4] = {0, 0, 0, 0};
    for (int r = threadIdx.x; r < nrows; r += blockDim.x)
#pragma unroll
        for (int c = 0; c < 4; c++) v[c] += partials[((size_t)slot * nrows + r) * 4 + c];
    block_reduce_store<4>(v, 0u, out + (size_t)slot * 4);
}
hipError_t launch_reduce_samples(const double* partials, int nrows, int first_slot, int count, double* out,
                                 hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(reduce_samples_kernel, dim3(count), dim3(256), 0, st, partials, nrows, first_slot, out);
    return hipGetLastError();
}

hipError_t launch_reduce_rows(const double* partials, int nrows, int ncols, double* out, hipStream_t st)
{
    if (ncols == 4) {
        hipLaunchKernelGGL(reduce_rows_kernel<4>, dim3(1), dim3(256), 0, st, partials, nrows, 0u, out);
    } else if (ncols == 8) {
        // diagnostics layout: columns 1 and 6 are maxima
        hipLaunchKernelGGL(reduce_rows_kernel<8>, dim3(1), dim3(256), 0, st, partials, nrows, (1u << 1) | (1u << 6),
                           out);
    } else if (ncols == 2) {
        hipLaunchKernelGGL(reduce_rows_kernel<2>, dim3(1), dim3(256), 0, st, partials, nrows, 3u, out);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// The drift watchdog's comparison of the diagnostics dout[10] (the columns
// of cpic_diagnostics) with the baseline taken when the state was installed
// (take_base: store dout as the baseline).  flags: bit 0 a non-finite
// column, 1 unitarity max|UU^+ - 1| > thr[0], 2 Gauss drift
// |max|G| - max|G|_0| > thr[1] max(1, max|G|_0), 3 Casimir drift: max|q2 -
// q2(R)| or max|q3 - q3(R)| moved from its baseline by more than thr[2]
// max(1, q2(R)).  The first breach is kept: watch[0] flags, watch[1] step,
// vals the unitarity and the three drifts.
__global__ void watchdog_kernel(const double* dout, double* base, int take_base, int with_casimir, double thr_u,
                                double thr_g, double thr_c, double q2ref, int n, int* watch, double* vals)
{
    if (threadIdx.x != 0) return;
    if (take_base) {
        for (int k = 0; k < 10; k++) base[k] = dout[k];
        return;
    }
    const double dg = fabs(dout[1] - base[1]);
    const double d2 = with_casimir ? fabs(dout[8] - base[8]) : 0.0, d3 = with_casimir ? fabs(dout[9] - base[9]) : 0.0;
    int f = 0;
    for (int k = 0; k < (with_casimir ? 10 : 8); k++)
        if (!isfinite(dout[k])) f |= 1;
    if (dout[6] > thr_u) f |= 2;
    if (dg > thr_g * fmax(1.0, base[1])) f |= 4;
    if (d2 > thr_c * fmax(1.0, q2ref) || d3 > thr_c * fmax(1.0, q2ref)) f |= 8;
    if (f && watch[0] == 0) {
        watch[0] = f;
        watch[1] = n;
        vals[0] = dout[6];
        vals[1] = dg;
        vals[2] = d2;
        vals[3] = d3;
    }
}
hipError_t launch_watchdog(const double* dout, double* base, bool take_base, bool with_casimir, const double thr[3],
                           double q2ref, int n, int* watch, double* vals, hipStream_t st)
{
    hipLaunchKernelGGL(watchdog_kernel, dim3(1), dim3(64), 0, st, dout, base, take_base ? 1 : 0, with_casimir ? 1 : 0,
                       thr[0], thr[1], thr[2], q2ref, n, watch, vals);
    return hipGetLastError();
}

// per block: max |q2 - q2_0|, max |q3 - q3_0| over the particles
template <typename T>
__global__ __launch_bounds__(256) void part_diag_kernel(Parts<T> P, int np, double q2r, double q3r, double* partials)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    double v[2] = {0, 0};
    if (p < np) {
        a8<double> Q;
        for (int q = 0; q < 8; q++) Q.v[q] = P.r[(size_t)(PQ0 + q) * np + p];
        const m3<double> H = herm(Q);
        const m3<double> H2 = mul(H, H);
        double tr3 = 0;
        for (int i = 0; i < 3; i++)
            for (int k = 0; k < 3; k++) tr3 += H.e[3 * i + k].re * H2.e[3 * k + i].re - H.e[3 * i + k].im * H2.e[3 * k + i].im;
        v[0] = fabs(dot(Q, Q) - q2r);
        v[1] = fabs(4.0 * tr3 - q3r);
    }
    block_reduce_store<2>(v, 3u, partials + (size_t)blockIdx.x * 2);
}
template <typename T>
hipError_t launch_part_diag(const Parts<T>& P, int np, double q2, double q3, double* partials, hipStream_t st)
{
    hipLaunchKernelGGL(part_diag_kernel<T>, dim3(push_blocks(np, 1)), dim3(256), 0, st, P, np, q2, q3, partials);
    return hipGetLastError();
}

template hipError_t launch_push<double>(const Fields<double>&, const Fields<double>&, const double*,
                                        const Parts<double>&, const PushArgs&, int*, double*, int*, hipStream_t,
                                        const KTimer&);
template hipError_t launch_push<float>(const Fields<float>&, const Fields<float>&, const float*, const Parts<float>&,
                                       const PushArgs&, int*, double*, int*, hipStream_t, const KTimer&);
template hipError_t launch_part_diag<double>(const Parts<double>&, int, double, double, double*, hipStream_t);
template hipError_t launch_part_diag<float>(const Parts<float>&, int, double, double, double*, hipStream_t);

}  // namespace cpic
