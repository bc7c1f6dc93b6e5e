// internal.h -- declarations shared by the translation units of libcpic.
// Device data layout (structure of arrays, site index s = y*N + x):
//   links  U[i][c][s]  i = 0 (e1), 1 (e2); c = 2*(3*row+col) + {0: re, 1: im}
//   fields phi[a][s], E[i][a][s], pi[a][s] (8 algebra components a)
// One field buffer set holds U, phi, E, pi contiguously (68 reals per site).
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace cpic {

constexpr int kRealsPerSite = 68;
// x y eta px py peta deta ux0 uy0 pt0 Q1..Q8, and p^tau integrated from its own
// equation of motion (the temporal-constraint check of Appendix D)
constexpr int kPartReals = 19;
enum PartCol { PX_ = 0, PY_, PETA_, PPX, PPY, PPETA, PDETA, PUX0, PUY0, PPT0, PQ0, PPTAU = PQ0 + 8 };

template <typename T> struct Fields {
    T* U;    // [2][18][V]
    T* phi;  // [8][V]
    T* E;    // [2][8][V]
    T* pi;   // [8][V]
};
template <typename T> __host__ __device__ inline Fields<T> fields_at(void* base, int V)
{
    T* p = static_cast<T*>(base);
    return {p, p + 36 * (size_t)V, p + 44 * (size_t)V, p + 60 * (size_t)V};
}

// SU(2) buffer set (20 reals per site): U[i][4][V] quaternions (w, a1, a2, a3),
// phi[3][V], E[2][3][V], pi[3][V]
constexpr int kRealsPerSite2 = 20;
template <typename T> struct Fields2 {
    T* U;
    T* phi;
    T* E;
    T* pi;
};
template <typename T> __host__ __device__ inline Fields2<T> fields2_at(void* base, int V)
{
    T* p = static_cast<T*>(base);
    return {p, p + 8 * (size_t)V, p + 11 * (size_t)V, p + 17 * (size_t)V};
}

template <typename T> struct Parts {
    T* r;       // [19][np] (PartCol order)
    int* cell;  // [2][np]
};

// Step schedule.  The current step n lives in device memory (one int per
// event) so that a captured sequence of launches can be replayed for any n:
// every kernel derives t_n, the kick/formation/recording/reunitarisation
// decisions and the sample slot from n.  The last kernel of a step advances n.
struct Schedule {
    double dt;         // dtau / a
    int n_max;         // steps to tau_max
    int n_form;        // first step of the particle push
    int n_plaq;        // first step whose field update stores the plaquette field G (the push's B_eta)
    int record_every;  // samples after steps with (n+1) % record_every == 0, and after n_max - 1
    int reunit_every;  // FP32: reunitarise links / renormalise charges after steps with (n+1) % k == 0
};
__host__ __device__ inline bool is_record_step(const Schedule& s, int n)
{
    return n >= s.n_form && n < s.n_max && ((n + 1) % s.record_every == 0 || n + 1 == s.n_max);
}
__host__ __device__ inline int record_slot_of(const Schedule& s, int n)
{
    return n / s.record_every - s.n_form / s.record_every;
}
__host__ __device__ inline int num_slots(const Schedule& s)
{
    return s.n_max > s.n_form ? record_slot_of(s, s.n_max - 1) + 1 : 0;
}
__host__ __device__ inline bool is_reunit_step(const Schedule& s, int n)
{
    return s.reunit_every > 0 && (n + 1) % s.reunit_every == 0;
}

struct LaunchCfg {
    int bx = 64, by = 4;  // field kernel block shape
    int xcd_remap = 1;    // map consecutive tiles onto one XCD
    int waves = 1;        // register-allocation occupancy target of the field kernel (1 = compiler default)
    int split = 0;        // kernel variant: 0 one thread per site, 1 one thread per link (128 sites per
                          // block), 2 one thread per site with the tile and its halo staged in LDS,
                          // 3 as 2 with two rows per link in LDS and the scalars from global memory,
                          // 4 as 3 with the particle push of the tile in the same kernel (fused.hip)
    int nt_store = 0;     // variant 3 with particles: the new links and phi stored non-temporal
};

struct PushArgs {
    int N, np, is_static;
    int tpp;          // wavefronts per particle group (1, 2, 4)
    int color_log;    // 1: colour update from the matrix logarithm of the links instead of the rotation
    double mhat;
    double q0eig[3];  // sorted eigenvalues of Q0 (charge renormalisation)
    Schedule sc;
};

// one event of a batch, as the batched kernels see it
struct EventDesc {
    void* f[2];        // field buffer sets; the state at step n is in f[(n & 1) ^ flip]
    int flip;
    void* pr;          // particle records [19][np]
    void* gpl;         // plaquette field G [8][V] (NULL without particles)
    int* cell;         // [2][np]
    int N;
    PushArgs pa;
    int* d_step;       // [2] (see the step counter protocol)
    int* d_err;
    double* partials;  // [slots][particle groups][4]
};

// particle blocks of the push: 256 / tpp particles per block (64 in the
// 512-thread blocks of tpp = 8)
__host__ __device__ inline int push_blocks_d(int np, int tpp)
{
    const int ppb = tpp == 8 ? 64 : 256 / (tpp > 0 ? tpp : 1);
    return (np + ppb - 1) / ppb;
}

// Optional kernel timing: with `start` set, the launch records the kernel's
// own start and stop times in the two events (no extra queue packets).
struct KTimer {
    hipEvent_t start = nullptr, stop = nullptr;
};
template <typename F, typename... Args>
inline void klaunch(const KTimer& tm, F kernel, dim3 grid, dim3 block, hipStream_t st, Args... args)
{
    if (tm.start)
        hipExtLaunchKernelGGL(kernel, grid, block, 0, st, tm.start, tm.stop, 0, args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, 0, st, args...);
}

// ---- field kernels (field.hip)
// gpl (may be NULL): the plaquette field G = Proj U_12 of every site at step
// n, [8][V], stored by the field update of steps n >= sc.n_plaq for the push,
// the force table and the light-like paths (B_eta from the clover, cellfields.h)
constexpr int kPlaqReals = 8;
template <typename T>
hipError_t launch_field_step(const Fields<T>& in, const Fields<T>& out, T* gpl, int N, const Schedule& sc,
                             int* d_step, const LaunchCfg& cfg, hipStream_t st, const KTimer& tm = KTimer{});
// energies = false: the energy columns are left 0 (the drift watchdog's checks)
template <typename T>
hipError_t launch_field_diag(const Fields<T>& f, int N, double dt, int n, double* partials, int nblk_cap,
                             int* nblk_out, hipStream_t st, bool energies = true);
// batched launches: logical block g works on tile (particle block) map[g].y
// of event map[g].x of the descriptor table
template <typename T>
hipError_t launch_batch_field(const EventDesc* ev, const int2* map, int total_tiles, const LaunchCfg& cfg,
                              hipStream_t st);

// ---- fused field update and tile push (fused.hip)
// Variant 4 of the field launch: one workgroup per tile of bx x by sites
// updates the fields and pushes the particles whose records the last
// reordering put in the tile's range (records ordered by these tiles);
// particles that have left their tile since then (stragglers) are pushed by
// a second kernel that gathers their fields from the buffer sets.
struct TileParts {
    const int* tile_start;  // [ntiles + 1]: records of tile t at [tile_start[t], tile_start[t+1])
    int* strag;             // [np]: stragglers of tile t at strag[tile_start[t] ...]
    int* strag_count;       // [ntiles]: how many
    unsigned long long* strag_total;  // running sum of the stragglers pushed (kernel timing), or NULL
};
constexpr int kStragTiles = 8;  // tiles per block of the straggler push
__host__ __device__ inline bool fused_shape(int bx, int by)
{
    return (bx == 64 && by == 8) || (bx == 32 && by == 8) || (bx == 16 && by == 16) || (bx == 8 && by == 8);
}
__host__ __device__ inline int fused_tiles(int N, int bx, int by) { return ((N + bx - 1) / bx) * ((N + by - 1) / by); }
// sample groups of the fused step: the tiles, then the straggler blocks
__host__ __device__ inline int fused_groups(int N, int bx, int by)
{
    const int nt = fused_tiles(N, bx, by);
    return nt + (nt + kStragTiles - 1) / kStragTiles;
}
// most sample groups of any fused shape (8 x 8 tiles)
inline int fused_groups_max(int N) { return fused_groups(N, 8, 8); }
// A holds the state at step n (read), B receives step n+1; the two timers
// time the tile kernel and the straggler push
template <typename T>
hipError_t launch_fused(const Fields<T>& A, const Fields<T>& B, const LaunchCfg& cfg, const Parts<T>& P,
                        const PushArgs& a, const TileParts& tp, int* d_step, double* partials, int* err,
                        hipStream_t st, const KTimer& tm_tile = KTimer{}, const KTimer& tm_strag = KTimer{});

// ---- particle kernels (push.hip)
// push at t_n: A holds U(n), phi(n), E(n-1/2), pi(n-1/2); B holds E(n+1/2), pi(n+1/2);
// the fields at a particle's cell are evaluated from them (cellfields.h)
// (gpl: the plaquette field of step n, see launch_field_step)
template <typename T>
hipError_t launch_push(const Fields<T>& A, const Fields<T>& B, const T* gpl, const Parts<T>& P, const PushArgs& a,
                       int* d_step, double* partials, int* err, hipStream_t st, const KTimer& tm = KTimer{});
int push_blocks(int np, int tpp);
// the six field vectors of every site at t_n into table [48][V] (job order,
// zero where a field is inactive at step n or, with electric_only, magnetic),
// for steps sc.n_form <= n < sc.n_max
template <typename T>
hipError_t launch_force_table(const Fields<T>& A, const Fields<T>& B, const T* gpl, T* table, int N,
                              const Schedule& sc, bool electric_only, const int* d_step, hipStream_t st,
                              const KTimer& tm = KTimer{});
// the stragglers of the fused step (A, B as for the push, B_eta from the links)
template <typename T>
hipError_t launch_stragglers(const Fields<T>& A, const Fields<T>& B, const Parts<T>& P, const PushArgs& a,
                             const TileParts& tp, int ntiles, int* d_step, double* partials, int ngroups, int* err,
                             hipStream_t st, const KTimer& tm = KTimer{});
// dense ensembles: a push that reads the fields at the cell from the force
// table (one wavefront per 64 particles)
template <typename T>
hipError_t launch_push_table(const Fields<T>& A, const Fields<T>& B, const T* table, const Parts<T>& P,
                             const PushArgs& a, int* d_step, double* partials, int* err, hipStream_t st,
                             const KTimer& tm = KTimer{});
template <typename T>
hipError_t launch_batch_push(const EventDesc* ev, const int2* map, int total_blocks, int tpp, hipStream_t st);
hipError_t launch_reduce_rows(const double* partials, int nrows, int ncols, double* out, hipStream_t st);
// out[slot] for slots first_slot .. first_slot + count - 1 of partials[slot][nrows][4], one launch
// (the same fixed-order sums as launch_reduce_rows)
hipError_t launch_reduce_samples(const double* partials, int nrows, int first_slot, int count, double* out,
                                 hipStream_t st);
// Step counter protocol: d_step[0] is the current step n; the field update
// copies it to d_step[1]; the push (or, without particles, the step advance)
// sets d_step[0] = d_step[1] + 1.
hipError_t launch_step_advance(int* d_step, hipStream_t st);
// samples: partials[slot][group of 64 particles][4]
inline int obs_groups(int np) { return (np + 63) / 64; }
template <typename T>
hipError_t launch_part_diag(const Parts<T>& P, int np, double q2, double q3, double* partials, hipStream_t st);
// drift watchdog on the diagnostics columns dout[10] (push.hip)
hipError_t launch_watchdog(const double* dout, double* base, bool take_base, bool with_casimir, const double thr[3],
                           double q2ref, int n, int* watch, double* vals, hipStream_t st);

// ---- light-like path integral (jets.hip)
// One path per site p = y*N + i, along +x at the speed of light from
// x = i + x_off at step sc.n_form; W [18][V] its Wilson line (row-major
// re/im), F [24][V] the integrated transported force components x, y, z.
struct JetArgs {
    int N;
    int stride;    // force evaluated on every stride-th step, weight stride * dt
    double x_off;  // start inside the cell, [0, 1)
    Schedule sc;   // n_form: first step of the paths; samples as for particles
};
// A holds U(n); table the force table of step n (launch_force_table)
template <typename T>
hipError_t launch_jets(const Fields<T>& A, const T* table, T* W, T* F, const JetArgs& a, const int* d_step,
                       double* partials, hipStream_t st, const KTimer& tm = KTimer{});
// samples: partials[slot][group of 64 paths][4] (|F_x|^2, |F_y|^2, |F_z|^2, 0)
__host__ __device__ inline int jet_groups(int V) { return (V + 63) / 64; }

// ---- SU(2) variant (su2.hip): site-parallel field update, one thread per particle
template <typename T>
hipError_t launch_su2_field(const Fields2<T>& in, const Fields2<T>& out, int N, const Schedule& sc, int* d_step,
                            hipStream_t st, const KTimer& tm = KTimer{});
template <typename T>
hipError_t launch_su2_push(const Fields2<T>& A, const Fields2<T>& B, const Parts<T>& P, const PushArgs& a,
                           int* d_step, double* partials, int* err, hipStream_t st, const KTimer& tm = KTimer{});
template <typename T>
hipError_t launch_su2_diag(const Fields2<T>& f, int N, double dt, int n, double* partials, int nblk_cap,
                           int* nblk_out, hipStream_t st);

// ---- particle ordering (sort.hip)
struct SortBufs {
    unsigned *keys = nullptr, *keys2 = nullptr;
    int* perm = nullptr;
    int *count = nullptr, *offs = nullptr;  // [key_cap] records per key (zero between reorderings), run ends
    int key_cap = 0;
    void* temp = nullptr;  // the scan's temporary storage
    size_t temp_bytes = 0;
    void* r2 = nullptr;  // [19][np] scratch records
    int *cell2 = nullptr, *pid2 = nullptr;
};
// keys of an N x N lattice lie below key_capacity(N) for every tile shape
int key_capacity(int N);
size_t sort_temp_bytes(int N);
// Orders the records by tiles of tx x ty cells (keys from the nearest grid
// point of the position with from_position, else from the cell); with
// tile_start ([ntiles + 1]) also the range of records of every tile.  The
// sorted keys stay in b.keys2 (launch_tile_start rebuilds the ranges from them).
template <typename T>
hipError_t sort_particles(const SortBufs& b, T* r, int* cell, int* pid, int np, int N, int tx, int ty,
                          bool from_position, int* tile_start, hipStream_t st);
hipError_t launch_tile_start(const unsigned* sorted_keys, int np, int N, int tx, int ty, int* tile_start,
                             hipStream_t st);
// the gather push's order: tiles of 32 x 16 cells, 32 cells being one
// 128-byte line of a single-precision component array (two of a double-precision
// one), so that no line is split between the tiles of two particle blocks
constexpr int kGatherSortTileX = 32, kGatherSortTileY = 16;
constexpr int kSortEvery = 16;  // steps between reorderings of moving particles (measured best of 8, 16, 32, 64)

// ---- initial condition (ic.hip), always double precision
struct ICArgs {
    int N;
    int n_sheets;
    uint64_t seed;
    double g2mua, mhat, uvhat;
    double tol;
    int maxit;
};
// builds U, pi (phi = E = 0) into a double buffer set; returns failures in *fails (device int)
hipError_t ic_glasma(const ICArgs& a, Fields<double> out, int* d_fails, hipStream_t st);
struct PartICArgs {
    int N, np, azimuth_uniform;
    uint64_t seed;
    double pt_min, pt_max;
    double q0[8];
};
hipError_t ic_particles(const PartICArgs& a, double* r /*[19][np]*/, int* cell, hipStream_t st);
// SU(2) variant: links, pi(0) into a double Fields2 set; Darboux charges with |Q|^2 = q2
hipError_t ic_glasma2(const ICArgs& a, Fields2<double> out, hipStream_t st);
hipError_t ic_particles2(const PartICArgs& a, double q2, double* r, int* cell, hipStream_t st);
hipError_t convert_to_float(const double* src, float* dst, size_t n, hipStream_t st);

}  // namespace cpic
