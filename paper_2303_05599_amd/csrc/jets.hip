// jets.hip -- the light-like jet limit of the momentum broadening
// (Sec. V.B, [eq:mombroadjets]).
//
// A parton moving along +x at the speed of light picks up the colour Lorentz
// force f_x = E_x, f_y = E_y - B_eta, f_z = E_eta + B_y, seen through the
// Wilson line W of the links it has crossed: f~ = W f W^+.  Its broadening
// is <dp_i^2> = (q2/8) |F_i|^2 for charges rotated uniformly over their
// orbit, F_i = sum_n w f~_i(t_n).  The kernel follows one straight path per
// lattice site: all paths of a step sit at the same offset k from their
// start, so the lanes of a wavefront read consecutive sites (a coalesced
// stream through the lattice, like the field update).
//
// Per step and path: W is multiplied by the crossed x link when the nearest
// grid point moves (once per 1/dt steps), the five fields f needs are read
// at the nearest grid point from the per-site force table of the step
// (force_table_kernel: the fields of Sec. III.B at every site, zero where
// they vanish at t_0), transported with W and added to F.  On recording steps each
// wavefront writes the double-precision sum of |F_i|^2 over its 64 paths.
#include "cellfields.h"
#include "reduce.h"

namespace cpic {

// cell offset of every path after m steps: floor(x_off + m dt + 1/2),
// evaluated without contraction so that it matches a plain double evaluation
__device__ __forceinline__ int path_offset(double x_off, int m, double dt)
{
#pragma clang fp contract(off)
    return (int)floor(x_off + (double)m * dt + 0.5);
}

// Three wavefronts share a group of 64 paths, one per force component
// (role 0: f_x, 1: f_y, 2: f_z): each reads the group's Wilson lines, applies
// a crossing, evaluates and transports its own component and adds it to its
// part of F.  Role 0 stores the Wilson lines.  Splitting by component keeps
// each wavefront's chain of dependent loads and its live registers short.
constexpr int kJetRoles = 3;

template <typename T>
__global__ __launch_bounds__(64 * kJetRoles) void jet_kernel(Fields<T> Af, const T* table, T* Wb, T* Fb, JetArgs a,
                                                             const int* d_step, double* partials)
{
    const int N = a.N, V = N * N;
    const int ngroups = jet_groups(V);
    const int group = xcd_block(ngroups);
    if (group >= ngroups) return;
    const int n = d_step[1];
    if (n < a.sc.n_form || n >= a.sc.n_max) return;  // uniform over the grid
    const int m = n - a.sc.n_form;
    const int k = path_offset(a.x_off, m, a.sc.dt);
    const int kp = m > 0 ? path_offset(a.x_off, m - 1, a.sc.dt) : k;
    const bool hop = k != kp, eval = m % a.stride == 0, rec = is_record_step(a.sc, n);
    if (!(m == 0 || hop || eval || rec)) return;

    const int role = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6), lane = (int)threadIdx.x & 63;
    const int p = group * 64 + lane;
    const bool live = p < V;
    const int q = live ? p : 0;
    const int y = q / N, i = q - y * N;
    const uint32_t po = (uint32_t)q * (uint32_t)sizeof(T);
    const View<T> A = make_view<T>(Af.U, kRealsPerSite, V), TV = make_view<T>(table, 48, V);
    const View<T> WV = make_view<T>(Wb, 18, V), FV = make_view<T>(Fb, 24, V);

    m3<T> w;
    if (m == 0) {
        w = identity<T>();
    } else {
#pragma unroll
        for (int c = 0; c < 9; c++) w.e[c] = {bld(WV, po, 2 * c), bld(WV, po, 2 * c + 1)};
    }
    if (hop) {
        // the path left cell i + kp for i + kp + 1: W <- W U_x(i + kp), links at t_n
        const int xo = (i + kp % N) % N;  // kp >= 0
        w = mul(w, vU(A, (uint32_t)(y * N + xo) * (uint32_t)sizeof(T), 0));
        if constexpr (sizeof(T) == 4) w = reunitarize(w);
    }
    if (m == 0 || hop) {  // uniform over the grid
        // every wavefront of the group has read the old Wilson line (the
        // barrier waits for its loads) before role 0 overwrites it
        __syncthreads();
        if (role == 0 && live) {
#pragma unroll
            for (int c = 0; c < 9; c++) {
                bst(WV, po, 2 * c, w.e[c].re);
                bst(WV, po, 2 * c + 1, w.e[c].im);
            }
        }
    }
    CPIC_PHASE();

    // this wavefront's component: transported with W, added to F_role
    const uint32_t fc = 8 * (uint32_t)role;
    a8<T> Fj = m == 0 ? azero<T>() : vA(FV, po, fc);
    if (eval) {
        const int x = (i + k % N) % N;
        const uint32_t cs = (uint32_t)(y * N + x) * (uint32_t)sizeof(T);
        // f_x = E_x, f_y = E_y - B_eta, f_z = E_eta + B_y (table slots in job order)
        a8<T> f = vA(TV, cs, 8 * (uint32_t)(role == 0 ? kJobEx : (role == 1 ? kJobEy : kJobEeta)));
        if (role > 0) {
            const a8<T> g = vA(TV, cs, 8 * (uint32_t)(role == 1 ? kJobBeta : kJobBy));
            const T sg = role == 1 ? T(-1) : T(1);
#pragma unroll
            for (int c = 0; c < 8; c++) f.v[c] += sg * g.v[c];
        }
        const a8<T> ft = transport(w, f);
        const T wgt = T(a.stride * a.sc.dt);
#pragma unroll
        for (int c = 0; c < 8; c++) Fj.v[c] += wgt * ft.v[c];
        if (live) vA_st(FV, po, fc, Fj);
    }

    if (rec) {
        double sq = 0;
        if (live)
#pragma unroll
            for (int c = 0; c < 8; c++) sq += (double)Fj.v[c] * (double)Fj.v[c];
        const double v = wave_sum(sq);
        double* dst = partials + ((size_t)record_slot_of(a.sc, n) * ngroups + group) * 4;
        if (lane == 0) {
            dst[role] = v;
            if (role == 0) dst[3] = 0.0;
        }
    }
}

template <typename T>
hipError_t launch_jets(const Fields<T>& A, const T* table, T* W, T* F, const JetArgs& a, const int* d_step,
                       double* partials, hipStream_t st, const KTimer& tm)
{
    if (!table || !W || !F || a.N <= 0 || a.stride < 1 || !(a.sc.dt > 0 && a.sc.dt <= 1)) return hipErrorInvalidValue;
    const int nb = jet_groups(a.N * a.N);
    klaunch(tm, jet_kernel<T>, dim3(8 * ((nb + 7) / 8)), dim3(64 * kJetRoles), st, A, table, W, F, a, d_step,
            partials);
    return hipGetLastError();
}
template hipError_t launch_jets<double>(const Fields<double>&, const double*, double*, double*, const JetArgs&,
                                        const int*, double*, hipStream_t, const KTimer&);
template hipError_t launch_jets<float>(const Fields<float>&, const float*, float*, float*, const JetArgs&, const int*,
                                       double*, hipStream_t, const KTimer&);

}  // namespace cpic
