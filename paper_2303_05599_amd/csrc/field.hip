// field.hip -- the Glasma field update: one fused kick + drift pass per
// leapfrog step (Sec. II.A), plus the per-site diagnostics (Gauss residual,
// lattice energy, link unitarity).
//
// One thread owns one site.  Links and scalars of the neighbouring sites
// are read straight from the structure-of-arrays buffers; tiles are
// assigned so that the workgroups that share halos run on the same XCD and
// hit the same L2.  The step reads buffer `in` and writes buffer `out`
// (ping-pong), so the particle push can still see U(n), phi(n), E(n-1/2),
// pi(n-1/2) next to E(n+1/2), pi(n+1/2).
#include "internal.h"
#include "reduce.h"
#include "su3.h"
#include "bufio.h"
#include "tiles.h"

namespace cpic {


// Where the stencil reads links and scalars: straight from the global buffer
// (sites as byte offsets) or from a halo tile staged in LDS (sites as tile
// indices).  Same interface, so one stencil serves both kernels.
template <typename T> struct GlobalSrc {
    View<T> v;
    __device__ __forceinline__ m3<T> U(uint32_t s, int i) const { return vU(v, s, i); }
    __device__ __forceinline__ a8<T> A(uint32_t s, uint32_t c0) const { return vA(v, s, c0); }
};
// LDS halo tile: component c of tile site h at l[c * HS + h], components 0..43
// (links, then phi) in the buffer-set order
template <typename T, int HS> struct LdsSrc {
    const T* l;
    __device__ __forceinline__ m3<T> U(uint32_t h, int i) const
    {
        m3<T> m;
#pragma unroll
        for (int c = 0; c < 6; c++)
            m.e[c] = {l[(18 * i + 2 * c) * HS + h], l[(18 * i + 2 * c + 1) * HS + h]};
        rebuild_row3(m);
        return m;
    }
    __device__ __forceinline__ a8<T> A(uint32_t h, uint32_t c0) const
    {
        a8<T> r;
#pragma unroll
        for (int a = 0; a < 8; a++) r.v[a] = l[(c0 + a) * HS + h];
        return r;
    }
};

// Kick forces at time t from U(t), phi(t) (lattice equations of motion, Sec. II.A):
//   F_i  = -t (Proj U_ij + Proj U_{i,-j}) + (1/t) i[phi->_i, phi]
//   F_pi = (1/t) sum_i (phi->_i + phi<-_i - 2 phi)
// Also returns the plaquette trace Re Tr U_12 and the scalar-gradient
// term sum_i |phi->_i - phi|^2 / 2 for the energy, and, with gv, stores
// G = Proj U_12 at byte offset gs of the plaquette buffer (plaq_on below).
// The stencil is organised by link: each of the four links touching x is
// loaded in one phase, every product it enters is formed there, and it is
// dropped, so at most two partial plaquettes stay in registers.
template <typename T, typename Src>
__device__ __forceinline__ void kick_forces(const Src& f, const Nbr& nb, T t, T inv_t, const a8<T>& PHI,
                                            a8<T>& F1, a8<T>& F2, a8<T>& Fpi, T* re_tr_p12 = nullptr,
                                            T* grad2 = nullptr, const View<T>* gv = nullptr, uint32_t gs = 0)
{
    m3<T> A12, A1m2, A2m1;
    a8<T> lap, c1, c2;
    T g2 = 0;
    {   // U_1(x): U_12 = [U_1 U_2(x+1)] ..., U_{1,-2} = [U_1 U_2(x+1-2)^+] ..., phi->_1
        const m3<T> U1 = f.U(nb.s, 0);
        A12 = mul(U1, f.U(nb.xp, 1));
        A1m2 = mul_adj(U1, f.U(nb.xpym, 1));
        const a8<T> f1 = transport(U1, f.A(nb.xp, kCompPhi));
        c1 = icomm(f1, PHI);
#pragma unroll
        for (int a = 0; a < 8; a++) {
            lap.v[a] = f1.v[a] - T(4) * PHI.v[a];
            const T d = f1.v[a] - PHI.v[a];
            g2 += T(0.5) * d * d;
        }
    }
    CPIC_PHASE();
    {   // U_2(x): U_12 = A12 [U_2 U_1(x+2)]^+, U_{2,-1} = [U_2 U_1(x-1+2)^+] ..., phi->_2
        const m3<T> U2 = f.U(nb.s, 1);
        const m3<T> P = mul_adj(A12, mul(U2, f.U(nb.yp, 0)));
        F1 = proj(P);
        if (gv) vA_st(*gv, gs, 0, F1);
#pragma unroll
        for (int a = 0; a < 8; a++) F2.v[a] = -F1.v[a];   // Proj U_21 = -Proj U_12
        if (re_tr_p12) *re_tr_p12 = P.e[0].re + P.e[4].re + P.e[8].re;
        A2m1 = mul_adj(U2, f.U(nb.xmyp, 0));
        const a8<T> f2 = transport(U2, f.A(nb.yp, kCompPhi));
        c2 = icomm(f2, PHI);
#pragma unroll
        for (int a = 0; a < 8; a++) {
            lap.v[a] += f2.v[a];
            const T d = f2.v[a] - PHI.v[a];
            g2 += T(0.5) * d * d;
        }
    }
    CPIC_PHASE();
    {   // U_2(x-2): U_{1,-2} = A1m2 [U_2(x-2)^+ U_1(x-2)]^+, phi<-_2
        const m3<T> U2ym = f.U(nb.ym, 1);
        const a8<T> p = proj(mul_adj(A1m2, adj_mul(U2ym, f.U(nb.ym, 0))));
        const a8<T> b2 = transport_adj(U2ym, f.A(nb.ym, kCompPhi));
#pragma unroll
        for (int a = 0; a < 8; a++) { F1.v[a] += p.v[a]; lap.v[a] += b2.v[a]; }
    }
    CPIC_PHASE();
    {   // U_1(x-1): U_{2,-1} = A2m1 [U_1(x-1)^+ U_2(x-1)]^+, phi<-_1
        const m3<T> U1xm = f.U(nb.xm, 0);
        const a8<T> p = proj(mul_adj(A2m1, adj_mul(U1xm, f.U(nb.xm, 1))));
        const a8<T> b1 = transport_adj(U1xm, f.A(nb.xm, kCompPhi));
#pragma unroll
        for (int a = 0; a < 8; a++) { F2.v[a] += p.v[a]; lap.v[a] += b1.v[a]; }
    }
#pragma unroll
    for (int a = 0; a < 8; a++) {
        F1.v[a] = -t * F1.v[a] + inv_t * c1.v[a];
        F2.v[a] = -t * F2.v[a] + inv_t * c2.v[a];
        Fpi.v[a] = inv_t * lap.v[a];
    }
    if (grad2) *grad2 = g2;
}

// The particle push and the force table take B_eta from the plaquette field
// G = Proj U_12 of every site (cellfields.h): with a plaquette buffer gpl
// ([8][V]), the field update stores G from the first step that reads it on
// (sc.n_plaq; at n = 0 the forces vanish with t = 1/t = 0, so the kick is
// still skipped while the plaquettes are formed).
template <typename T> __device__ __forceinline__ bool plaq_on(const T* gpl, const Schedule& sc, int n)
{
    return gpl != nullptr && n >= sc.n_plaq;
}

template <typename T>
__device__ __forceinline__ void field_step_body(const Fields<T>& in, const Fields<T>& out, T* gpl, int N, int bx,
                                                int by, int tile, const Schedule& sc, int* d_step)
{
    const int ntx = (N + bx - 1) / bx;
    const int x = (tile % ntx) * bx + (int)threadIdx.x, y = (tile / ntx) * by + (int)threadIdx.y;
    if (x >= N || y >= N) return;
    const int n = d_step[0];
    // hand the step to this step's push (which advances d_step[0])
    if (tile == 0 && threadIdx.x == 0 && threadIdx.y == 0) d_step[1] = n;
    const double td = n * sc.dt, thd = (n + 0.5) * sc.dt;
    const T t = T(td), inv_t = n > 0 ? T(1.0 / td) : T(0), dt = T(sc.dt);
    const T eps_drift = T(sc.dt / thd), phi_drift = T(sc.dt * thd);
    const bool kick = n > 0, reunit = is_reunit_step(sc, n);
    const uint32_t V = (uint32_t)N * N;
    const View<T> vi = make_view<T>(in.U, kRealsPerSite, V), vo = make_view<T>(out.U, kRealsPerSite, V);
    const Nbr nb = neighbours<T>(x, y, N);
    a8<T> PHI = vA(vi, nb.s, kCompPhi);
    a8<T> F1 = azero<T>(), F2 = azero<T>(), Fpi = azero<T>();
    const bool gon = plaq_on(gpl, sc, n);
    if (kick || gon) {
        const View<T> gv = make_view<T>(gpl, kPlaqReals, V);
        kick_forces<T>(GlobalSrc<T>{vi}, nb, t, inv_t, PHI, F1, F2, Fpi, nullptr, nullptr, gon ? &gv : nullptr, nb.s);
    }
    CPIC_PHASE();
    a8<T> E1 = vA(vi, nb.s, kCompE), E2 = vA(vi, nb.s, kCompE + 8), PI = vA(vi, nb.s, kCompPi);
#pragma unroll
    for (int a = 0; a < 8; a++) {
        E1.v[a] += dt * F1.v[a];
        E2.v[a] += dt * F2.v[a];
        PI.v[a] += dt * Fpi.v[a];
    }
    CPIC_PHASE();
    // drift: U_i <- exp(i (dt/t_half) E_i) U_i ; phi <- phi + dt t_half pi
    m3<T> U1 = mul(expi(E1, eps_drift), vU(vi, nb.s, 0));
    if (reunit) U1 = reunitarize(U1);
    vU_st(vo, nb.s, 0, U1);
    CPIC_PHASE();
    m3<T> U2 = mul(expi(E2, eps_drift), vU(vi, nb.s, 1));
    if (reunit) U2 = reunitarize(U2);
    vU_st(vo, nb.s, 1, U2);
#pragma unroll
    for (int a = 0; a < 8; a++) PHI.v[a] += phi_drift * PI.v[a];
    vA_st(vo, nb.s, kCompPhi, PHI);
    vA_st(vo, nb.s, kCompE, E1);
    vA_st(vo, nb.s, kCompE + 8, E2);
    vA_st(vo, nb.s, kCompPi, PI);
}

// ---------------------------------------------------------------- LDS halo-tile variant
// One workgroup of BX x BY threads owns a BX x BY tile.  It first stages the
// links and scalars of the tile and its one-site halo ring in LDS with
// coalesced loads (each global value read once per tile instead of once per
// stencil use), then every thread runs the stencil out of LDS; E and pi of
// its own site come straight from global memory.
template <typename T, int BX, int BY>
__device__ __forceinline__ void field_tile_body(const Fields<T>& in, const Fields<T>& out, T* gpl, int N, int tile,
                                                const Schedule& sc, int* d_step)
{
    constexpr int HX = BX + 2, HY = BY + 2, HS = HX * HY, NT = BX * BY, NC = 44;
    __shared__ T lds[NC * HS];
    const int ntx = (N + BX - 1) / BX;
    const int x0 = (tile % ntx) * BX, y0 = (tile / ntx) * BY;
    const int tid = (int)threadIdx.x;
    const uint32_t V = (uint32_t)N * N;
    const View<T> vi = make_view<T>(in.U, kRealsPerSite, V), vo = make_view<T>(out.U, kRealsPerSite, V);
    // stage: thread tid loads tile sites h = tid, tid + NT, ... (all 44 components)
#pragma unroll
    for (int h0 = 0; h0 < HS; h0 += NT) {
        const int h = h0 + tid;
        if (h < HS) {
            const int hy = h / HX, hx = h - hy * HX;
            const int gx = (x0 + hx - 1 + N) % N, gy = (y0 + hy - 1 + N) % N;
            const uint32_t go = (uint32_t)(gy * N + gx) * (uint32_t)sizeof(T);
            // (the slots of the links' third rows, 12..17 and 30..35, stay unused)
            T v[NC];
#pragma unroll
            for (int c = 0; c < NC; c++)
                if (c % 18 < 12 || c >= 36) v[c] = bld(vi, go, (uint32_t)c);
#pragma unroll
            for (int c = 0; c < NC; c++)
                if (c % 18 < 12 || c >= 36) lds[c * HS + h] = v[c];
        }
    }
    __syncthreads();
    const int tx = tid % BX, ty = tid / BX;
    const int x = x0 + tx, y = y0 + ty;
    if (x >= N || y >= N) return;
    const int n = d_step[0];
    if (tile == 0 && tid == 0) d_step[1] = n;  // the step of this step's push
    const double td = n * sc.dt, thd = (n + 0.5) * sc.dt;
    const T t = T(td), inv_t = n > 0 ? T(1.0 / td) : T(0), dt = T(sc.dt);
    const T eps_drift = T(sc.dt / thd), phi_drift = T(sc.dt * thd);
    const bool kick = n > 0, reunit = is_reunit_step(sc, n);
    const uint32_t hs = (uint32_t)((ty + 1) * HX + tx + 1);
    const Nbr nb{hs, hs + 1, hs - 1, hs + HX, hs - HX, hs + 1 - HX, hs - 1 + HX};
    const uint32_t gs = (uint32_t)(y * N + x) * (uint32_t)sizeof(T);
    const LdsSrc<T, HS> src{lds};
    a8<T> PHI = src.A(hs, kCompPhi);
    a8<T> F1 = azero<T>(), F2 = azero<T>(), Fpi = azero<T>();
    const bool gon = plaq_on(gpl, sc, n);
    if (kick || gon) {
        const View<T> gv = make_view<T>(gpl, kPlaqReals, V);
        kick_forces<T>(src, nb, t, inv_t, PHI, F1, F2, Fpi, nullptr, nullptr, gon ? &gv : nullptr, gs);
    }
    CPIC_PHASE();
    a8<T> E1 = vA(vi, gs, kCompE), E2 = vA(vi, gs, kCompE + 8), PI = vA(vi, gs, kCompPi);
#pragma unroll
    for (int a = 0; a < 8; a++) {
        E1.v[a] += dt * F1.v[a];
        E2.v[a] += dt * F2.v[a];
        PI.v[a] += dt * Fpi.v[a];
    }
    CPIC_PHASE();
    // drift: U_i <- exp(i (dt/t_half) E_i) U_i ; phi <- phi + dt t_half pi
    m3<T> U1 = mul(expi(E1, eps_drift), src.U(hs, 0));
    if (reunit) U1 = reunitarize(U1);
    vU_st(vo, gs, 0, U1);
    CPIC_PHASE();
    m3<T> U2 = mul(expi(E2, eps_drift), src.U(hs, 1));
    if (reunit) U2 = reunitarize(U2);
    vU_st(vo, gs, 1, U2);
#pragma unroll
    for (int a = 0; a < 8; a++) PHI.v[a] += phi_drift * PI.v[a];
    vA_st(vo, gs, kCompPhi, PHI);
    vA_st(vo, gs, kCompE, E1);
    vA_st(vo, gs, kCompE + 8, E2);
    vA_st(vo, gs, kCompPi, PI);
}

template <typename T, int BX, int BY>
__global__ __launch_bounds__(BX * BY) void field_tile_kernel(Fields<T> in, Fields<T> out, T* gpl, int N, int remap,
                                                             Schedule sc, int* d_step)
{
    const int nt = ((N + BX - 1) / BX) * ((N + BY - 1) / BY), tile = logical_block(nt, remap);
    if (tile < nt) field_tile_body<T, BX, BY>(in, out, gpl, N, tile, sc, d_step);
}

// ---------------------------------------------------------------- compressed-link LDS tiles
// (LdsLinks2, tiles.h)
template <typename T, int BX, int BY, int CP = 0>
__device__ __forceinline__ void field_ctile_body(const Fields<T>& in, const Fields<T>& out, T* gpl, int N, int tile,
                                                 const Schedule& sc, int* d_step)
{
    constexpr int HX = BX + 2, HS = HX * (BY + 2), NC = 24;
    __shared__ T lds[NC * HS];
    const int ntx = (N + BX - 1) / BX;
    const int x0 = (tile % ntx) * BX, y0 = (tile / ntx) * BY;
    const int tid = (int)threadIdx.x;
    const uint32_t V = (uint32_t)N * N;
    const View<T> vi = make_view<T>(in.U, kRealsPerSite, V), vo = make_view<T>(out.U, kRealsPerSite, V);
    stage_links2<T, BX, BY>(lds, vi, x0, y0, N, tid);
    __syncthreads();
    const int tx = tid % BX, ty = tid / BX;
    const int x = x0 + tx, y = y0 + ty;
    if (x >= N || y >= N) return;
    const int n = d_step[0];
    if (tile == 0 && tid == 0) d_step[1] = n;  // the step of this step's push
    const double td = n * sc.dt, thd = (n + 0.5) * sc.dt;
    const T t = T(td), inv_t = n > 0 ? T(1.0 / td) : T(0), dt = T(sc.dt);
    const T eps_drift = T(sc.dt / thd), phi_drift = T(sc.dt * thd);
    const bool kick = n > 0, reunit = is_reunit_step(sc, n);
    const uint32_t s = (uint32_t)((ty + 1) * HX + tx + 1);  // tile site
    const uint32_t xp = s + 1, xm = s - 1, yp = s + HX, ym = s - HX, xpym = s + 1 - HX, xmyp = s - 1 + HX;
    const Nbr g = neighbours<T>(x, y, N);                   // global sites (scalars, E, pi, outputs)
    const LdsLinks2<T, HS> L{lds};
    a8<T> PHI = vA(vi, g.s, kCompPhi);
    a8<T> F1 = azero<T>(), F2 = azero<T>(), Fpi = azero<T>();
    const bool gon = plaq_on(gpl, sc, n);
    if (kick || gon) {
        {   // U_12(x) = U_1(x) U_2(x+1) U_1(x+2)^+ U_2(x)^+
            m3<T> M = mul(L.U(s, 0), L.U(xp, 1));
            M = mul_adj(M, L.U(yp, 0));
            M = mul_adj(M, L.U(s, 1));
            F1 = proj(M);
            if (gon) vA_st(make_view<T>(gpl, kPlaqReals, V), g.s, 0, F1);
#pragma unroll
            for (int a = 0; a < 8; a++) F2.v[a] = -F1.v[a];
        }
        CPIC_PHASE();
        {   // U_{1,-2}(x) = U_1(x) U_2(x+1-2)^+ U_1(x-2)^+ U_2(x-2)
            m3<T> M = mul_adj(L.U(s, 0), L.U(xpym, 1));
            M = mul_adj(M, L.U(ym, 0));
            M = mul(M, L.U(ym, 1));
            const a8<T> p = proj(M);
#pragma unroll
            for (int a = 0; a < 8; a++) F1.v[a] += p.v[a];
        }
        CPIC_PHASE();
        {   // U_{2,-1}(x) = U_2(x) U_1(x-1+2)^+ U_2(x-1)^+ U_1(x-1)
            m3<T> M = mul_adj(L.U(s, 1), L.U(xmyp, 0));
            M = mul_adj(M, L.U(xm, 1));
            M = mul(M, L.U(xm, 0));
            const a8<T> p = proj(M);
#pragma unroll
            for (int a = 0; a < 8; a++) F2.v[a] += p.v[a];
        }
        CPIC_PHASE();
        a8<T> lap;
        {   // phi->_1, phi<-_1
            const a8<T> f1 = transport(L.U(s, 0), vA(vi, g.xp, kCompPhi));
            const a8<T> c1 = icomm(f1, PHI);
            const a8<T> b1 = transport_adj(L.U(xm, 0), vA(vi, g.xm, kCompPhi));
#pragma unroll
            for (int a = 0; a < 8; a++) {
                F1.v[a] = -t * F1.v[a] + inv_t * c1.v[a];
                lap.v[a] = f1.v[a] + b1.v[a] - T(4) * PHI.v[a];
            }
        }
        CPIC_PHASE();
        {   // phi->_2, phi<-_2
            const a8<T> f2 = transport(L.U(s, 1), vA(vi, g.yp, kCompPhi));
            const a8<T> c2 = icomm(f2, PHI);
            const a8<T> b2 = transport_adj(L.U(ym, 1), vA(vi, g.ym, kCompPhi));
#pragma unroll
            for (int a = 0; a < 8; a++) {
                F2.v[a] = -t * F2.v[a] + inv_t * c2.v[a];
                Fpi.v[a] = inv_t * (lap.v[a] + f2.v[a] + b2.v[a]);
            }
        }
    }
    CPIC_PHASE();
    a8<T> E1 = vA(vi, g.s, kCompE), E2 = vA(vi, g.s, kCompE + 8), PI = vA(vi, g.s, kCompPi);
#pragma unroll
    for (int a = 0; a < 8; a++) {
        E1.v[a] += dt * F1.v[a];
        E2.v[a] += dt * F2.v[a];
        PI.v[a] += dt * Fpi.v[a];
    }
    CPIC_PHASE();
    // drift: U_i <- exp(i (dt/t_half) E_i) U_i ; phi <- phi + dt t_half pi
    // CP: cache policy of the new links and phi, which only the next step's
    // field update reads, chosen by the host from the step's working set
    // (set_store_policy in capi.hip); the new E and pi, which this step's push
    // reads right after, keep the default policy.
    m3<T> U1 = mul(expi(E1, eps_drift), L.U(s, 0));
    if (reunit) U1 = reunitarize(U1);
    vU_st<T, CP>(vo, g.s, 0, U1);
    CPIC_PHASE();
    m3<T> U2 = mul(expi(E2, eps_drift), L.U(s, 1));
    if (reunit) U2 = reunitarize(U2);
    vU_st<T, CP>(vo, g.s, 1, U2);
#pragma unroll
    for (int a = 0; a < 8; a++) PHI.v[a] += phi_drift * PI.v[a];
    vA_st<T, CP>(vo, g.s, kCompPhi, PHI);
    vA_st(vo, g.s, kCompE, E1);
    vA_st(vo, g.s, kCompE + 8, E2);
    vA_st(vo, g.s, kCompPi, PI);
}

template <typename T, int BX, int BY, int CP>
__global__ __launch_bounds__(BX * BY) void field_ctile_kernel(Fields<T> in, Fields<T> out, T* gpl, int N, int remap,
                                                              Schedule sc, int* d_step)
{
    const int nt = ((N + BX - 1) / BX) * ((N + BY - 1) / BY), tile = logical_block(nt, remap);
    if (tile < nt) field_ctile_body<T, BX, BY, CP>(in, out, gpl, N, tile, sc, d_step);
}

// ---------------------------------------------------------------- link-parallel variant
// One thread per link: half-wavefront h of a wavefront handles direction i = h
// for the same 32 sites.  Thread (x, i) forms the two plaquettes of its link,
// U_ij(x) and U_{i,-j}(x), the transported scalar phi->_i and phi<-_i, updates
// E_i and drifts U_i; the pi force is the sum of both directions' scalar terms
// (one lane exchange, lanes l and l ^ 32), and the i = 0 thread writes phi, pi.
template <typename T>
__device__ __forceinline__ void field_link_body(const Fields<T>& in, const Fields<T>& out, T* gpl, int N, int bx,
                                                int by, int remap, const Schedule& sc, int* d_step)
{
    const int lane = (int)threadIdx.x & 63, wave = (int)threadIdx.x >> 6;
    const int i = lane >> 5, j = 1 - i;
    const int local = wave * 32 + (lane & 31);          // site within the block tile
    const int ntx = (N + bx - 1) / bx, nty = (N + by - 1) / by, ntiles = ntx * nty;
    int tile = blockIdx.x;
    if (remap) {
        const int per = (ntiles + 7) / 8;
        tile = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    }
    const int x = (tile % ntx) * bx + local % bx, y = (tile / ntx) * by + local / bx;
    const bool live = tile < ntiles && x < N && y < N;
    const int n = d_step[0];
    if (tile == 0 && threadIdx.x == 0) d_step[1] = n;  // the step of this step's push
    const double td = n * sc.dt, thd = (n + 0.5) * sc.dt;
    const T t = T(td), inv_t = n > 0 ? T(1.0 / td) : T(0), dt = T(sc.dt);
    const T eps_drift = T(sc.dt / thd), phi_drift = T(sc.dt * thd);
    const bool kick = n > 0, reunit = is_reunit_step(sc, n);
    const uint32_t V = (uint32_t)N * N;
    const View<T> vi = make_view<T>(in.U, kRealsPerSite, V), vo = make_view<T>(out.U, kRealsPerSite, V);
    constexpr uint32_t b = sizeof(T);
    const int xs = live ? x : 0, ys = live ? y : 0;
    auto site = [&](int dx, int dy) {
        int xx = xs + dx, yy = ys + dy;
        xx = xx < 0 ? xx + N : (xx >= N ? xx - N : xx);
        yy = yy < 0 ? yy + N : (yy >= N ? yy - N : yy);
        return (uint32_t)(yy * N + xx) * b;
    };
    // unit steps along i and j
    const int ix = i == 0 ? 1 : 0, iy = 1 - ix, jx = iy, jy = ix;
    const uint32_t s = site(0, 0);
    // the link of direction d at byte offset o: components start at 18 d
    auto link = [&](const View<T>& v, uint32_t o, int d) {
        m3<T> m;
#pragma unroll
        for (int c = 0; c < 6; c++)
            m.e[c] = {bld(v, o + (uint32_t)(18 * d) * v.cs, 2 * c), bld(v, o + (uint32_t)(18 * d) * v.cs, 2 * c + 1)};
        rebuild_row3(m);
        return m;
    };
    const a8<T> PHI = vA(vi, s, kCompPhi);
    a8<T> F = azero<T>(), lap = azero<T>();
    const bool gon = plaq_on(gpl, sc, n) && live;
    if (kick || gon) {
        {   // U_ij(x) = U_i(x) U_j(x+i) [U_j(x) U_i(x+j)]^+ (G from the i = 0 thread)
            const m3<T> Pm = mul_adj(mul(link(vi, s, i), link(vi, site(ix, iy), j)),
                                     mul(link(vi, s, j), link(vi, site(jx, jy), i)));
            F = proj(Pm);
            if (gon && i == 0) vA_st(make_view<T>(gpl, kPlaqReals, V), s, 0, F);
        }
        CPIC_PHASE();
        {   // U_{i,-j}(x) = U_i(x) U_j(x+i-j)^+ [U_j(x-j)^+ U_i(x-j)]^+
            const uint32_t smj = site(-jx, -jy);
            const m3<T> Pm = mul_adj(mul_adj(link(vi, s, i), link(vi, site(ix - jx, iy - jy), j)),
                                     adj_mul(link(vi, smj, j), link(vi, smj, i)));
            const a8<T> p = proj(Pm);
#pragma unroll
            for (int a = 0; a < 8; a++) F.v[a] = -t * (F.v[a] + p.v[a]);
        }
        CPIC_PHASE();
        {   // phi->_i and phi<-_i
            const a8<T> fw = transport(link(vi, s, i), vA(vi, site(ix, iy), kCompPhi));
            const uint32_t smi = site(-ix, -iy);
            const a8<T> bw = transport_adj(link(vi, smi, i), vA(vi, smi, kCompPhi));
            const a8<T> cm = icomm(fw, PHI);
#pragma unroll
            for (int a = 0; a < 8; a++) {
                F.v[a] += inv_t * cm.v[a];
                lap.v[a] = fw.v[a] + bw.v[a] - T(2) * PHI.v[a];
            }
        }
        if (!kick) F = lap = azero<T>();
    }
    // pi force: add the other direction's scalar terms
#pragma unroll
    for (int a = 0; a < 8; a++) lap.v[a] += __shfl_xor(lap.v[a], 32, 64);
    CPIC_PHASE();
    a8<T> Ei = vA(vi, s, kCompE + 8 * i), PI = vA(vi, s, kCompPi);
#pragma unroll
    for (int a = 0; a < 8; a++) {
        Ei.v[a] += dt * F.v[a];
        PI.v[a] += dt * inv_t * lap.v[a];
    }
    m3<T> Ui = mul(expi(Ei, eps_drift), link(vi, s, i));
    if (reunit) Ui = reunitarize(Ui);
    if (!live) return;
    vU_st(vo, s + (uint32_t)(18 * i) * vo.cs, 0, Ui);
    vA_st(vo, s, kCompE + 8 * i, Ei);
    if (i == 0) {
        a8<T> ph = PHI;
#pragma unroll
        for (int a = 0; a < 8; a++) ph.v[a] += phi_drift * PI.v[a];
        vA_st(vo, s, kCompPhi, ph);
        vA_st(vo, s, kCompPi, PI);
    }
}

template <typename T>
__global__ __launch_bounds__(256) void field_link_kernel(Fields<T> in, Fields<T> out, T* gpl, int N, int bx, int by,
                                                         int remap, Schedule sc, int* d_step)
{
    field_link_body<T>(in, out, gpl, N, bx, by, remap, sc, d_step);
}
template <typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void field_link_kernel_w2(
    Fields<T> in, Fields<T> out, T* gpl, int N, int bx, int by, int remap, Schedule sc, int* d_step)
{
    field_link_body<T>(in, out, gpl, N, bx, by, remap, sc, d_step);
}
template <typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 3))) void field_link_kernel_w3(
    Fields<T> in, Fields<T> out, T* gpl, int N, int bx, int by, int remap, Schedule sc, int* d_step)
{
    field_link_body<T>(in, out, gpl, N, bx, by, remap, sc, d_step);
}

// Occupancy variants: W waves per SIMD requested from the register
// allocator (W = 1: no request).  Chosen per lattice size and precision by
// the launch tuner.
__device__ __forceinline__ int field_tiles(int N, int bx, int by) { return ((N + bx - 1) / bx) * ((N + by - 1) / by); }

template <typename T>
__global__ __launch_bounds__(256) void field_step_kernel(Fields<T> in, Fields<T> out, T* gpl, int N, int bx, int by,
                                                         int remap, Schedule sc, int* d_step)
{
    const int nt = field_tiles(N, bx, by), tile = logical_block(nt, remap);
    if (tile < nt) field_step_body<T>(in, out, gpl, N, bx, by, tile, sc, d_step);
}
#define CPIC_FIELD_VARIANT(W)                                                                                     \
    template <typename T>                                                                                         \
    __global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(W, W))) void field_step_kernel_w##W(    \
        Fields<T> in, Fields<T> out, T* gpl, int N, int bx, int by, int remap, Schedule sc, int* d_step)          \
    {                                                                                                             \
        const int nt = field_tiles(N, bx, by), tile = logical_block(nt, remap);                                   \
        if (tile < nt) field_step_body<T>(in, out, gpl, N, bx, by, tile, sc, d_step);                             \
    }
CPIC_FIELD_VARIANT(2)
CPIC_FIELD_VARIANT(3)
CPIC_FIELD_VARIANT(4)
#undef CPIC_FIELD_VARIANT

// ---------------------------------------------------------------- batched events
// One launch advances every event of a launch group by one step: logical
// block g works on tile map[g].y of event map[g].x; all events share the tile
// shape.
template <typename T, int BX, int BY>
__global__ __launch_bounds__(BX * BY) void batch_field_kernel(const EventDesc* __restrict__ ev,
                                                              const int2* __restrict__ map, int total, int remap)
{
    const int g = logical_block(total, remap);
    if (g >= total) return;
    // the work item is uniform over the workgroup: keep it (and every address
    // derived from it) in scalar registers
    const int2 m = map[g];
    const int e = __builtin_amdgcn_readfirstlane(m.x), tile = __builtin_amdgcn_readfirstlane(m.y);
    const EventDesc& d = ev[e];
    const int parity = __builtin_amdgcn_readfirstlane((d.d_step[0] & 1) ^ d.flip);
    const Fields<T> A = fields_at<T>(d.f[parity], d.N * d.N), B = fields_at<T>(d.f[parity ^ 1], d.N * d.N);
    field_ctile_body<T, BX, BY>(A, B, static_cast<T*>(d.gpl), d.N, tile, d.pa.sc, d.d_step);
}

template <typename T, int BX, int BY>
static void launch_batch_field_t(const EventDesc* ev, const int2* map, int total_tiles, int remap, hipStream_t st)
{
    const int grid = remap ? 8 * ((total_tiles + 7) / 8) : total_tiles;
    hipLaunchKernelGGL((batch_field_kernel<T, BX, BY>), dim3(grid), dim3(BX * BY), 0, st, ev, map, total_tiles, remap);
}

// compressed-link LDS tiles (variant 3) of the instantiated shapes
template <typename T>
hipError_t launch_batch_field(const EventDesc* ev, const int2* map, int total_tiles, const LaunchCfg& cfg,
                              hipStream_t st)
{
    if (cfg.split != 3 || total_tiles <= 0) return hipErrorInvalidValue;
    const int r = cfg.xcd_remap;
    if (cfg.bx == 64 && cfg.by == 4) launch_batch_field_t<T, 64, 4>(ev, map, total_tiles, r, st);
    else if (cfg.bx == 32 && cfg.by == 8) launch_batch_field_t<T, 32, 8>(ev, map, total_tiles, r, st);
    else if (cfg.bx == 16 && cfg.by == 16) launch_batch_field_t<T, 16, 16>(ev, map, total_tiles, r, st);
    else if (cfg.bx == 32 && cfg.by == 4) launch_batch_field_t<T, 32, 4>(ev, map, total_tiles, r, st);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}
template hipError_t launch_batch_field<double>(const EventDesc*, const int2*, int, const LaunchCfg&, hipStream_t);
template hipError_t launch_batch_field<float>(const EventDesc*, const int2*, int, const LaunchCfg&, hipStream_t);

template <typename T, int BX, int BY>
static hipError_t launch_tile(const Fields<T>& in, const Fields<T>& out, T* gpl, int N, const Schedule& sc,
                              int* d_step, int remap, hipStream_t st, const KTimer& tm)
{
    const int ntiles = ((N + BX - 1) / BX) * ((N + BY - 1) / BY);
    const dim3 g(remap ? 8 * ((ntiles + 7) / 8) : ntiles), blk(BX * BY);
    klaunch(tm, field_tile_kernel<T, BX, BY>, g, blk, st, in, out, gpl, N, remap, sc, d_step);
    return hipGetLastError();
}

template <typename T, int BX, int BY>
static hipError_t launch_ctile(const Fields<T>& in, const Fields<T>& out, T* gpl, int N, const Schedule& sc,
                               int* d_step, int remap, int nt_store, hipStream_t st, const KTimer& tm)
{
    const int ntiles = ((N + BX - 1) / BX) * ((N + BY - 1) / BY);
    const dim3 g(remap ? 8 * ((ntiles + 7) / 8) : ntiles), blk(BX * BY);
    if (nt_store)
        klaunch(tm, field_ctile_kernel<T, BX, BY, kStoreNT>, g, blk, st, in, out, gpl, N, remap, sc, d_step);
    else
        klaunch(tm, field_ctile_kernel<T, BX, BY, 0>, g, blk, st, in, out, gpl, N, remap, sc, d_step);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_field_step(const Fields<T>& in, const Fields<T>& out, T* gpl, int N, const Schedule& sc,
                             int* d_step, const LaunchCfg& cfg, hipStream_t st, const KTimer& tm)
{
    if (cfg.bx <= 0 || cfg.by <= 0 || cfg.waves < 1 || cfg.waves > 4) return hipErrorInvalidValue;
    if (cfg.split == 3 || cfg.split == 4) {
        // compressed-link LDS tiles of the instantiated shapes (variant 4, the
        // fused step, runs as these when it has no particles to push)
        const int r = cfg.xcd_remap, nts = cfg.nt_store;
        if (cfg.bx == 64 && cfg.by == 4) return launch_ctile<T, 64, 4>(in, out, gpl, N, sc, d_step, r, nts, st, tm);
        if (cfg.bx == 32 && cfg.by == 8) return launch_ctile<T, 32, 8>(in, out, gpl, N, sc, d_step, r, nts, st, tm);
        if (cfg.bx == 16 && cfg.by == 16) return launch_ctile<T, 16, 16>(in, out, gpl, N, sc, d_step, r, nts, st, tm);
        if (cfg.bx == 32 && cfg.by == 4) return launch_ctile<T, 32, 4>(in, out, gpl, N, sc, d_step, r, nts, st, tm);
        if (cfg.bx == 64 && cfg.by == 8) return launch_ctile<T, 64, 8>(in, out, gpl, N, sc, d_step, r, nts, st, tm);
        if (cfg.bx == 8 && cfg.by == 8) return launch_ctile<T, 8, 8>(in, out, gpl, N, sc, d_step, r, nts, st, tm);
        return hipErrorInvalidValue;
    }
    if (cfg.split == 2) {
        // LDS halo tiles of the instantiated shapes
        const int r = cfg.xcd_remap;
        if (cfg.bx == 64 && cfg.by == 4) return launch_tile<T, 64, 4>(in, out, gpl, N, sc, d_step, r, st, tm);
        if (cfg.bx == 32 && cfg.by == 4) return launch_tile<T, 32, 4>(in, out, gpl, N, sc, d_step, r, st, tm);
        if (cfg.bx == 64 && cfg.by == 2) return launch_tile<T, 64, 2>(in, out, gpl, N, sc, d_step, r, st, tm);
        if (cfg.bx == 32 && cfg.by == 8) return launch_tile<T, 32, 8>(in, out, gpl, N, sc, d_step, r, st, tm);
        if (cfg.bx == 16 && cfg.by == 8) return launch_tile<T, 16, 8>(in, out, gpl, N, sc, d_step, r, st, tm);
        return hipErrorInvalidValue;
    }
    if (cfg.split) {
        // 128 sites (256 link threads) per block
        if (cfg.bx * cfg.by != 128 || cfg.bx % 32 != 0) return hipErrorInvalidValue;
        const int ntiles = ((N + cfg.bx - 1) / cfg.bx) * ((N + cfg.by - 1) / cfg.by);
        const dim3 g(cfg.xcd_remap ? 8 * ((ntiles + 7) / 8) : ntiles), blk(256);
        switch (cfg.waves) {
        case 2: klaunch(tm, field_link_kernel_w2<T>, g, blk, st, in, out, gpl, N, cfg.bx, cfg.by, cfg.xcd_remap, sc, d_step); break;
        case 3: klaunch(tm, field_link_kernel_w3<T>, g, blk, st, in, out, gpl, N, cfg.bx, cfg.by, cfg.xcd_remap, sc, d_step); break;
        default: klaunch(tm, field_link_kernel<T>, g, blk, st, in, out, gpl, N, cfg.bx, cfg.by, cfg.xcd_remap, sc, d_step);
        }
        return hipGetLastError();
    }
    if (cfg.bx * cfg.by > 256) return hipErrorInvalidValue;
    const int ntx = (N + cfg.bx - 1) / cfg.bx, nty = (N + cfg.by - 1) / cfg.by;
    const int ntiles = ntx * nty;
    const int grid = cfg.xcd_remap ? 8 * ((ntiles + 7) / 8) : ntiles;
    const dim3 g(grid), b(cfg.bx, cfg.by);
    switch (cfg.waves) {
    case 2: klaunch(tm, field_step_kernel_w2<T>, g, b, st, in, out, gpl, N, cfg.bx, cfg.by, cfg.xcd_remap, sc, d_step); break;
    case 3: klaunch(tm, field_step_kernel_w3<T>, g, b, st, in, out, gpl, N, cfg.bx, cfg.by, cfg.xcd_remap, sc, d_step); break;
    case 4: klaunch(tm, field_step_kernel_w4<T>, g, b, st, in, out, gpl, N, cfg.bx, cfg.by, cfg.xcd_remap, sc, d_step); break;
    default: klaunch(tm, field_step_kernel<T>, g, b, st, in, out, gpl, N, cfg.bx, cfg.by, cfg.xcd_remap, sc, d_step);
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------ diagnostics
// Per block: [sum |G|^2, max |G|, K_T, K_L, V_B, V_phi, max |U U^+ - 1|, sum |U U^+ - 1|^2]
// with the momenta averaged to integer time n: E(n) = E(n-1/2) + (dt/2) F(n).
// Without ENERGIES (the drift watchdog, which reads the Gauss and unitarity
// columns) the energy columns stay 0; every state array still enters the
// sums of columns 0 and 7, so a non-finite value anywhere shows there.
constexpr int kDiagCols = 8;

template <typename T, bool ENERGIES>
__global__ __launch_bounds__(256) void field_diag_kernel(Fields<T> f, int N, T t, T inv_t, T half_dt, int n,
                                                         double* partials)
{
    const int V = N * N;
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    double v[kDiagCols] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (s < V) {
        const int x = s % N, y = s / N;
        const View<T> vf = make_view<T>(f.U, kRealsPerSite, (uint32_t)V);
        const Nbr nb = neighbours<T>(x, y, N);
        const a8<T> PHI = vA(vf, nb.s, kCompPhi), PI = vA(vf, nb.s, kCompPi);
        const a8<T> E1 = vA(vf, nb.s, kCompE), E2 = vA(vf, nb.s, kCompE + 8);
        // Gauss residual, sum_i [E_i(x) - U_i(x-i)^+ E_i(x-i) U_i(x-i)] + i[phi, pi]
        const a8<T> g1 = transport_adj(vU(vf, nb.xm, 0), vA(vf, nb.xm, kCompE));
        const a8<T> g2 = transport_adj(vU(vf, nb.ym, 1), vA(vf, nb.ym, kCompE + 8));
        const a8<T> gc = icomm(PHI, PI);
        double G2 = 0;
        for (int a = 0; a < 8; a++) {
            const double g = (double)E1.v[a] - g1.v[a] + E2.v[a] - g2.v[a] + gc.v[a];
            G2 += g * g;
        }
        v[0] = G2;
        v[1] = sqrt(G2);
        if constexpr (ENERGIES) {
        a8<T> F1, F2, Fpi;
        T retr = 0, grad2 = 0;
        kick_forces<T>(GlobalSrc<T>{vf}, nb, t, inv_t, PHI, F1, F2, Fpi, &retr, &grad2);
        const T h = n > 0 ? half_dt : T(0);
        double e2 = 0, p2 = 0;
        for (int a = 0; a < 8; a++) {
            const double ea = E1.v[a] + h * F1.v[a], eb = E2.v[a] + h * F2.v[a], pa = PI.v[a] + h * Fpi.v[a];
            e2 += 0.5 * (ea * ea + eb * eb);
            p2 += 0.5 * pa * pa;
        }
        v[2] = (double)inv_t * e2;
        v[3] = (double)t * p2;
        v[4] = 2.0 * (double)t * (3.0 - (double)retr);
        v[5] = (double)inv_t * (double)grad2;
        }
        double umax = 0, usq = 0;
        for (int i = 0; i < 2; i++) {
            const m3<T> u = vU(vf, nb.s, i);
            const m3<T> w = mul_adj(u, u);
            for (int c = 0; c < 9; c++) {
                const double dr = (double)w.e[c].re - ((c % 4) == 0 ? 1.0 : 0.0), di = w.e[c].im;
                const double d = sqrt(dr * dr + di * di);
                umax = fmax(umax, d);
                usq += d * d;
            }
        }
        v[6] = umax;
        v[7] = usq;
    }
    block_reduce_store<kDiagCols>(v, (1u << 1) | (1u << 6), partials + (size_t)blockIdx.x * kDiagCols);
}

template <typename T>
hipError_t launch_field_diag(const Fields<T>& f, int N, double dt, int n, double* partials, int nblk_cap,
                             int* nblk_out, hipStream_t st, bool energies)
{
    const int V = N * N, nblk = (V + 255) / 256;
    if (nblk > nblk_cap) return hipErrorInvalidValue;
    *nblk_out = nblk;
    const double t = n * dt;
    if (energies)
        hipLaunchKernelGGL((field_diag_kernel<T, true>), dim3(nblk), dim3(256), 0, st, f, N, T(t),
                           T(n > 0 ? 1.0 / t : 0.0), T(0.5 * dt), n, partials);
    else
        hipLaunchKernelGGL((field_diag_kernel<T, false>), dim3(nblk), dim3(256), 0, st, f, N, T(t),
                           T(n > 0 ? 1.0 / t : 0.0), T(0.5 * dt), n, partials);
    return hipGetLastError();
}

template hipError_t launch_field_step<double>(const Fields<double>&, const Fields<double>&, double*, int,
                                              const Schedule&, int*, const LaunchCfg&, hipStream_t, const KTimer&);
template hipError_t launch_field_step<float>(const Fields<float>&, const Fields<float>&, float*, int, const Schedule&,
                                             int*, const LaunchCfg&, hipStream_t, const KTimer&);
template hipError_t launch_field_diag<double>(const Fields<double>&, int, double, int, double*, int, int*,
                                              hipStream_t, bool);
template hipError_t launch_field_diag<float>(const Fields<float>&, int, double, int, double*, int, int*,
                                             hipStream_t, bool);

}  // namespace cpic
