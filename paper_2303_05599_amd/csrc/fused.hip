// fused.hip -- the field update and the particle push of one step in one pass
// over lattice tiles (Sec. II.A leapfrog, Sec. III.B push).
//
// The particle records are ordered by the tiles of this kernel (sort.hip), so
// the workgroup that updates a tile also owns the particles that were in it at
// the last reordering (the tile's range of records).  After the kick and drift
// of its sites, done as in the compressed-link tile kernel of field.hip, the
// workgroup evaluates the six colour fields at t_n at every site of the tile
// (the interpolations of Sec. III.B) from values it already holds:
//   E_i   = (1/4t) [S_i(c) + U_i(c-i)^+ S_i(c-i) U_i(c-i)],
//           S_i = E_i(n-1/2) + E_i(n+1/2): the site thread has S_i(c) from its
//           kick; the thread of c-i transports its own S_i and hands it over
//           through LDS.  For the column left of the tile and the row below it
//           the kicks of E_x and E_y are redone from the staged halo of links
//           (both plaquettes of those links lie inside it).
//   E_eta = [pi(n-1/2) + pi(n+1/2)] / 2 from the site's own kick.
//   B_x = -(1/2t) D_y, B_y = +(1/2t) D_x with D_i = phi->_i - phi<-_i, the
//           transported scalars the kick has formed anyway.
//   B_eta = -(1/4) Proj of the four counter-clockwise clover leaves: U_12 and
//           U_{2,-1} are plaquettes of the kick, U_{-2,1} = U_{1,-2}^+ is the
//           third, and the fourth, U_{-1,-2}, is formed from the halo.
// The fields go to the particle lanes through LDS (the electric ones, then
// the magnetic ones, in the space the links occupied), one particle per
// thread, so the particle records are read and written once, contiguously,
// and no field is read back from memory.  Particles that have left the tile
// since the last reordering are listed for the straggler push that follows
// (the gather push of push.hip with B_eta from the links).
//
// Broadening sums: each tile writes the sums of its particles (fixed-order
// block reduction) and each straggler block the sums of its stragglers, into
// partials[slot][ntiles + straggler blocks][4].
#include "internal.h"
#include "reduce.h"
#include "tiles.h"
#include "wong.h"

namespace cpic {

// S_x = E_x(n-1/2) + E_x(n+1/2) at tile site h of the halo from its kick
//   E_x(n+1/2) = E_x(n-1/2) + dt [-t (Proj U_12 + Proj U_{1,-2}) + (1/t) i[phi->_x, phi]]
// in the operation order of the site kick (field.hip), gs the site's and gxp
// its +x neighbour's byte offsets in the buffer set
template <typename T, int HS, int HX>
__device__ __forceinline__ a8<T> halo_Sx(const LdsLinks2<T, HS>& L, uint32_t h, const View<T>& vi, uint32_t gs,
                                         uint32_t gxp, T t, T inv_t, T dt)
{
    a8<T> F;
    {
        m3<T> M = mul(L.U(h, 0), L.U(h + 1, 1));
        M = mul_adj(M, L.U(h + HX, 0));
        M = mul_adj(M, L.U(h, 1));
        F = proj(M);
    }
    CPIC_PHASE();
    {
        m3<T> M = mul_adj(L.U(h, 0), L.U(h + 1 - HX, 1));
        M = mul_adj(M, L.U(h - HX, 0));
        M = mul(M, L.U(h - HX, 1));
        const a8<T> p = proj(M);
#pragma unroll
        for (int a = 0; a < 8; a++) F.v[a] += p.v[a];
    }
    CPIC_PHASE();
    const a8<T> c1 = icomm(transport(L.U(h, 0), vA(vi, gxp, kCompPhi)), vA(vi, gs, kCompPhi));
    const a8<T> E = vA(vi, gs, kCompE);
    a8<T> S;
#pragma unroll
    for (int a = 0; a < 8; a++) {
        F.v[a] = -t * F.v[a] + inv_t * c1.v[a];
        S.v[a] = E.v[a] + (E.v[a] + dt * F.v[a]);
    }
    return S;
}
// S_y at tile site h of the halo:
//   E_y(n+1/2) = E_y(n-1/2) + dt [-t (-Proj U_12 + Proj U_{2,-1}) + (1/t) i[phi->_y, phi]]
template <typename T, int HS, int HX>
__device__ __forceinline__ a8<T> halo_Sy(const LdsLinks2<T, HS>& L, uint32_t h, const View<T>& vi, uint32_t gs,
                                         uint32_t gyp, T t, T inv_t, T dt)
{
    a8<T> F;
    {
        m3<T> M = mul(L.U(h, 0), L.U(h + 1, 1));
        M = mul_adj(M, L.U(h + HX, 0));
        M = mul_adj(M, L.U(h, 1));
        const a8<T> g = proj(M);
#pragma unroll
        for (int a = 0; a < 8; a++) F.v[a] = -g.v[a];
    }
    CPIC_PHASE();
    {
        m3<T> M = mul_adj(L.U(h, 1), L.U(h - 1 + HX, 0));
        M = mul_adj(M, L.U(h - 1, 1));
        M = mul(M, L.U(h - 1, 0));
        const a8<T> p = proj(M);
#pragma unroll
        for (int a = 0; a < 8; a++) F.v[a] += p.v[a];
    }
    CPIC_PHASE();
    const a8<T> c2 = icomm(transport(L.U(h, 1), vA(vi, gyp, kCompPhi)), vA(vi, gs, kCompPhi));
    const a8<T> E = vA(vi, gs, kCompE + 8);
    a8<T> S;
#pragma unroll
    for (int a = 0; a < 8; a++) {
        F.v[a] = -t * F.v[a] + inv_t * c2.v[a];
        S.v[a] = E.v[a] + (E.v[a] + dt * F.v[a]);
    }
    return S;
}

// One tile of BX x BY sites and its particles.  CP: cache policy of the new
// state (as the compressed-tile field kernel).
template <typename T, int BX, int BY, int CP>
__global__ __launch_bounds__(BX * BY) void fused_kernel(Fields<T> in, Fields<T> out, int N, int remap, Parts<T> P,
                                                        PushArgs a, TileParts tp, int* d_step, double* partials,
                                                        int ngroups, int* err)
{
    constexpr int HX = BX + 2, HS = HX * (BY + 2), NT = BX * BY, NC = 24, NW = NT / 64;
    static_assert(NT % 64 == 0, "whole wavefronts per tile");
    // the halo of links, then the transported S_i of the tile and its left
    // column / bottom row ([8][(BX+1) BY] then [8][BX (BY+1)]), then the
    // field table of the particle lanes ([24][NT])
    static_assert(16 * NT + 8 * (BX + BY) <= NC * HS && 24 * NT <= NC * HS, "LDS reuse");
    __shared__ T lds[NC * HS];
    __shared__ int wcount[NW];
    const int ntx = (N + BX - 1) / BX, nt = ntx * ((N + BY - 1) / BY);
    const int tile = logical_block(nt, remap);
    if (tile >= nt) return;
    const int x0 = (tile % ntx) * BX, y0 = (tile / ntx) * BY;
    const int tid = (int)threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t V = (uint32_t)N * N;
    const View<T> vi = make_view<T>(in.U, kRealsPerSite, V), vo = make_view<T>(out.U, kRealsPerSite, V);
    stage_links2<T, BX, BY>(lds, vi, x0, y0, N, tid);
    const int n = d_step[0];
    if (tile == 0 && tid == 0) d_step[1] = n;  // the step of the straggler push
    const bool pstep = n >= a.sc.n_form && n < a.sc.n_max;
    // the tile's records (kept inside [0, np], so that no ordering can send
    // a store out of the straggler list)
    const int p1 = pstep ? min(max(tp.tile_start[tile + 1], 0), a.np) : 0;
    const int p0 = pstep ? min(max(tp.tile_start[tile], 0), p1) : 0;
    const bool tpush = p1 > p0;  // uniform over the block
    __syncthreads();
    const int tx = tid % BX, ty = tid / BX;
    // sites beyond the lattice (a ragged last tile) compute on a valid site
    // and store nothing
    const bool inside = x0 + tx < N && y0 + ty < N;
    const int x = inside ? x0 + tx : x0, y = inside ? y0 + ty : y0;
    const double td = n * a.sc.dt, thd = (n + 0.5) * a.sc.dt;
    const T t = T(td), inv_t = n > 0 ? T(1.0 / td) : T(0), dt = T(a.sc.dt);
    const T eps_drift = T(a.sc.dt / thd), phi_drift = T(a.sc.dt * thd);
    const bool kick = n > 0, reunit = is_reunit_step(a.sc, n);
    const uint32_t s = (uint32_t)((ty + 1) * HX + tx + 1);
    const uint32_t xp = s + 1, xm = s - 1, yp = s + HX, ym = s - HX, xpym = s + 1 - HX, xmyp = s - 1 + HX;
    const Nbr g = neighbours<T>(x, y, N);
    const LdsLinks2<T, HS> L{lds};
    a8<T> PHI = vA(vi, g.s, kCompPhi);
    a8<T> F1 = azero<T>(), F2 = azero<T>(), Fpi = azero<T>();
    a8<T> BE = azero<T>();  // the clover sum (particle steps only)
    if (kick || tpush) {
        {   // U_12
            m3<T> M = mul(L.U(s, 0), L.U(xp, 1));
            M = mul_adj(M, L.U(yp, 0));
            M = mul_adj(M, L.U(s, 1));
            F1 = proj(M);
#pragma unroll
            for (int q = 0; q < 8; q++) {
                F2.v[q] = -F1.v[q];
                BE.v[q] = F1.v[q];
            }
        }
        CPIC_PHASE();
        {   // U_{1,-2} (= U_{-2,1}^+, the clover leaf with the opposite sign)
            m3<T> M = mul_adj(L.U(s, 0), L.U(xpym, 1));
            M = mul_adj(M, L.U(ym, 0));
            M = mul(M, L.U(ym, 1));
            const a8<T> p = proj(M);
#pragma unroll
            for (int q = 0; q < 8; q++) {
                F1.v[q] += p.v[q];
                BE.v[q] -= p.v[q];
            }
        }
        CPIC_PHASE();
        {   // U_{2,-1}
            m3<T> M = mul_adj(L.U(s, 1), L.U(xmyp, 0));
            M = mul_adj(M, L.U(xm, 1));
            M = mul(M, L.U(xm, 0));
            const a8<T> p = proj(M);
#pragma unroll
            for (int q = 0; q < 8; q++) {
                F2.v[q] += p.v[q];
                BE.v[q] += p.v[q];
            }
        }
        CPIC_PHASE();
        a8<T> lap;
        {
            const a8<T> f1 = transport(L.U(s, 0), vA(vi, g.xp, kCompPhi));
            const a8<T> c1 = icomm(f1, PHI);
            const a8<T> b1 = transport_adj(L.U(xm, 0), vA(vi, g.xm, kCompPhi));
#pragma unroll
            for (int q = 0; q < 8; q++) {
                F1.v[q] = -t * F1.v[q] + inv_t * c1.v[q];
                lap.v[q] = f1.v[q] + b1.v[q] - T(4) * PHI.v[q];
            }
        }
        CPIC_PHASE();
        {
            const a8<T> f2 = transport(L.U(s, 1), vA(vi, g.yp, kCompPhi));
            const a8<T> c2 = icomm(f2, PHI);
            const a8<T> b2 = transport_adj(L.U(ym, 1), vA(vi, g.ym, kCompPhi));
#pragma unroll
            for (int q = 0; q < 8; q++) {
                F2.v[q] = -t * F2.v[q] + inv_t * c2.v[q];
                Fpi.v[q] = inv_t * (lap.v[q] + f2.v[q] + b2.v[q]);
            }
        }
    }
    CPIC_PHASE();
    a8<T> E1 = vA(vi, g.s, kCompE), E2 = vA(vi, g.s, kCompE + 8), PI = vA(vi, g.s, kCompPi);
#pragma unroll
    for (int q = 0; q < 8; q++) {
        E1.v[q] += dt * F1.v[q];
        E2.v[q] += dt * F2.v[q];
        PI.v[q] += dt * Fpi.v[q];
    }
    CPIC_PHASE();
    {   // drift: U_i <- exp(i (dt/t_half) E_i) U_i ; phi <- phi + dt t_half pi
        m3<T> U1 = mul(expi(E1, eps_drift), L.U(s, 0));
        if (reunit) U1 = reunitarize(U1);
        if (inside) vU_st<T, CP>(vo, g.s, 0, U1);
    }
    CPIC_PHASE();
    {
        m3<T> U2 = mul(expi(E2, eps_drift), L.U(s, 1));
        if (reunit) U2 = reunitarize(U2);
        if (inside) vU_st<T, CP>(vo, g.s, 1, U2);
    }
    if (inside) {
        a8<T> PH = PHI;
#pragma unroll
        for (int q = 0; q < 8; q++) PH.v[q] += phi_drift * PI.v[q];
        vA_st<T, CP>(vo, g.s, kCompPhi, PH);
        vA_st<T, CP>(vo, g.s, kCompE, E1);
        vA_st<T, CP>(vo, g.s, kCompE + 8, E2);
        vA_st<T, CP>(vo, g.s, kCompPi, PI);
    }
    if (!pstep) return;  // uniform: no particle work before formation or after the end

    // ---- the colour fields at the tile's sites (tiles with particles), in an
    // order that keeps few values live: the halo kicks, S_i, the fourth leaf,
    // the magnetic fields; then S_i go through LDS to the sites c+i, which
    // transport them with U_i(c) read again from memory (cached)
    const bool eonly = a.is_static != 0;
    a8<T> S1 = azero<T>(), S2 = azero<T>(), SH = azero<T>();
    a8<T> GX = azero<T>(), GY = azero<T>();
    if (tpush) {
        if (kick) {
            CPIC_PHASE();
            // S at the column left of the tile (threads 0 .. BY-1) and at the
            // row below it (threads BY .. BY+BX-1)
            if (tid < BY) {
                const uint32_t h = (uint32_t)((tid + 1) * HX);
                const int hy = (y0 + tid) % N, hx = (x0 - 1 + N) % N;
                const uint32_t gs = (uint32_t)(hy * N + hx) * (uint32_t)sizeof(T);
                const uint32_t gxp = (uint32_t)(hy * N + x0 % N) * (uint32_t)sizeof(T);
                SH = halo_Sx<T, HS, HX>(L, h, vi, gs, gxp, t, inv_t, dt);
            } else if (tid < BY + BX) {
                const int i = tid - BY;
                const uint32_t h = (uint32_t)(i + 1);
                const int hx = (x0 + i) % N, hy = (y0 - 1 + N) % N;
                const uint32_t gs = (uint32_t)(hy * N + hx) * (uint32_t)sizeof(T);
                const uint32_t gyp = (uint32_t)((y0 % N) * N + hx) * (uint32_t)sizeof(T);
                SH = halo_Sy<T, HS, HX>(L, h, vi, gs, gyp, t, inv_t, dt);
            }
            CPIC_PHASE();
            // S_i = E_i(n-1/2) + E_i(n+1/2) (the old values read again, cached)
            const a8<T> o1 = vA(vi, g.s, kCompE), o2 = vA(vi, g.s, kCompE + 8);
#pragma unroll
            for (int q = 0; q < 8; q++) {
                S1.v[q] = o1.v[q] + E1.v[q];
                S2.v[q] = o2.v[q] + E2.v[q];
            }
        }
        CPIC_PHASE();
        if (!eonly) {   // fourth leaf U_{-1,-2}(c) = [U_y(c-x-y) U_x(c-x)]^+ U_x(c-x-y) U_y(c-y)
            const uint32_t xmym = s - 1 - HX;
            const m3<T> M1 = mul(L.U(xmym, 1), L.U(xm, 0));
            const m3<T> M2 = mul(L.U(xmym, 0), L.U(ym, 1));
            const a8<T> q4 = proj(adj_mul(M1, M2));
#pragma unroll
            for (int q = 0; q < 8; q++) BE.v[q] += q4.v[q];
        }
        // B_x = -(1/2t) D_y, B_y = +(1/2t) D_x,
        // D_i = U_i(c) phi(c+i) U_i(c)^+ - U_i(c-i)^+ phi(c-i) U_i(c-i)
        if (kick && !eonly) {
            CPIC_PHASE();
            const T hb = T(1) / (T(2) * t);
            {
                const a8<T> f = transport(L.U(s, 0), vA(vi, g.xp, kCompPhi));
                const a8<T> b = transport_adj(L.U(xm, 0), vA(vi, g.xm, kCompPhi));
#pragma unroll
                for (int q = 0; q < 8; q++) GY.v[q] = hb * (f.v[q] - b.v[q]);
            }
            CPIC_PHASE();
            {
                const a8<T> f = transport(L.U(s, 1), vA(vi, g.yp, kCompPhi));
                const a8<T> b = transport_adj(L.U(ym, 1), vA(vi, g.ym, kCompPhi));
#pragma unroll
                for (int q = 0; q < 8; q++) GX.v[q] = -hb * (f.v[q] - b.v[q]);
            }
        }
    }
    CPIC_PHASE();
    // ---- the tile's particles: one per thread; those beyond the first NT of
    // the range and those that have left the tile go to the straggler list
    // (this block's in thread order, then the excess in record order)
    const View<T> R = make_view<T>(P.r, kPartReals, (uint32_t)a.np);
    const View<int> C = make_view<int>(P.cell, 2, (uint32_t)a.np);
    const bool record = is_record_step(a.sc, n), renorm = is_reunit_step(a.sc, n);
    const int p = p0 + tid;
    const bool live = p < p1;
    const uint32_t po = (uint32_t)(live ? p : 0) * sizeof(T), pi = (uint32_t)(live ? p : 0) * sizeof(int);
    Particle<T> ps;
    particle_cell(R, C, po, pi, N, eonly, ps);
    const int lx = ps.nx - x0, ly = ps.ny - y0;
    const bool mine = live && lx >= 0 && lx < BX && ly >= 0 && ly < BY;
    const bool strag = live && !mine;
    const uint64_t bal = __ballot(strag);
    if (lane == 0) wcount[wave] = __popcll(bal);
    __syncthreads();  // the links are no longer read (and wcount is complete)
    {
        int before = 0, total = 0;
#pragma unroll
        for (int w = 0; w < NW; w++) {
            before += w < wave ? wcount[w] : 0;
            total += wcount[w];
        }
        if (strag) tp.strag[p0 + before + __popcll(bal & ((1ull << lane) - 1ull))] = p;
        for (int q = p0 + NT + tid; q < p1; q += NT) tp.strag[q - NT + total] = q;
        if (tid == 0) tp.strag_count[tile] = total + max(0, p1 - p0 - NT);
    }
    // S_x of site (tx, ty) at ty*(BX+1) + tx + 1 (the left column at
    // ty*(BX+1)); S_y at (ty+1)*BX + tx (the bottom row at tx)
    constexpr int RXW = BX + 1, RX = RXW * BY, RYN = BX * (BY + 1);
    T* X = lds;
    if (tpush && kick) {
#pragma unroll
        for (int q = 0; q < 8; q++) {
            X[q * RX + ty * RXW + tx + 1] = S1.v[q];
            X[8 * RX + q * RYN + (ty + 1) * BX + tx] = S2.v[q];
        }
        if (tid < BY) {
#pragma unroll
            for (int q = 0; q < 8; q++) X[q * RX + tid * RXW] = SH.v[q];
        } else if (tid < BY + BX) {
#pragma unroll
            for (int q = 0; q < 8; q++) X[8 * RX + q * RYN + (tid - BY)] = SH.v[q];
        }
    }
    __syncthreads();
    // the electric fields at this thread's site (zero where inactive at step n)
    a8<T> FX = azero<T>(), FY = azero<T>(), FE = azero<T>();
    if (tpush) {
        if (kick) {
            const T w = T(1) / (T(4) * t);
            {
                a8<T> b;
#pragma unroll
                for (int q = 0; q < 8; q++) b.v[q] = X[q * RX + ty * RXW + tx];
                const a8<T> tb = transport_adj(vU(vi, g.xm, 0), b);
#pragma unroll
                for (int q = 0; q < 8; q++) FX.v[q] = w * (X[q * RX + ty * RXW + tx + 1] + tb.v[q]);
            }
            CPIC_PHASE();
            {
                a8<T> b;
#pragma unroll
                for (int q = 0; q < 8; q++) b.v[q] = X[8 * RX + q * RYN + ty * BX + tx];
                const a8<T> tb = transport_adj(vU(vi, g.ym, 1), b);
#pragma unroll
                for (int q = 0; q < 8; q++) FY.v[q] = w * (X[8 * RX + q * RYN + (ty + 1) * BX + tx] + tb.v[q]);
            }
            const a8<T> o = vA(vi, g.s, kCompPi);
#pragma unroll
            for (int q = 0; q < 8; q++) FE.v[q] = T(0.5) * (o.v[q] + PI.v[q]);
        } else {
            FE = PI;  // E_eta = pi(c, 1/2) at n = 0
        }
    }
    const Cell cell = make_cell<T>(mine ? ps.nx : x, mine ? ps.ny : y, N);
    if (mine) particle_load_rotate<T, false, true>(vi, R, C, po, pi, cell, a, n, true, renorm, err, ps);
    T f[6] = {0, 0, 0, 0, 0, 0};
    T* tab = lds;
    const int lc = mine ? ly * BX + lx : 0;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 8; q++) {
        tab[q * NT + tid] = FX.v[q];
        tab[(8 + q) * NT + tid] = FY.v[q];
        tab[(16 + q) * NT + tid] = FE.v[q];
    }
    __syncthreads();
    if (mine) {
#pragma unroll
        for (int j = 0; j < 3; j++) {
            T d = ps.Q.v[0] * tab[(8 * j) * NT + lc];
#pragma unroll
            for (int q = 1; q < 8; q++) d = fmaT(ps.Q.v[q], tab[(8 * j + q) * NT + lc], d);
            f[j] = d;
        }
    }
    __syncthreads();
    // the magnetic fields
#pragma unroll
    for (int q = 0; q < 8; q++) {
        tab[q * NT + tid] = GX.v[q];
        tab[(8 + q) * NT + tid] = GY.v[q];
        tab[(16 + q) * NT + tid] = eonly ? T(0) : T(-0.25) * BE.v[q];
    }
    __syncthreads();
    double obs[4] = {0, 0, 0, 0};
    if (mine) {
#pragma unroll
        for (int j = 0; j < 3; j++) {
            T d = ps.Q.v[0] * tab[(8 * j) * NT + lc];
#pragma unroll
            for (int q = 1; q < 8; q++) d = fmaT(ps.Q.v[q], tab[(8 * j + q) * NT + lc], d);
            f[3 + j] = d;
        }
        particle_update<T, false>(vi, R, C, po, pi, cell, a, n, renorm, record, f, ps, obs);
    }
    if (record) block_reduce_store<4>(obs, 0u, partials + ((size_t)record_slot_of(a.sc, n) * ngroups + tile) * 4);
}

template <typename T, int BX, int BY>
static void launch_fused_t(const Fields<T>& A, const Fields<T>& B, int N, int remap, int nt_store, const Parts<T>& P,
                           const PushArgs& a, const TileParts& tp, int* d_step, double* partials, int ngroups,
                           int* err, hipStream_t st, const KTimer& tm)
{
    const int nt = fused_tiles(N, BX, BY);
    const dim3 g(remap ? 8 * ((nt + 7) / 8) : nt), b(BX * BY);
    if (nt_store)
        klaunch(tm, fused_kernel<T, BX, BY, kStoreNT>, g, b, st, A, B, N, remap, P, a, tp, d_step, partials, ngroups,
                err);
    else
        klaunch(tm, fused_kernel<T, BX, BY, 0>, g, b, st, A, B, N, remap, P, a, tp, d_step, partials, ngroups, err);
}

template <typename T>
hipError_t launch_fused(const Fields<T>& A, const Fields<T>& B, const LaunchCfg& cfg, const Parts<T>& P,
                        const PushArgs& a, const TileParts& tp, int* d_step, double* partials, int* err,
                        hipStream_t st, const KTimer& tm_tile, const KTimer& tm_strag)
{
    const int N = a.N, nt = fused_tiles(N, cfg.bx, cfg.by), ngroups = fused_groups(N, cfg.bx, cfg.by);
    if (a.np <= 0 || nt <= 0 || !fused_shape(cfg.bx, cfg.by)) return hipErrorInvalidValue;
    const int r = cfg.xcd_remap, nts = cfg.nt_store;
    if (cfg.bx == 64 && cfg.by == 8)
        launch_fused_t<T, 64, 8>(A, B, N, r, nts, P, a, tp, d_step, partials, ngroups, err, st, tm_tile);
    else if (cfg.bx == 32 && cfg.by == 8)
        launch_fused_t<T, 32, 8>(A, B, N, r, nts, P, a, tp, d_step, partials, ngroups, err, st, tm_tile);
    else if (cfg.bx == 16 && cfg.by == 16)
        launch_fused_t<T, 16, 16>(A, B, N, r, nts, P, a, tp, d_step, partials, ngroups, err, st, tm_tile);
    else
        launch_fused_t<T, 8, 8>(A, B, N, r, nts, P, a, tp, d_step, partials, ngroups, err, st, tm_tile);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_stragglers<T>(A, B, P, a, tp, nt, d_step, partials, ngroups, err, st, tm_strag);
}
template hipError_t launch_fused<double>(const Fields<double>&, const Fields<double>&, const LaunchCfg&,
                                         const Parts<double>&, const PushArgs&, const TileParts&, int*, double*, int*,
                                         hipStream_t, const KTimer&, const KTimer&);
template hipError_t launch_fused<float>(const Fields<float>&, const Fields<float>&, const LaunchCfg&,
                                        const Parts<float>&, const PushArgs&, const TileParts&, int*, double*, int*,
                                        hipStream_t, const KTimer&, const KTimer&);

}  // namespace cpic
