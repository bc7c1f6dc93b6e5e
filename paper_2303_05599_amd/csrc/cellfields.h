// cellfields.h -- the colour fields at a lattice cell at time t_n, as the
// particle push and the force table evaluate them (Sec. III.B
// interpolations, hat units), from the two field buffer sets of the step (A
// holds U(n), phi(n), E(n-1/2), pi(n-1/2) and B holds E(n+1/2), pi(n+1/2))
// and the plaquette field G = Proj U_12 that the field update stores.
#pragma once
#include "internal.h"
#include "su3.h"
#include "bufio.h"

namespace cpic {

__device__ __forceinline__ int wrap(int v, int N) { return v < 0 ? v + N : (v >= N ? v - N : v); }

#ifndef CPIC_PHASE
// compiler barrier between phases: keeps the links of one phase from being
// loaded (and held in registers) during another
#define CPIC_PHASE() __builtin_amdgcn_sched_barrier(0)
#endif

// The colour fields at a cell c at time t_n enter the particle push only
// through Q.F and the light-like path integral only through W F W^+, so each
// field is evaluated as an algebra vector F on its own:
//   E_i  = (1/4t) [S_i(c) + U_i(c-i)^+ S_i(c-i) U_i(c-i)], S_i = E_i(n-1/2) + E_i(n+1/2)
//          (n > 0; E_i = 0 at n = 0)
//   E_eta = [pi(c, n-1/2) + pi(c, n+1/2)] / 2 (n > 0); pi(c, 1/2) at n = 0
//   B_x  = -(1/2t) D_y(c),  B_y = +(1/2t) D_x(c),
//          D_i = U_i(c) phi(c+i) U_i(c)^+ - U_i(c-i)^+ phi(c-i) U_i(c-i)
//          (B_i = eps_ij F_{eta j} / tau with F_{eta j} = -D_j A_eta)
//   B_eta = -(1/4) Proj[U_12 + U_{2,-1} + U_{-1,-2} + U_{-2,1}](c), the four
//          counter-clockwise clover leaves.  Each leaf is the plaquette of a
//          neighbouring cell carried to c by the links between (exact for
//          unitary links), so with G(x) = Proj U_12(x):
//          Proj U_{2,-1}(c)  = U_x(c-x)^+ G(c-x) U_x(c-x)
//          Proj U_{-2,1}(c)  = U_y(c-y)^+ G(c-y) U_y(c-y)
//          Proj U_{-1,-2}(c) = U_x(c-x)^+ U_y(c-x-y)^+ G(c-x-y) U_y(c-x-y) U_x(c-x)
// The links are read as two rows with the third rebuilt (vU in bufio.h).
enum PushJob { kJobEx = 0, kJobEy, kJobEeta, kJobBx, kJobBy, kJobBeta, kJobs };

// The same fields split into eight sub-jobs, each one memory round trip of a
// wavefront: 0..4 are E_x, E_y, E_eta, B_x, B_y; 5..7 are the parts of B_eta
//   5: -(1/4) [G(c) + U_x(c-x)^+ G(c-x) U_x(c-x)]
//   6: -(1/4) U_y(c-y)^+ G(c-y) U_y(c-y)
//   7: -(1/4) U_x(c-x)^+ U_y(c-x-y)^+ G(c-x-y) U_y(c-x-y) U_x(c-x)
constexpr int kSubJobs = 8;
__host__ __device__ constexpr int subjob_field(int k) { return k < 5 ? k : kJobBeta; }

// the cell and the neighbours the fields read, as byte offsets into a component array
struct Cell {
    uint32_t s, s_xm, s_ym, s_xmym, s_xp, s_yp;
};
template <typename T> __device__ __forceinline__ Cell make_cell(int cx, int cy, int N)
{
    constexpr uint32_t b = sizeof(T);
    const int xm = wrap(cx - 1, N), ym = wrap(cy - 1, N), xp = wrap(cx + 1, N), yp = wrap(cy + 1, N);
    return {(uint32_t)(cy * N + cx) * b, (uint32_t)(cy * N + xm) * b, (uint32_t)(ym * N + cx) * b,
            (uint32_t)(ym * N + xm) * b, (uint32_t)(cy * N + xp) * b, (uint32_t)(yp * N + cx) * b};
}

__device__ __forceinline__ bool job_active(int j, int n, bool electric_only)
{
    if (j == kJobEeta) return true;
    if (j <= kJobEy) return n > 0;
    if (j <= kJobBy) return n > 0 && !electric_only;
    return !electric_only;
}

// E_i at the cell (n > 0)
template <typename T>
__device__ __forceinline__ a8<T> cell_E(int i, const View<T>& A, const View<T>& B, const Cell& c, T t)
{
    const uint32_t sb = i == 0 ? c.s_xm : c.s_ym, ce = kCompE + 8 * (uint32_t)i;
    const m3<T> L = vU(A, sb, i);
    const a8<T> h0 = vA(A, c.s, ce), h1 = vA(B, c.s, ce), b0 = vA(A, sb, ce), b1 = vA(B, sb, ce);
    a8<T> back;
#pragma unroll
    for (int q = 0; q < 8; q++) back.v[q] = b0.v[q] + b1.v[q];
    const a8<T> tb = transport_adj(L, back);
    const T w = T(1) / (T(4) * t);
    a8<T> F;
#pragma unroll
    for (int q = 0; q < 8; q++) F.v[q] = w * ((h0.v[q] + h1.v[q]) + tb.v[q]);
    return F;
}
// E_eta at the cell
template <typename T>
__device__ __forceinline__ a8<T> cell_Eeta(const View<T>& A, const View<T>& B, const Cell& c, int n)
{
    const a8<T> p1 = vA(B, c.s, kCompPi);
    if (n == 0) return p1;
    const a8<T> p0 = vA(A, c.s, kCompPi);
    a8<T> F;
#pragma unroll
    for (int q = 0; q < 8; q++) F.v[q] = T(0.5) * (p0.v[q] + p1.v[q]);
    return F;
}
// scale * D_i at the cell
template <typename T>
__device__ __forceinline__ a8<T> cell_D(int i, const View<T>& A, const Cell& c, T scale)
{
    const uint32_t sf = i == 0 ? c.s_xp : c.s_yp, sb = i == 0 ? c.s_xm : c.s_ym;
    const a8<T> f = transport(vU(A, c.s, i), vA(A, sf, kCompPhi));
    const a8<T> b = transport_adj(vU(A, sb, i), vA(A, sb, kCompPhi));
    a8<T> F;
#pragma unroll
    for (int q = 0; q < 8; q++) F.v[q] = scale * (f.v[q] - b.v[q]);
    return F;
}
// B_eta from the links alone (no plaquette field): the four counter-clockwise
// leaves at c formed as loops from c, summed as the fused step's tile push
// sums them (fused.hip), so that a particle gets the same field, bit for bit,
// from either push:
//   -(1/4) [((Proj U_12 - Proj U_{1,-2}) + Proj U_{2,-1}) + Proj U_{-1,-2}](c),
// with Proj U_{-2,1} = -Proj U_{1,-2} (U_{-2,1} = U_{1,-2}^+)
template <typename T>
__device__ __forceinline__ a8<T> clover_links(const View<T>& A, const Cell& c)
{
    // c-x+y and c+x-y: the row of c+y (c-y) at the column of c-x (c+x), in
    // modular offset arithmetic
    const uint32_t s_xmyp = c.s_yp + (c.s_xm - c.s), s_xpym = c.s_ym + (c.s_xp - c.s);
    a8<T> BE;
    {
        m3<T> M = mul(vU(A, c.s, 0), vU(A, c.s_xp, 1));
        M = mul_adj(M, vU(A, c.s_yp, 0));
        BE = proj(mul_adj(M, vU(A, c.s, 1)));
    }
    CPIC_PHASE();
    {
        m3<T> M = mul_adj(vU(A, c.s, 0), vU(A, s_xpym, 1));
        M = mul_adj(M, vU(A, c.s_ym, 0));
        const a8<T> p = proj(mul(M, vU(A, c.s_ym, 1)));
#pragma unroll
        for (int q = 0; q < 8; q++) BE.v[q] -= p.v[q];
    }
    CPIC_PHASE();
    {
        m3<T> M = mul_adj(vU(A, c.s, 1), vU(A, s_xmyp, 0));
        M = mul_adj(M, vU(A, c.s_xm, 1));
        const a8<T> p = proj(mul(M, vU(A, c.s_xm, 0)));
#pragma unroll
        for (int q = 0; q < 8; q++) BE.v[q] += p.v[q];
    }
    CPIC_PHASE();
    {
        const m3<T> M1 = mul(vU(A, c.s_xmym, 1), vU(A, c.s_xm, 0));   // U_y(c-x-y) U_x(c-x)
        const m3<T> M2 = mul(vU(A, c.s_xmym, 0), vU(A, c.s_ym, 1));   // U_x(c-x-y) U_y(c-y)
        const a8<T> p = proj(adj_mul(M1, M2));
#pragma unroll
        for (int q = 0; q < 8; q++) BE.v[q] += p.v[q];
    }
    a8<T> F;
#pragma unroll
    for (int q = 0; q < 8; q++) F.v[q] = T(-0.25) * BE.v[q];
    return F;
}

// sub-job k at the cell (the caller zeroes inactive ones); GL: B_eta whole
// from the links as sub-job 5 (6 and 7 then inactive, subjob_active)
template <typename T, bool GL = false>
__device__ __forceinline__ a8<T> subjob(int k, const View<T>& A, const View<T>& B, const View<T>& G, const Cell& c,
                                        int n, T t)
{
    if (k <= kJobEy) return cell_E<T>(k, A, B, c, t);
    if (k == kJobEeta) return cell_Eeta<T>(A, B, c, n);
    // B_x = -(1/2t) D_y, B_y = +(1/2t) D_x
    if (k == kJobBx) return cell_D<T>(1, A, c, T(-1) / (T(2) * t));
    if (k == kJobBy) return cell_D<T>(0, A, c, T(1) / (T(2) * t));
    if (GL) return clover_links<T>(A, c);
    a8<T> F;
    if (k == 5) {
        const a8<T> g0 = vA(G, c.s, 0), tg = transport_adj(vU(A, c.s_xm, 0), vA(G, c.s_xm, 0));
#pragma unroll
        for (int q = 0; q < 8; q++) F.v[q] = g0.v[q] + tg.v[q];
    } else if (k == 6) {
        F = transport_adj(vU(A, c.s_ym, 1), vA(G, c.s_ym, 0));
    } else {
        const m3<T> Lx = vU(A, c.s_xm, 0), Ly = vU(A, c.s_xmym, 1);
        F = transport_adj(Lx, transport_adj(Ly, vA(G, c.s_xmym, 0)));
    }
#pragma unroll
    for (int q = 0; q < 8; q++) F.v[q] *= T(-0.25);
    return F;
}
template <bool GL = false> __device__ __forceinline__ bool subjob_active(int k, int n, bool electric_only)
{
    if (GL && k > 5) return false;
    return job_active(subjob_field(k), n, electric_only);
}

// field j at the cell
template <typename T>
__device__ __forceinline__ a8<T> job_field(int j, const View<T>& A, const View<T>& B, const View<T>& G, const Cell& c,
                                           int n, T t)
{
    if (j != kJobBeta) return subjob<T>(j, A, B, G, c, n, t);
    a8<T> F = subjob<T>(5, A, B, G, c, n, t);
#pragma unroll 1
    for (int k = 6; k < kSubJobs; k++) {
        CPIC_PHASE();
        const a8<T> l = subjob<T>(k, A, B, G, c, n, t);
#pragma unroll
        for (int q = 0; q < 8; q++) F.v[q] += l.v[q];
    }
    return F;
}

// particle block b of the grid -> logical block: consecutive logical blocks
// (neighbouring cells once the particles are sorted) share one XCD's L2
__device__ __forceinline__ int xcd_block(int nblocks)
{
    const int per = (nblocks + 7) / 8;
    return (blockIdx.x & 7) * per + (blockIdx.x >> 3);
}

}  // namespace cpic
