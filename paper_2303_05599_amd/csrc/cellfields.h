// cellfields.h -- the colour fields at a lattice cell at time t_n, as the
// particle push and the light-like path integral evaluate them (Sec. III.B
// interpolations, hat units), from U(n), pi(n + 1/2) and the per-site pieces
// that the field update writes to the aux buffer.
#pragma once
#include "internal.h"
#include "su3.h"
#include "bufio.h"

namespace cpic {

__device__ __forceinline__ int wrap(int v, int N) { return v < 0 ? v + N : (v >= N ? v - N : v); }

// compiler barrier between phases: keeps the links of one phase from being
// loaded (and held in registers) during another
#define CPIC_PHASE() __builtin_amdgcn_sched_barrier(0)

// The colour fields at a cell c at time t_n (Sec. III.B interpolations, hat
// units) enter the particle push only through Q.F and the light-like path
// integral only through W F W^+, so each field is evaluated as an algebra
// vector F on its own:
//   E_i  = (1/4t) [S_i(c) + U_i(c-i)^+ S_i(c-i) U_i(c-i)], S_i = E_i(n-1/2) + E_i(n+1/2)
//          (n > 0; E_i = 0 at n = 0)
//   E_eta = P(c) / 2, P = pi(n-1/2) + pi(n+1/2) (n > 0); pi(1/2)(c) at n = 0
//   B_x  = -(1/2t) [U_y(c) phi(c+y) U_y(c)^+ - U_y(c-y)^+ phi(c-y) U_y(c-y)] = -(1/2t) D_y(c)
//   B_y  = +(1/2t) [U_x(c) phi(c+x) U_x(c)^+ - U_x(c-x)^+ phi(c-x) U_x(c-x)] = +(1/2t) D_x(c)
//   B_eta = -(1/4) Proj[U_12 + U_{2,-1} + U_{-1,-2} + U_{-2,1}] (clover, all
//          counter-clockwise).
// Each clover leaf is the plaquette of a neighbouring cell carried to c by
// the links between: with G(x) = Proj U_12(x) and unitary links,
//   Proj U_{2,-1}(c)  = U_1(c-1)^+ G(c-1) U_1(c-1)
//   Proj U_{-1,-2}(c) = U_1(c-1)^+ U_2(c-1-2)^+ G(c-1-2) U_2(c-1-2) U_1(c-1)
//   Proj U_{-2,1}(c)  = U_2(c-2)^+ G(c-2) U_2(c-2)
// The field update writes G, D_x, D_y, S_x, S_y and P for every site (the aux
// buffer), so a cell's fields take four G's, three sums and three links.
// The links are read as two rows with the third rebuilt (vU in bufio.h).
enum PushJob { kJobEx = 0, kJobEy, kJobEeta, kJobBx, kJobBy, kJobBeta, kJobs };

// the cell and the neighbours the push reads, as byte offsets into a component array
struct Cell {
    uint32_t s, s_xm, s_ym, s_xmym;
};
template <typename T> __device__ __forceinline__ Cell make_cell(int cx, int cy, int N)
{
    constexpr uint32_t b = sizeof(T);
    const int xm = wrap(cx - 1, N), ym = wrap(cy - 1, N);
    return {(uint32_t)(cy * N + cx) * b, (uint32_t)(cy * N + xm) * b, (uint32_t)(ym * N + cx) * b,
            (uint32_t)(ym * N + xm) * b};
}

__device__ __forceinline__ bool job_active(int j, int n, bool electric_only)
{
    if (j == kJobEeta) return true;
    if (j <= kJobEy) return n > 0;
    if (j <= kJobBy) return n > 0 && !electric_only;
    return !electric_only;
}

template <typename T>
__device__ __forceinline__ a8<T> job_field(int j, const View<T>& A, const View<T>& B, const View<T>& X, const Cell& c,
                                           int n, T t)
{
    a8<T> F;
    if (j <= kJobEy) {
        // E_i from the half-step sums S_i = E_i(n-1/2) + E_i(n+1/2) of the aux buffer
        const int i = j;
        const uint32_t sb = i == 0 ? c.s_xm : c.s_ym;
        const uint32_t cs = i == 0 ? kAuxS1 : kAuxS2;
        const a8<T> here = vA(X, c.s, cs);
        const a8<T> tb = transport_adj(vU(A, sb, i), vA(X, sb, cs));
        const T q = T(1) / (T(4) * t);
#pragma unroll
        for (int a = 0; a < 8; a++) F.v[a] = q * (here.v[a] + tb.v[a]);
    } else if (j == kJobEeta) {
        if (n > 0) {
            const a8<T> P = vA(X, c.s, kAuxP);
#pragma unroll
            for (int a = 0; a < 8; a++) F.v[a] = T(0.5) * P.v[a];
        } else {
            F = vA(B, c.s, kCompPi);
        }
    } else if (j <= kJobBy) {
        // B_x = -(1/2t) D_y, B_y = +(1/2t) D_x
        const bool bx = j == kJobBx;
        const T q = (bx ? T(-1) : T(1)) / (T(2) * t);
        const a8<T> D = vA(X, c.s, bx ? kAuxDy : kAuxDx);
#pragma unroll
        for (int a = 0; a < 8; a++) F.v[a] = q * D.v[a];
    } else {
        const a8<T> g2 = transport_adj(vU(A, c.s_ym, 1), vA(X, c.s_ym, kAuxG));
        CPIC_PHASE();
        const a8<T> g12 = transport_adj(vU(A, c.s_xmym, 1), vA(X, c.s_xmym, kAuxG));
        a8<T> g1 = vA(X, c.s_xm, kAuxG);
#pragma unroll
        for (int a = 0; a < 8; a++) g1.v[a] += g12.v[a];
        CPIC_PHASE();
        const a8<T> g1t = transport_adj(vU(A, c.s_xm, 0), g1);
        const a8<T> g0 = vA(X, c.s, kAuxG);
#pragma unroll
        for (int a = 0; a < 8; a++) F.v[a] = T(-0.25) * (g0.v[a] + g1t.v[a] + g2.v[a]);
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
