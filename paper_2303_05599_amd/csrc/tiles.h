// tiles.h -- site tiles of the field update: neighbour offsets, the
// XCD-aware tile order and the LDS halo of two-row links, shared by the
// field kernels (field.hip) and the fused field-and-particle step (fused.hip).
#pragma once
#include "bufio.h"
#include "su3.h"

namespace cpic {

#ifndef CPIC_PHASE
// scheduling barrier between the phases of a stencil: keeps the machine
// scheduler from hoisting every link load of a site to the top (which would
// hold ~10 matrices in registers at once)
#define CPIC_PHASE() __builtin_amdgcn_sched_barrier(0)
#endif

// byte offsets (site * sizeof(T)) of a site and the neighbours its stencil reads
struct Nbr {
    uint32_t s, xp, xm, yp, ym, xpym, xmyp;
};
template <typename T> __device__ __forceinline__ Nbr neighbours(int x, int y, int N)
{
    const int xp = x + 1 == N ? 0 : x + 1, xm = x == 0 ? N - 1 : x - 1;
    const int yp = y + 1 == N ? 0 : y + 1, ym = y == 0 ? N - 1 : y - 1;
    constexpr uint32_t b = sizeof(T);
    return {(uint32_t)(y * N + x) * b,  (uint32_t)(y * N + xp) * b,  (uint32_t)(y * N + xm) * b,
            (uint32_t)(yp * N + x) * b, (uint32_t)(ym * N + x) * b,  (uint32_t)(ym * N + xp) * b,
            (uint32_t)(yp * N + xm) * b};
}

// Workgroups are dealt round-robin to the 8 XCDs; with remapping, logical
// block g of `total` goes to XCD g / per, so each XCD works on a contiguous
// band of tiles and their shared halos stay in its L2.
__device__ __forceinline__ int logical_block(int total, int remap)
{
    if (!remap) return blockIdx.x;
    const int per = (total + 7) / 8;
    return (blockIdx.x & 7) * per + (blockIdx.x >> 3);
}

// An LDS tile of BX x BY sites with a halo of one site on every side that
// holds only the first two rows of each link (12 of 18 reals; the third row
// of an SU(3) matrix is the complex conjugate of the cross product of the
// first two); the scalars are read from global memory (L1/L2).  Small tiles
// let two workgroups share a CU, and a stencil forms each plaquette in one
// phase from links re-read out of LDS, so no partial products stay live
// across phases.  Tile site (hx, hy) is global site (x0 + hx - 1, y0 + hy - 1)
// (periodic), at index hy * (BX + 2) + hx.
template <typename T, int HS> struct LdsLinks2 {
    const T* l;  // [24][HS]: rows 0, 1 of U_x, then of U_y
    __device__ __forceinline__ m3<T> U(uint32_t h, int i) const
    {
        m3<T> m;
#pragma unroll
        for (int c = 0; c < 6; c++) m.e[c] = {l[(12 * i + 2 * c) * HS + h], l[(12 * i + 2 * c + 1) * HS + h]};
#pragma unroll
        for (int j = 0; j < 3; j++) {
            const int j1 = (j + 1) % 3, j2 = (j + 2) % 3;
            const cx<T> p = cmul(m.e[j1], m.e[3 + j2]), q = cmul(m.e[j2], m.e[3 + j1]);
            m.e[6 + j] = {p.re - q.re, q.im - p.im};
        }
        return m;
    }
};


// stage rows 0, 1 of both links (buffer components 0..11 and 18..29) of the
// tile at (x0, y0) and its halo into lds[24][HS]; NT threads of the block
template <typename T, int BX, int BY>
__device__ __forceinline__ void stage_links2(T* lds, const View<T>& vi, int x0, int y0, int N, int tid)
{
    constexpr int HX = BX + 2, HY = BY + 2, HS = HX * HY, NT = BX * BY, NC = 24;
#pragma unroll
    for (int h0 = 0; h0 < HS; h0 += NT) {
        const int h = h0 + tid;
        if (h < HS) {
            const int hy = h / HX, hx = h - hy * HX;
            const int gx = (x0 + hx - 1 + N) % N, gy = (y0 + hy - 1 + N) % N;
            const uint32_t go = (uint32_t)(gy * N + gx) * (uint32_t)sizeof(T);
            T v[NC];
#pragma unroll
            for (int c = 0; c < NC; c++) v[c] = bld(vi, go, (uint32_t)(c < 12 ? c : c + 6));
#pragma unroll
            for (int c = 0; c < NC; c++) lds[c * HS + h] = v[c];
        }
    }
}

}  // namespace cpic
