// bufio.h -- structure-of-arrays access through buffer resources.
//
// A buffer set holds C components of V sites each (component-major).  A
// load of component c at site s is a raw buffer load with the per-lane
// offset s*sizeof(T) in one VGPR and the uniform offset c*V*sizeof(T) in an
// SGPR, so all components of a site share one address register; loads
// outside the buffer return 0 instead of faulting.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "su3.h"

namespace cpic {

// descriptor word 3 for gfx9-family targets (raw buffer, 32-bit data format)
constexpr int kBufferFlags = 0x00020000;
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

template <typename T> struct View {
    __amdgpu_buffer_rsrc_t r;
    uint32_t cs;  // bytes between components
};

template <typename T> __device__ __forceinline__ View<T> make_view(const T* base, uint32_t ncomp, uint32_t V)
{
    View<T> v;
    v.r = __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(base), 0, (int)(ncomp * V * sizeof(T)), kBufferFlags);
    v.cs = V * (uint32_t)sizeof(T);
    return v;
}

template <typename T> __device__ __forceinline__ T bld(const View<T>& v, uint32_t voff, uint32_t comp)
{
    if constexpr (sizeof(T) == 8)
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(v.r, voff, comp * v.cs, 0));
    else
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(v.r, voff, comp * v.cs, 0));
}
// cache policy of a store: 0 default, kStoreNT non-temporal (data the next
// kernel does not read: it should not displace data that it does)
constexpr int kStoreNT = 2;
template <typename T, int CP = 0>
__device__ __forceinline__ void bst(const View<T>& v, uint32_t voff, uint32_t comp, T x)
{
    if constexpr (sizeof(T) == 8)
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, x), v.r, voff, comp * v.cs, CP);
    else
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, x), v.r, voff, comp * v.cs, CP);
}
__device__ __forceinline__ int bld_i(const View<int>& v, uint32_t voff, uint32_t comp)
{
    return (int)__builtin_amdgcn_raw_buffer_load_b32(v.r, voff, comp * v.cs, 0);
}
__device__ __forceinline__ void bst_i(const View<int>& v, uint32_t voff, uint32_t comp, int x)
{
    __builtin_amdgcn_raw_buffer_store_b32((uint32_t)x, v.r, voff, comp * v.cs, 0);
}

// component offsets inside one field buffer set (68 components)
constexpr uint32_t kCompU = 0, kCompPhi = 36, kCompE = 44, kCompPi = 60;

// Links are kept as their first two rows (components 0..11 of the 18 of
// link i): no kernel reads the slots of the third row, and the field updates
// do not write them.  The third row of an SU(3) matrix is the complex
// conjugate of the cross product of the first two (exact for det U = 1, to
// the link's unitarity otherwise), and every reader rebuilds it.
template <typename T> __device__ __forceinline__ void rebuild_row3(m3<T>& m)
{
#pragma unroll
    for (int j = 0; j < 3; j++) {
        const int j1 = (j + 1) % 3, j2 = (j + 2) % 3;
        const cx<T> p = cmul(m.e[j1], m.e[3 + j2]), q = cmul(m.e[j2], m.e[3 + j1]);
        m.e[6 + j] = {p.re - q.re, q.im - p.im};
    }
}
template <typename T> __device__ __forceinline__ m3<T> vU(const View<T>& v, uint32_t voff, int i)
{
    m3<T> m;
#pragma unroll
    for (int c = 0; c < 6; c++)
        m.e[c] = {bld(v, voff, kCompU + 18 * i + 2 * c), bld(v, voff, kCompU + 18 * i + 2 * c + 1)};
    rebuild_row3(m);
    return m;
}
template <typename T, int CP = 0>
__device__ __forceinline__ void vU_st(const View<T>& v, uint32_t voff, int i, const m3<T>& m)
{
#pragma unroll
    for (int c = 0; c < 6; c++) {
        bst<T, CP>(v, voff, kCompU + 18 * i + 2 * c, m.e[c].re);
        bst<T, CP>(v, voff, kCompU + 18 * i + 2 * c + 1, m.e[c].im);
    }
}
template <typename T> __device__ __forceinline__ a8<T> vA(const View<T>& v, uint32_t voff, uint32_t comp0)
{
    a8<T> r;
#pragma unroll
    for (int a = 0; a < 8; a++) r.v[a] = bld(v, voff, comp0 + a);
    return r;
}
template <typename T, int CP = 0>
__device__ __forceinline__ void vA_st(const View<T>& v, uint32_t voff, uint32_t comp0, const a8<T>& r)
{
#pragma unroll
    for (int a = 0; a < 8; a++) bst<T, CP>(v, voff, comp0 + a, r.v[a]);
}

}  // namespace cpic
