// reduce.h -- deterministic block reductions in double precision
// (wavefront shuffles, then one LDS pass in fixed wave order).
#pragma once
#include <hip/hip_runtime.h>

namespace cpic {

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Reduces NC values per thread over the block (<= 1024 threads) and writes
// them to out[0..NC) from thread 0.  Columns whose bit is set in max_mask are
// max-reduced, the others summed.  Every thread of the block must call it.
template <int NC>
__device__ void block_reduce_store(const double (&v)[NC], unsigned max_mask, double* out)
{
    __shared__ double sh[16][NC];
    const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
    const int nthreads = blockDim.x * blockDim.y * blockDim.z;
    const int lane = tid & 63, wave = tid >> 6, nwaves = (nthreads + 63) >> 6;
#pragma unroll
    for (int c = 0; c < NC; c++) {
        double r = ((max_mask >> c) & 1) ? wave_max(v[c]) : wave_sum(v[c]);
        if (lane == 0) sh[wave][c] = r;
    }
    __syncthreads();
    if (tid == 0) {
#pragma unroll
        for (int c = 0; c < NC; c++) {
            double r = sh[0][c];
            for (int w = 1; w < nwaves; w++) r = ((max_mask >> c) & 1) ? fmax(r, sh[w][c]) : r + sh[w][c];
            out[c] = r;
        }
    }
}

}  // namespace cpic
