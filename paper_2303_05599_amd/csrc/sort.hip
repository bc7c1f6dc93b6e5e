// sort.hip -- periodic reordering of the particle records by lattice cell.
//
// The push gathers the fields around each particle's nearest grid point.
// Particles are ordered by 16 x 16 cell tiles (tile-major, then row-major
// inside the tile): the 64 lanes of a wavefront and the workgroups that run
// together on one XCD then read a compact patch of the lattice, whose cache
// lines (16 sites of one row in double precision) they share.  The order is
// found with a stable radix sort of the cell keys (deterministic), the
// records are permuted into a scratch copy and copied back so that buffer
// addresses (captured in HIP graphs) never change.  pid tracks each record's
// original index for state exchange.
#include <hipcub/hipcub.hpp>

#include "internal.h"

namespace cpic {

constexpr int kSortTX = 16, kSortTY = 16;  // measured best of 16x16, 32x8, 32x4, 64x4, 128x2 (FP64 512^2)

__host__ __device__ inline unsigned sort_key_bound(int N)
{
    const unsigned ntx = (unsigned)((N + kSortTX - 1) / kSortTX), nty = (unsigned)((N + kSortTY - 1) / kSortTY);
    return ntx * nty * kSortTX * kSortTY;
}
static int key_bits(int N)
{
    int bits = 1;
    while ((1u << bits) < sort_key_bound(N)) bits++;
    return bits;
}

__global__ void cell_keys_kernel(const int* __restrict__ cell, int np, int N, unsigned* keys, int* vals)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const int cx = cell[p], cy = cell[np + p];
    const int ntx = (N + kSortTX - 1) / kSortTX;
    const int tile = (cy / kSortTY) * ntx + cx / kSortTX;
    keys[p] = (unsigned)(tile * kSortTX * kSortTY + (cy % kSortTY) * kSortTX + cx % kSortTX);
    vals[p] = p;
}

template <typename T>
__global__ void permute_kernel(const T* __restrict__ r, const int* __restrict__ cell, const int* __restrict__ pid,
                               const int* __restrict__ perm, int np, T* r2, int* cell2, int* pid2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    const int src = perm[i];
#pragma unroll
    for (int c = 0; c < kPartReals; c++) r2[(size_t)c * np + i] = r[(size_t)c * np + src];
    cell2[i] = cell[src];
    cell2[np + i] = cell[np + src];
    pid2[i] = pid[src];
}

// the permuted records back into the buffers the step graphs captured, in one
// pass (three device copies cost three launches)
template <typename T>
__global__ void copy_back_kernel(const T* __restrict__ r2, const int* __restrict__ cell2,
                                 const int* __restrict__ pid2, int np, T* r, int* cell, int* pid)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
#pragma unroll
    for (int c = 0; c < kPartReals; c++) r[(size_t)c * np + i] = r2[(size_t)c * np + i];
    cell[i] = cell2[i];
    cell[np + i] = cell2[np + i];
    pid[i] = pid2[i];
}

size_t sort_temp_bytes(int np, int N)
{
    size_t bytes = 0;
    // size query only: no device work, the status carries nothing more
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, (unsigned*)nullptr, (unsigned*)nullptr, (int*)nullptr,
                                             (int*)nullptr, np, 0, key_bits(N));
    return bytes;
}

template <typename T>
hipError_t sort_particles(const SortBufs& b, T* r, int* cell, int* pid, int np, int N, hipStream_t st)
{
    if (np <= 1) return hipSuccess;
    const int bits = key_bits(N);
    const int blocks = (np + 255) / 256;
    hipLaunchKernelGGL(cell_keys_kernel, dim3(blocks), dim3(256), 0, st, cell, np, N, b.keys, b.vals);
    size_t bytes = b.temp_bytes;
    hipError_t e = hipcub::DeviceRadixSort::SortPairs(b.temp, bytes, b.keys, b.keys2, b.vals, b.perm, np, 0, bits, st);
    if (e != hipSuccess) return e;
    T* r2 = static_cast<T*>(b.r2);
    hipLaunchKernelGGL(permute_kernel<T>, dim3(blocks), dim3(256), 0, st, r, cell, pid, b.perm, np, r2, b.cell2,
                       b.pid2);
    hipLaunchKernelGGL(copy_back_kernel<T>, dim3(blocks), dim3(256), 0, st, r2, b.cell2, b.pid2, np, r, cell, pid);
    return hipSuccess;  // launch errors surface at the stream's next synchronisation, as for every kernel
}

template hipError_t sort_particles<double>(const SortBufs&, double*, int*, int*, int, int, hipStream_t);
template hipError_t sort_particles<float>(const SortBufs&, float*, int*, int*, int, int, hipStream_t);

}  // namespace cpic
