// sort.hip -- periodic reordering of the particle records by lattice cell.
//
// The push gathers the fields around each particle's nearest grid point, and
// the fused step (fused.hip) pushes the particles of a tile in the workgroup
// that updates the tile.  Particles are ordered by tiles of tx x ty cells
// (tile-major, then row-major inside the tile): 32 x 16 for the gather push,
// whose wavefronts and the workgroups that run together on one XCD then read
// a compact patch of the lattice in whole cache lines, and the fused kernel's own tile shape for
// the fused step, which also receives the range of records of every tile.
// The key of a moving particle is its nearest grid point at the step the
// order is made for (from its position), of a static one its cell.  The order
// comes from a stable radix sort of the keys (rocPRIM, deterministic); the
// records are permuted into a scratch copy and copied back so that buffer
// addresses (captured in HIP graphs) never change.  pid tracks each record's
// original index for state exchange.
#include <rocprim/device/device_radix_sort.hpp>

#include "internal.h"

namespace cpic {

__host__ __device__ inline unsigned sort_key_bound(int N, int tx, int ty)
{
    return (unsigned)fused_tiles(N, tx, ty) * (unsigned)(tx * ty);
}
static int key_bits(int N, int tx, int ty)
{
    int bits = 1;
    while (bits < 32 && (1u << bits) < sort_key_bound(N, tx, ty)) bits++;
    return bits;
}

template <typename T>
__global__ void cell_keys_kernel(const T* __restrict__ r, const int* __restrict__ cell, int np, int N, int tx, int ty,
                                 int from_position, unsigned* keys, int* vals)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    int cx, cy;
    if (from_position) {
        // the nearest grid point as the push computes it
        const int nx = (int)floor(r[(size_t)PX_ * np + p] + T(0.5)), ny = (int)floor(r[(size_t)PY_ * np + p] + T(0.5));
        cx = nx >= N ? nx - N : nx;
        cy = ny >= N ? ny - N : ny;
    } else {
        cx = cell[p];
        cy = cell[np + p];
    }
    // a non-finite position (a diverged run, which the watchdog reports) still
    // gets a key inside the lattice's range
    cx = min(max(cx, 0), N - 1);
    cy = min(max(cy, 0), N - 1);
    const int ntx = (N + tx - 1) / tx;
    const int tile = (cy / ty) * ntx + cx / tx;
    keys[p] = (unsigned)(tile * tx * ty + (cy % ty) * tx + cx % tx);
    vals[p] = p;
}

// tile_start[t] = first record of tile t (or of the next non-empty tile),
// tile_start[ntiles] = np, from the sorted keys; every entry is written once
__global__ void tile_start_kernel(const unsigned* __restrict__ sorted, int np, unsigned per_tile, int ntiles,
                                  int* tile_start)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > np) return;
    const int ti = i < np ? (int)min(sorted[i] / per_tile, (unsigned)ntiles) : ntiles;
    const int tp = i > 0 ? (int)min(sorted[i - 1] / per_tile, (unsigned)ntiles) : -1;
    for (int t = tp + 1; t <= ti; t++) tile_start[t] = i;
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

// rocPRIM's radix sort takes a block sort and merge passes below
// merge_sort_limit keys and its Onesweep radix passes above it.  The
// reorderings run between the captured step graphs, so Onesweep's clearing of
// its own state (a memset on the stream) is allowed.  Measured at 512^2 with
// 18-bit cell keys: 10^5 records sort faster by merging (4.8 against 6.5 us per
// step, amortised over the 16 steps between reorderings), 10^6 by Onesweep
// (12.2 against 14.3 us per step), so the limit sits at 2^19 (rocPRIM's
// default is 2^20).
using SortConfig = rocprim::radix_sort_config<rocprim::default_config, rocprim::default_config,
                                              rocprim::default_config, (size_t)1 << 19>;

size_t sort_temp_bytes(int np)
{
    size_t bytes = 0;
    // size query only (no device work) for the widest keys any tile shape gives
    (void)rocprim::radix_sort_pairs<SortConfig>(nullptr, bytes, (unsigned*)nullptr, (unsigned*)nullptr, (int*)nullptr,
                                    (int*)nullptr, np, 0u, 32u);
    return bytes;
}

hipError_t launch_tile_start(const unsigned* sorted_keys, int np, int N, int tx, int ty, int* tile_start,
                             hipStream_t st)
{
    if (np <= 0 || !fused_shape(tx, ty)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(tile_start_kernel, dim3((np + 256) / 256), dim3(256), 0, st, sorted_keys, np,
                       (unsigned)(tx * ty), fused_tiles(N, tx, ty), tile_start);
    return hipGetLastError();
}

template <typename T>
hipError_t sort_particles(const SortBufs& b, T* r, int* cell, int* pid, int np, int N, int tx, int ty,
                          bool from_position, int* tile_start, hipStream_t st)
{
    if (np <= 0 || tx <= 0 || ty <= 0) return np <= 0 ? hipSuccess : hipErrorInvalidValue;
    const int blocks = (np + 255) / 256;
    // a single record needs no sort: its key is the sorted key array
    hipLaunchKernelGGL(cell_keys_kernel<T>, dim3(blocks), dim3(256), 0, st, r, cell, np, N, tx, ty,
                       from_position ? 1 : 0, np > 1 ? b.keys : b.keys2, b.vals);
    if (np > 1) {
        size_t bytes = b.temp_bytes;
        hipError_t e = rocprim::radix_sort_pairs<SortConfig>(b.temp, bytes, b.keys, b.keys2, b.vals, b.perm, np, 0u,
                                                 (unsigned)key_bits(N, tx, ty), st);
        if (e != hipSuccess) return e;
        T* r2 = static_cast<T*>(b.r2);
        hipLaunchKernelGGL(permute_kernel<T>, dim3(blocks), dim3(256), 0, st, r, cell, pid, b.perm, np, r2, b.cell2,
                           b.pid2);
        hipLaunchKernelGGL(copy_back_kernel<T>, dim3(blocks), dim3(256), 0, st, r2, b.cell2, b.pid2, np, r, cell,
                           pid);
    }
    if (tile_start) return launch_tile_start(b.keys2, np, N, tx, ty, tile_start, st);
    return hipGetLastError();  // launch errors surface at the stream's next synchronisation, as for every kernel
}

template hipError_t sort_particles<double>(const SortBufs&, double*, int*, int*, int, int, int, int, bool, int*,
                                           hipStream_t);
template hipError_t sort_particles<float>(const SortBufs&, float*, int*, int*, int, int, int, int, bool, int*,
                                          hipStream_t);

}  // namespace cpic
