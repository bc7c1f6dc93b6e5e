// sort.hip -- periodic reordering of the particle records by lattice cell.
//
// The push gathers the fields around each particle's nearest grid point, and
// the fused step (fused.hip) pushes the particles of a tile in the workgroup
// that updates the tile.  Particles are ordered by tiles of tx x ty cells
// (tile-major, then row-major inside the tile): 32 x 16 for the gather push,
// whose wavefronts and the workgroups that run together on one XCD then read
// a compact patch of the lattice in whole cache lines, and the fused kernel's
// own tile shape for the fused step, which also receives the range of records
// of every tile.  The key of a moving particle is its nearest grid point at
// the step the order is made for (from its position), of a static one its
// cell.  The order is that of a stable sort of the keys (a counting sort,
// below); the records are permuted into a scratch copy and copied back so
// that buffer addresses (captured in HIP graphs) never change.  pid tracks
// each record's original index for state exchange.
#include <rocprim/device/device_scan.hpp>

#include "internal.h"

namespace cpic {

__host__ __device__ inline unsigned sort_key_bound(int N, int tx, int ty)
{
    return (unsigned)fused_tiles(N, tx, ty) * (unsigned)(tx * ty);
}

template <typename T>
__global__ void cell_keys_kernel(const T* __restrict__ r, const int* __restrict__ cell, int np, int N, int tx, int ty,
                                 int from_position, unsigned* keys, int* count)
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
    const unsigned key = (unsigned)(tile * tx * ty + (cy % ty) * tx + cx % tx);
    keys[p] = key;
    if (count) atomicAdd(&count[key], 1);
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

// The order comes from a counting sort of the cell keys (dense integers below
// key_capacity(N)): count the records of every key as the keys are formed
// (atomic increments, whose totals do not depend on their order), an
// exclusive scan of the counts (rocPRIM, integers: exact), and a scatter that
// takes each record's slot in its key's run with an atomic increment of the
// run's cursor.  The slots inside a run then follow the order the increments
// happened in, so a last pass orders every run of more than one record by
// input index: the result is the permutation of a stable sort, the same on
// every run.  Runs are short (a few records per cell); a long one (records
// piled on one cell) is heap-sorted, so its cost stays n log n.  The last pass
// also clears the counts: they are zero between reorderings (and from
// allocation on).
__global__ void zero_kernel(int* a, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = 0;
}
// offs: exclusive scan of the counts on entry, the end of every run on exit
__global__ void scatter_keys_kernel(const unsigned* __restrict__ keys, int np, int* offs, unsigned* keys_out,
                                    int* perm)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const unsigned k = keys[p];
    const int slot = atomicAdd(&offs[k], 1);
    keys_out[slot] = k;
    perm[slot] = p;
}
__device__ void sift_down(int* a, int root, int n)
{
    while (2 * root + 1 < n) {
        int child = 2 * root + 1;
        if (child + 1 < n && a[child + 1] > a[child]) child++;
        if (a[root] >= a[child]) return;
        const int t = a[root];
        a[root] = a[child];
        a[child] = t;
        root = child;
    }
}
__global__ void order_runs_kernel(int* count, const int* __restrict__ ends, int nkeys, int* perm)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nkeys) return;
    const int c = count[k];
    count[k] = 0;
    if (c < 2) return;
    int* a = perm + (ends[k] - c);
    if (c <= 32) {
        for (int i = 1; i < c; i++) {
            const int v = a[i];
            int j = i - 1;
            while (j >= 0 && a[j] > v) {
                a[j + 1] = a[j];
                j--;
            }
            a[j + 1] = v;
        }
        return;
    }
    for (int i = c / 2 - 1; i >= 0; i--) sift_down(a, i, c);
    for (int n = c - 1; n > 0; n--) {
        const int t = a[0];
        a[0] = a[n];
        a[n] = t;
        sift_down(a, 0, n);
    }
}

int key_capacity(int N)
{
    // the largest key bound of any tile shape (tiles of at most 64 x 64 cells)
    return (N + 64) * (N + 64);
}

size_t sort_temp_bytes(int N)
{
    size_t bytes = 0;
    // size query only (no device work)
    (void)rocprim::exclusive_scan(nullptr, bytes, (int*)nullptr, (int*)nullptr, 0, (size_t)key_capacity(N),
                                  rocprim::plus<int>());
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
    const unsigned nkeys = sort_key_bound(N, tx, ty);
    if (nkeys > (unsigned)b.key_cap) return hipErrorInvalidValue;
    const int blocks = (np + 255) / 256, kblocks = (int)((nkeys + 255) / 256);
    // a single record needs no sort: its key is the sorted key array
    hipLaunchKernelGGL(cell_keys_kernel<T>, dim3(blocks), dim3(256), 0, st, r, cell, np, N, tx, ty,
                       from_position ? 1 : 0, np > 1 ? b.keys : b.keys2, np > 1 ? b.count : nullptr);
    if (np > 1) {
        size_t bytes = b.temp_bytes;
        hipError_t e = rocprim::exclusive_scan(b.temp, bytes, b.count, b.offs, 0, (size_t)nkeys, rocprim::plus<int>(),
                                               st);
        if (e != hipSuccess) {
            // keep the counts zero for the next reordering
            hipLaunchKernelGGL(zero_kernel, dim3(kblocks), dim3(256), 0, st, b.count, (int)nkeys);
            return e;
        }
        hipLaunchKernelGGL(scatter_keys_kernel, dim3(blocks), dim3(256), 0, st, b.keys, np, b.offs, b.keys2, b.perm);
        hipLaunchKernelGGL(order_runs_kernel, dim3(kblocks), dim3(256), 0, st, b.count, b.offs, (int)nkeys, b.perm);
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
