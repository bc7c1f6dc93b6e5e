// noalloc.hip -- the field diagnostics of cpic_diagnostics (Gauss residual of
// Sec. II, lattice energy terms, link unitarity) on a caller-owned device
// buffer set, without any device allocation: the per-block partial sums of
// the reduction live in a fixed device array of this translation unit.
//
// The array is resolved to a device address once per device (hipGetSymbolAddress
// with that device current) and the address is kept per device: host code
// passes only that address to kernels, never the array's own name.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <string>

#include "../../include/cpic.h"
#include "ctx.h"
#include "internal.h"

using namespace cpic;

namespace {

// largest lattice of the library: N = 1024, 4096 blocks of 256 sites, eight
// partial columns per block (256 KiB per device)
constexpr int kNoallocMaxN = 1024;
constexpr int kNoallocMaxBlocks = (kNoallocMaxN * kNoallocMaxN + 255) / 256;
constexpr int kDiagColumns = 8;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

static __device__ __align__(256) double scratch[kNoallocMaxBlocks * kDiagColumns];

// Device address of the scratch array on the current device, resolved on the
// first call per device.
cpic_status cpic::noalloc_scratch(double** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(nullptr, e, "noalloc scratch: hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices)
        return fail(nullptr, CPIC_E_INVALID, "noalloc scratch: device index " + std::to_string(dev) + " out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(nullptr, e, "noalloc scratch: hipGetSymbolAddress");
        if (!p) return fail(nullptr, CPIC_E_HIP, "noalloc scratch: hipGetSymbolAddress returned NULL");
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[dev];
    return CPIC_OK;
}

extern "C" cpic_status cpic_field_diagnostics_noalloc(int32_t precision, int32_t N, double dtau_over_a, int64_t n,
                                                      const void* fields_dev, double* out_dev, void* hip_stream)
{
    if (!fields_dev || !out_dev)
        return fail(nullptr, CPIC_E_INVALID, "cpic_field_diagnostics_noalloc: NULL buffer");
    if (precision != CPIC_FP64 && precision != CPIC_FP32)
        return fail(nullptr, CPIC_E_INVALID, "cpic_field_diagnostics_noalloc: precision must be CPIC_FP64 or CPIC_FP32");
    if (N < 4 || N > kNoallocMaxN)
        return fail(nullptr, CPIC_E_INVALID,
                    "cpic_field_diagnostics_noalloc: N = " + std::to_string(N) + " outside [4, " +
                        std::to_string(kNoallocMaxN) + "] (the fixed scratch holds the partials of N <= " +
                        std::to_string(kNoallocMaxN) + ")");
    if (!(dtau_over_a > 0) || !std::isfinite(dtau_over_a))
        return fail(nullptr, CPIC_E_INVALID, "cpic_field_diagnostics_noalloc: dtau_over_a must be positive");
    if (n < 0 || n > (int64_t)INT32_MAX || !std::isfinite((double)n * dtau_over_a))
        return fail(nullptr, CPIC_E_INVALID, "cpic_field_diagnostics_noalloc: step out of range");
    double* part = nullptr;
    cpic_status s = noalloc_scratch(&part);
    if (s) return s;
    const hipStream_t st = static_cast<hipStream_t>(hip_stream);
    const int V = N * N;
    int nb = 0;
    hipError_t e = precision == CPIC_FP64
                       ? launch_field_diag<double>(fields_at<double>(const_cast<void*>(fields_dev), V), N, dtau_over_a,
                                                   (int)n, part, kNoallocMaxBlocks, &nb, st)
                       : launch_field_diag<float>(fields_at<float>(const_cast<void*>(fields_dev), V), N, dtau_over_a,
                                                  (int)n, part, kNoallocMaxBlocks, &nb, st);
    if (e != hipSuccess) return hip_fail(nullptr, e, "cpic_field_diagnostics_noalloc: diagnostics kernel");
    // every partial the reduction reads was written by the launch above
    e = launch_reduce_rows(part, nb, kDiagColumns, out_dev, st);
    if (e != hipSuccess) return hip_fail(nullptr, e, "cpic_field_diagnostics_noalloc: reduction");
    return CPIC_OK;
}
