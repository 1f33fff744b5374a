// sample_sort.hip -- the order in which qsv_sample walks its shots: indices of the
// uniforms sorted by value, equal values in index order, computed on the device with a
// stable radix sort (rocPRIM) of the uniforms' bit patterns.  For uniforms in [0, 1) the
// IEEE-754 bit pattern, read as an unsigned integer, orders like the value (sign bit 0);
// -0.0, which qsv_sample accepts as 0, is mapped to +0.0 first.
#include <hip/hip_runtime.h>

#include <cstring>

#include <rocprim/device/device_radix_sort.hpp>

#include "qsv_internal.h"

namespace qsv {

namespace {

__global__ __launch_bounds__(kThreads) void k_uniform_keys(const double* __restrict__ u, long long n,
                                                           unsigned long long* __restrict__ key,
                                                           long long* __restrict__ idx)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double v = u[i] == 0.0 ? 0.0 : u[i];
        key[i] = (unsigned long long)__double_as_longlong(v);
        idx[i] = i;
    }
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

size_t sort_uniforms_scratch(long long n)
{
    size_t temp = 0;
    (void)rocprim::radix_sort_pairs(nullptr, temp, (const unsigned long long*)nullptr, (unsigned long long*)nullptr,
                                    (const long long*)nullptr, (long long*)nullptr, (size_t)n, 0, 63);
    return 3 * align256(sizeof(long long) * (size_t)n) + align256(temp);
}

hipError_t sort_uniforms(const double* u, long long n, long long* order, void* scratch, size_t scratch_bytes,
                         hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const size_t nb = align256(sizeof(long long) * (size_t)n);
    if (scratch_bytes < 3 * nb) return hipErrorInvalidValue;
    unsigned char* p = static_cast<unsigned char*>(scratch);
    unsigned long long* key_in = reinterpret_cast<unsigned long long*>(p);
    unsigned long long* key_out = reinterpret_cast<unsigned long long*>(p + nb);
    long long* idx_in = reinterpret_cast<long long*>(p + 2 * nb);
    void* temp = p + 3 * nb;
    size_t temp_bytes = scratch_bytes - 3 * nb;
    const int grid = (int)std::min<long long>(1024, (n + kThreads - 1) / kThreads);
    hipLaunchKernelGGL(k_uniform_keys, dim3(grid), dim3(kThreads), 0, s, u, n, key_in, idx_in);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // bit 63 (the sign) is 0 for every key
    return rocprim::radix_sort_pairs(temp, temp_bytes, key_in, key_out, idx_in, order, (size_t)n, 0, 63, s);
}

}  // namespace qsv
