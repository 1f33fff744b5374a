// sample_sort.hip -- qsv_sample's device-side bookkeeping of the shots.  The order: the
// indices of the uniforms sorted by value, equal values in index order, by a stable
// radix sort (rocPRIM) of the uniforms' bit patterns (for uniforms in [0, 1) the IEEE-754
// pattern, read as an unsigned integer, orders like the value; -0.0, which qsv_sample
// accepts as 0, is mapped to +0.0 first).  Then each sorted shot's chunk and residual,
// the runs of shots in one chunk, and the scatter of the outcomes back to shot order.
#include <hip/hip_runtime.h>

#include <cstring>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

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

namespace qsv {

namespace {

// Shot k (in sorted order) at t = u[order[k]] * P goes to the first chunk c >= c0 with
// cum[c + 1] > t (such a chunk has mass: cum[c] <= t there), or to lastnz when none is
// below it (t rounded up to P), residual t - cum[c]: the host's walk over the sorted
// shots, element by element, with the same FP64 operations.
__global__ __launch_bounds__(kThreads) void k_assign_shots(const double* __restrict__ u,
                                                           const long long* __restrict__ order, long long n,
                                                           const double* __restrict__ cum, long long c0,
                                                           long long lastnz, double P,
                                                           long long* __restrict__ chunk_of,
                                                           double* __restrict__ residual)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) {
        const double t = u[order[k]] * P;
        long long lo = c0, hi = lastnz;   // smallest c in [c0, lastnz) with cum[c + 1] > t, else lastnz
        while (lo < hi) {
            const long long mid = lo + ((hi - lo) >> 1);
            if (cum[mid + 1] > t) hi = mid;
            else lo = mid + 1;
        }
        chunk_of[k] = lo;
        residual[k] = t - cum[lo];
    }
}

__global__ __launch_bounds__(kThreads) void k_run_starts(const long long* __restrict__ chunk_of, long long n,
                                                         int* __restrict__ flag)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride)
        flag[k] = (k == 0 || chunk_of[k] != chunk_of[k - 1]) ? 1 : 0;
}

// Runs of equal chunks among the sorted shots, in order: run r = pos[k] for its first
// shot k; it ends where the next run starts (or at n).
__global__ __launch_bounds__(kThreads) void k_run_list(const long long* __restrict__ chunk_of,
                                                       const int* __restrict__ flag, const int* __restrict__ pos,
                                                       long long n, SampleChunk* __restrict__ list,
                                                       long long* __restrict__ nruns)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) {
        if (flag[k]) {
            list[pos[k]].chunk = chunk_of[k];
            list[pos[k]].lo = k;
            if (pos[k] > 0) list[pos[k] - 1].hi = k;
        }
        if (k == n - 1) {
            const long long runs = (long long)pos[k] + flag[k];
            list[runs - 1].hi = n;
            *nruns = runs;
        }
    }
}

__global__ __launch_bounds__(kThreads) void k_scatter_outcomes(const long long* __restrict__ order,
                                                               const long long* __restrict__ got, long long n,
                                                               long long* __restrict__ out)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) out[order[k]] = got[k];
}

int grid_for(long long n) { return (int)std::min<long long>(4096, std::max<long long>(1, (n + kThreads - 1) / kThreads)); }

}  // namespace

size_t sample_assign_scratch(long long n)
{
    size_t temp = 0;
    (void)rocprim::exclusive_scan(nullptr, temp, (const int*)nullptr, (int*)nullptr, 0, (size_t)n, rocprim::plus<int>());
    return align256(sizeof(long long) * (size_t)n) + 2 * align256(sizeof(int) * (size_t)n) + align256(temp);
}

hipError_t sample_assign(const double* u, const long long* order, long long n, const double* cum, long long c0,
                         long long lastnz, double P, double* residual, SampleChunk* list, long long* nruns,
                         void* scratch, size_t scratch_bytes, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    unsigned char* p = static_cast<unsigned char*>(scratch);
    const size_t b64 = align256(sizeof(long long) * (size_t)n), b32 = align256(sizeof(int) * (size_t)n);
    if (scratch_bytes < b64 + 2 * b32) return hipErrorInvalidValue;
    long long* chunk_of = reinterpret_cast<long long*>(p);
    int* flag = reinterpret_cast<int*>(p + b64);
    int* pos = reinterpret_cast<int*>(p + b64 + b32);
    void* temp = p + b64 + 2 * b32;
    size_t temp_bytes = scratch_bytes - b64 - 2 * b32;
    const int g = grid_for(n);
    hipLaunchKernelGGL(k_assign_shots, dim3(g), dim3(kThreads), 0, s, u, order, n, cum, c0, lastnz, P, chunk_of,
                       residual);
    hipLaunchKernelGGL(k_run_starts, dim3(g), dim3(kThreads), 0, s, (const long long*)chunk_of, n, flag);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = rocprim::exclusive_scan(temp, temp_bytes, (const int*)flag, pos, 0, (size_t)n, rocprim::plus<int>(), s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_run_list, dim3(g), dim3(kThreads), 0, s, (const long long*)chunk_of, (const int*)flag,
                       (const int*)pos, n, list, nruns);
    return hipGetLastError();
}

hipError_t scatter_outcomes(const long long* order, const long long* got, long long n, long long* out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter_outcomes, dim3(grid_for(n)), dim3(kThreads), 0, s, order, got, n, out);
    return hipGetLastError();
}

}  // namespace qsv
