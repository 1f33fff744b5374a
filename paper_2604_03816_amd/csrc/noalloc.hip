// noalloc.hip -- qsv_norm_noalloc: the squared norm of a device state vector with no
// allocation of any kind, for callers that cannot allocate (code under stream or graph
// capture, tight serving loops).
//
// It runs the same reduction kernel as qsv_norm (k_norm: FP64 per thread, a fixed-order
// tree per workgroup, one (sum, compensation) pair per workgroup), but the workgroup
// partials go to `scratch`, a file-scope device array of fixed size, instead of a
// per-state workspace, and one more single-thread kernel combines them in workgroup
// order with the same Neumaier sequence as qsv_norm's host combine, writing the result
// to the caller's device double.  The result is therefore bit-identical to qsv_norm's.
//
// `scratch` is per device (each GPU the library runs on holds its own copy until the
// process ends).  In host code its name is only a host-side stand-in, so its device
// address is fetched once per device with hipGetSymbolAddress and kept; kernels receive
// that address.  Every call on one device shares the array: calls that overlap on one
// device (different streams, or different host threads without ordering) race.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/qsv.h"
#include "qsv_internal.h"

namespace qsv {

qsv_status set_error(qsv_status st, const std::string& msg);   // capi.cpp

namespace {

// The norm kernel's grid never exceeds 1024 workgroups (norm_grid); two doubles each:
// 16 KiB per device.
constexpr int kNoallocPartials = 1024;
constexpr int kMaxDevices = 64;

}  // namespace

static __device__ __align__(256) double scratch[2 * kNoallocPartials];

namespace {

// Workgroup partials (sum, compensation) combined in workgroup order: the sums through
// Neumaier's compensated addition, the compensations added to the running correction
// (the host combine of qsv_norm, step for step).
__global__ void k_norm_combine(const double* __restrict__ partial, int grid, double* __restrict__ out)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    double s = 0.0, c = 0.0;
    for (int b = 0; b < grid; ++b) {
        const double x = partial[2 * b];
        const double t = s + x;
        c += (fabs(s) >= fabs(x)) ? ((s - t) + x) : ((x - t) + s);
        s = t;
        c += partial[2 * b + 1];
    }
    out[0] = s + c;
}

std::mutex g_mu;
double* g_scratch[kMaxDevices] = {};   // device address of `scratch`, per device

// The device address of `scratch` on the current device, fetched once per device.
qsv_status scratch_on_current_device(double** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return set_error(QSV_E_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return set_error(QSV_E_UNSUPPORTED, "device index beyond 63");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_error(QSV_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch[dev] = static_cast<double*>(p);
    }
    *out = g_scratch[dev];
    return QSV_OK;
}

}  // namespace
}  // namespace qsv

using namespace qsv;

extern "C" qsv_status qsv_norm_noalloc(const void* amps, int n_qubits, qsv_dtype dtype, double* out_dev,
                                       void* stream)
{
    if (!amps || !out_dev) return set_error(QSV_E_ARG, "amps and out_dev must be device pointers");
    if (dtype != QSV_C64 && dtype != QSV_C128) return set_error(QSV_E_ARG, "dtype must be QSV_C64 or QSV_C128");
    if (n_qubits < 1 || n_qubits > kMaxQubits) return set_error(QSV_E_ARG, "n_qubits must be in [1, 34]");
    if ((reinterpret_cast<uintptr_t>(amps) & 15) != 0) return set_error(QSV_E_ARG, "amps must be 16-byte aligned");
    const long long N = 1ll << n_qubits;
    const int grid = norm_grid(N);
    if (grid > kNoallocPartials) return set_error(QSV_E_UNSUPPORTED, "state needs more partials than the scratch holds");
    double* sp = nullptr;
    qsv_status st = scratch_on_current_device(&sp);
    if (st != QSV_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    // every partial the combine reads is written by this call's norm launch (one per
    // workgroup), so nothing in the array needs clearing first
    hipError_t e = launch_norm(dtype == QSV_C64 ? 0 : 1, amps, N, sp, grid, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_norm_combine, dim3(1), dim3(64), 0, s, (const double*)sp, grid, out_dev);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return set_error(QSV_E_DEVICE, std::string("norm launch: ") + hipGetErrorString(e));
    return QSV_OK;
}
