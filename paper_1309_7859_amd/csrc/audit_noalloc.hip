// audit_noalloc.hip -- the Gauss audit for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops, harnesses
// that forbid hipMalloc): memd_gauss_residual_noalloc runs the kernels of
// memd_gauss_residual on caller-owned device buffers and keeps what they
// produce on the way (the charge assignment and the per-block partials) in
// one fixed device-resident array instead of allocations.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "memd_internal.hpp"

using namespace memd;

namespace {

constexpr int kNoAllocMaxL = 128;
constexpr size_t kNoAllocMaxNs = (size_t)kNoAllocMaxL * kNoAllocMaxL * kNoAllocMaxL;
// Layout in doubles: the charge assignment rho[kNoAllocMaxNs], the audit's
// partials[2 * kSiteBlocks], the result (max, rms).
constexpr size_t kRhoOff = 0;
constexpr size_t kPartOff = kNoAllocMaxNs;
constexpr size_t kResOff = kPartOff + 2 * (size_t)kSiteBlocks;
constexpr size_t kScratchDoubles = kResOff + 32;  // 16 MiB + 128 KiB + 256 B

// Each GPU the library runs on holds its own copy until the process ends.
// Host code never uses this name as an address: the per-device address comes
// from hipGetSymbolAddress below.
__device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double *g_scratch[kMaxDevices];  // device address of `scratch` per device (null until looked up)

// The array's address on the current device, looked up once per device with
// that device current.
memd_status scratch_on_current_device(int *dev_out, double **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return MEMD_EDEVICE;
    }
    if (dev < 0 || dev >= kMaxDevices) return MEMD_EDEVICE;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return MEMD_EDEVICE;
        }
        g_scratch[dev] = (double *)p;
    }
    *dev_out = dev;
    *out = g_scratch[dev];
    return MEMD_OK;
}

// 1: device memory of device `dev`; 0: anything else (host memory, another
// device, an unknown pointer).
bool on_device(const void *p, int dev) {
    hipPointerAttribute_t at;
    if (hipPointerGetAttributes(&at, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return at.type == hipMemoryTypeDevice && at.device == dev;
}

}  // namespace

extern "C" {

memd_status memd_gauss_residual_noalloc(int L, double a, int n, const double *q, const double *r,
                                        const void *D, int precision, double *out, void *hip_stream) {
    if (L < 2 || !(a > 0.0) || !std::isfinite(a) || n < 0 || !D || !out || (n > 0 && (!q || !r)))
        return MEMD_EINVAL;
    if (precision != MEMD_FP64 && precision != MEMD_FP32_MIXED) return MEMD_EINVAL;
    if (L > kNoAllocMaxL) return MEMD_ESIZE;
    int dev = -1;
    double *sc = nullptr;
    const memd_status st = scratch_on_current_device(&dev, &sc);
    if (st != MEMD_OK) return st;
    if (!on_device(D, dev) || (n > 0 && (!on_device(q, dev) || !on_device(r, dev)))) return MEMD_EINVAL;
    const bool out_dev = on_device(out, dev);
    hipStream_t s = (hipStream_t)hip_stream;
    const size_t Ns = (size_t)L * L * L;
    double *rho = sc + kRhoOff, *partials = sc + kPartOff, *res = sc + kResOff;
    int nb = 0;
    // the assignment accumulates with atomics: its vertices start at zero
    // (a fill kernel, so that the sequence can be captured in a graph)
    if (launch_fill(s, rho, 0.0, Ns) != hipSuccess) return MEMD_EDEVICE;
    if (launch_spread_raw(s, n, L, a, q, r, rho) != hipSuccess) return MEMD_EDEVICE;
    if (launch_audit_raw(s, D, precision == MEMD_FP32_MIXED, rho, L, a, partials, &nb) != hipSuccess)
        return MEMD_EDEVICE;
    if (launch_finalize_audit(s, partials, nb, (double)Ns, out_dev ? out : res, nullptr) != hipSuccess)
        return MEMD_EDEVICE;
    if (!out_dev) {
        if (hipMemcpyAsync(out, res, 2 * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            (void)hipGetLastError();
            return MEMD_EDEVICE;
        }
    }
    return MEMD_OK;
}

}  // extern "C"
