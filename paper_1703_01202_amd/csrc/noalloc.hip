// The 2-D residual of Eq. (12) (Sec. 3) for callers that cannot allocate device memory: no
// solver context, no hipMalloc/hipFree.  The per-block partial sums of ||F||^2 that the
// residual kernel leaves go to a fixed device array in this file; F is the caller's.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "pfc.h"
#include "pfc_internal.h"

namespace {

// One partial sum per block of the residual kernel, whose persistent grid never exceeds
// 1024 blocks; 8 KiB, held by every GPU the library runs on until the process ends.
constexpr int kScratchDoubles = 1024;
__device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_scratch[kMaxDevices];   // device address of `scratch` on each device, looked up once

// Device address of this device's copy of `scratch` (the array's name is a host-side stand-in
// that must never reach a kernel or a copy).
hipError_t scratch_address(double** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch[dev] = static_cast<double*>(p);
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

}  // namespace

extern "C" pfc_status pfc_residual_noalloc(const pfc_grid* g, const pfc_model* m, const double* Phi,
                                           const double* phi, double dt, const double* src, double* F,
                                           double* norm2, void* stream) {
    if (!g || !m || !Phi || !phi || !F || !(dt > 0) || F == Phi || F == phi) return PFC_EINVAL;
    if (g->dim == 3) return PFC_EUNSUP;
    if (g->dim != 2 || g->n[0] < 8 || g->n[1] < 8 || !(g->L[0] > 0) || !(g->L[1] > 0) || m->mobility != 0 ||
        m->boundary != 0)
        return PFC_EINVAL;
    const int nx = g->n[0], ny = g->n[1];
    const int blocks = pfc::residual2d_blocks(nx, ny);
    if (blocks > kScratchDoubles) return PFC_EINVAL;   // more partial sums than the array holds
    double* part = nullptr;
    if (scratch_address(&part) != hipSuccess) return PFC_EHIP;
    const double hx = g->L[0] / nx, hy = g->L[1] / ny;   // as pfc_create forms them
    const hipStream_t s = static_cast<hipStream_t>(stream);
    if (pfc::launch_residual2d_plain(s, nx, ny, 1.0 / (hx * hx), 1.0 / (hy * hy), m->gamma, dt, Phi, phi, src, F,
                                     part) != hipSuccess)
        return PFC_EHIP;
    if (!norm2) return PFC_OK;
    double host[kScratchDoubles];
    if (hipMemcpyAsync(host, part, sizeof(double) * blocks, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return PFC_EHIP;
    double sum = 0.0;   // the order pfc_residual sums in
    for (int i = 0; i < blocks; ++i) sum += host[i];
    *norm2 = std::sqrt(sum);
    return std::isfinite(*norm2) ? PFC_OK : PFC_ENAN;
}
