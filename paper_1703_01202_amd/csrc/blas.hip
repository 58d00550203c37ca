// BLAS-1 kernels and deterministic reductions for the Krylov solver (Sec. 4, Eq. (21)).
//
// Every reduction is two-stage with a fixed grid: each of kRedBlocks blocks sums a
// fixed strided slice in a fixed order (shuffle tree, then waves in order), and one
// block per result sums the partials in a fixed order.  Results are therefore
// bitwise reproducible run to run.  No floating-point atomics are used.
#include "pfc_internal.h"

namespace pfc {
namespace {

constexpr int NT = kRedThreads;
constexpr int KG = 8;                  // vectors per pass of the multi-dot / multi-axpy

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// result valid in thread 0
__device__ __forceinline__ double block_sum(double v, double* red) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < NT / 64; ++i) s += red[i];
    return s;
}

__global__ __launch_bounds__(NT) void k_dot(const double* __restrict__ x, const double* __restrict__ y,
                                            long n, double* __restrict__ part) {
    __shared__ double red[NT / 64];
    double acc = 0.0;
    for (long i = blockIdx.x * (long)NT + threadIdx.x; i < n; i += (long)gridDim.x * NT)
        acc += x[i] * (y ? y[i] : 1.0);
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// out[r] = scale * sum_b partials[r * count + b], one block per row r
__global__ __launch_bounds__(NT) void k_reduce_rows(const double* __restrict__ part, int count,
                                                    double* __restrict__ out, double scale) {
    __shared__ double red[NT / 64];
    const double* row = part + (long)blockIdx.x * count;
    double acc = 0.0;
    for (int i = threadIdx.x; i < count; i += NT) acc += row[i];
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) out[blockIdx.x] = s * scale;
}

// partials[j * gridDim + b] = sum over block b's slice of V_j . w, j < k
__global__ __launch_bounds__(NT) void k_multidot(const double* __restrict__ V, long ld, int k,
                                                 const double* __restrict__ w, long n,
                                                 double* __restrict__ part) {
    __shared__ double red[NT / 64];
    for (int j0 = 0; j0 < k; j0 += KG) {
        double acc[KG];
#pragma unroll
        for (int q = 0; q < KG; ++q) acc[q] = 0.0;
        const int kk = min(KG, k - j0);
        for (long i = blockIdx.x * (long)NT + threadIdx.x; i < n; i += (long)gridDim.x * NT) {
            const double wi = w[i];
#pragma unroll
            for (int q = 0; q < KG; ++q)
                if (q < kk) acc[q] += V[(long)(j0 + q) * ld + i] * wi;
        }
#pragma unroll
        for (int q = 0; q < KG; ++q) {
            if (q < kk) {
                const double s = block_sum(acc[q], red);
                if (threadIdx.x == 0) part[(long)(j0 + q) * gridDim.x + blockIdx.x] = s;
            }
        }
    }
}

// w <- w + sign * sum_j coef[j] V_j ; optional partial sums of the new w^2
__global__ __launch_bounds__(NT) void k_maxpy(const double* __restrict__ V, long ld, int k,
                                              const double* __restrict__ coef, double sign,
                                              double* __restrict__ w, long n,
                                              double* __restrict__ part) {
    __shared__ double red[NT / 64];
    __shared__ double cf[64];
    for (int j = threadIdx.x; j < k; j += NT) cf[j] = sign * coef[j];
    __syncthreads();
    double acc = 0.0;
    for (long i = blockIdx.x * (long)NT + threadIdx.x; i < n; i += (long)gridDim.x * NT) {
        double s = w[i];
        for (int j = 0; j < k; ++j) s += cf[j] * V[(long)j * ld + i];
        w[i] = s;
        acc += s * s;
    }
    if (part) {
        const double t = block_sum(acc, red);
        if (threadIdx.x == 0) part[blockIdx.x] = t;
    }
}

__global__ void k_axpby(double a, const double* __restrict__ x, double b, const double* __restrict__ y,
                        double* __restrict__ out, long n) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        out[i] = a * x[i] + (y ? b * y[i] : 0.0);
}

__global__ void k_shift(double* __restrict__ x, const double* __restrict__ s, double sign, long n) {
    const double v = sign * (*s);
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        x[i] += v;
}

__global__ void k_extrap(const double* __restrict__ phi, const double* __restrict__ prev, double ratio,
                         double* __restrict__ out, long n) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        out[i] = phi[i] + ratio * (phi[i] - prev[i]);
}

inline dim3 ew_grid(long n) {
    long b = (n + 255) / 256;
    return dim3((unsigned)(b < 4096 ? (b < 1 ? 1 : b) : 4096));
}

}  // namespace

hipError_t launch_dot_partials(hipStream_t s, const double* x, const double* y, long n, double* partials) {
    hipLaunchKernelGGL(k_dot, dim3(kRedBlocks), dim3(NT), 0, s, x, y, n, partials);
    return hipGetLastError();
}

hipError_t launch_sum_partials(hipStream_t s, const double* x, long n, double* partials) {
    hipLaunchKernelGGL(k_dot, dim3(kRedBlocks), dim3(NT), 0, s, x, nullptr, n, partials);
    return hipGetLastError();
}

hipError_t launch_reduce_rows_n(hipStream_t s, const double* partials, int rows, int count, double* out,
                                double scale) {
    hipLaunchKernelGGL(k_reduce_rows, dim3(rows), dim3(NT), 0, s, partials, count, out, scale);
    return hipGetLastError();
}

hipError_t launch_reduce_rows(hipStream_t s, const double* partials, int rows, double* out, double scale) {
    return launch_reduce_rows_n(s, partials, rows, kRedBlocks, out, scale);
}

hipError_t launch_multidot(hipStream_t s, const double* V, long ld, int k, const double* w, long n,
                           double* partials) {
    hipLaunchKernelGGL(k_multidot, dim3(kRedBlocks), dim3(NT), 0, s, V, ld, k, w, n, partials);
    return hipGetLastError();
}

hipError_t launch_maxpy(hipStream_t s, const double* V, long ld, int k, const double* coef, double sign,
                        double* w, long n, double* norm_partials) {
    hipLaunchKernelGGL(k_maxpy, dim3(kRedBlocks), dim3(NT), 0, s, V, ld, k, coef, sign, w, n, norm_partials);
    return hipGetLastError();
}

hipError_t launch_axpby(hipStream_t s, double a, const double* x, double b, const double* y, double* out,
                        long n) {
    hipLaunchKernelGGL(k_axpby, ew_grid(n), dim3(256), 0, s, a, x, b, y, out, n);
    return hipGetLastError();
}

hipError_t launch_scale(hipStream_t s, const double* x, double a, double* out, long n) {
    return launch_axpby(s, a, x, 0.0, nullptr, out, n);
}

hipError_t launch_shift(hipStream_t s, double* x, const double* dev_scalar, double sign, long n) {
    hipLaunchKernelGGL(k_shift, ew_grid(n), dim3(256), 0, s, x, dev_scalar, sign, n);
    return hipGetLastError();
}

hipError_t launch_extrap(hipStream_t s, const double* phi, const double* prev, double ratio, double* out,
                         long n) {
    hipLaunchKernelGGL(k_extrap, ew_grid(n), dim3(256), 0, s, phi, prev, ratio, out, n);
    return hipGetLastError();
}

}  // namespace pfc
