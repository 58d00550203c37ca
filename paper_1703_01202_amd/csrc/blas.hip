// BLAS-1 kernels and deterministic reductions for the Krylov solver (Sec. 4, Eq. (21)).
//
// Every reduction has a fixed grid: each of kRedBlocks blocks sums a fixed strided slice
// in a fixed order and writes one partial; the partials are summed in a fixed order by
// the host or by the consuming kernel (device_reduce.h).  Results are bitwise
// reproducible run to run, with no floating-point atomics.
#include "device_reduce.h"
#include "pfc_internal.h"

namespace pfc {
namespace {

constexpr int NT = kRedThreads;
constexpr int KG = 8;                  // vectors per pass of the multi-dot

// part[b] = block b's share of sum_i x_i y_i (y == nullptr: of sum_i x_i)
__global__ __launch_bounds__(NT) void k_dot(const double* __restrict__ x, const double* __restrict__ y,
                                            long n, double* __restrict__ part) {
    __shared__ double red[NT / 64];
    double acc = 0.0;
    for (long i = blockIdx.x * (long)NT + threadIdx.x; i < n; i += (long)gridDim.x * NT)
        acc += x[i] * (y ? y[i] : 1.0);
    const double s = block_sum_det(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// out[r] = scale * sum_b partials[r * count + b], one block per row r (for partials that
// a kernel without its own finishing step produced)
__global__ __launch_bounds__(NT) void k_reduce_rows(const double* __restrict__ part, int count,
                                                    double* __restrict__ out, double scale) {
    __shared__ double red[NT / 64];
    const double* row = part + (long)blockIdx.x * count;
    double acc = 0.0;
    for (int i = threadIdx.x; i < count; i += NT) acc += row[i];
    const double s = block_sum_det(acc, red);
    if (threadIdx.x == 0) out[blockIdx.x] = s * scale;
}

// part[j * gridDim + b] = block b's share of V_j . w for j0 <= j < j0 + KK.  The vector count
// is a template parameter so that the KK loads of an element are unconditional and in flight
// together (a runtime count made each load a branch with its own wait).
template <int KK>
__device__ __forceinline__ void multidot_pass(const double* __restrict__ V, long ld, int j0,
                                              const double* __restrict__ w, long n, double* __restrict__ part,
                                              double* red) {
    double acc[KK];
#pragma unroll
    for (int q = 0; q < KK; ++q) acc[q] = 0.0;
    for (long i = blockIdx.x * (long)NT + threadIdx.x; i < n; i += (long)gridDim.x * NT) {
        const double wi = w[i];
#pragma unroll
        for (int q = 0; q < KK; ++q) acc[q] += V[(long)(j0 + q) * ld + i] * wi;
    }
#pragma unroll
    for (int q = 0; q < KK; ++q) {
        const double t = block_sum_det(acc[q], red);
        if (threadIdx.x == 0) part[(long)(j0 + q) * gridDim.x + blockIdx.x] = t;
    }
}

// part[j * gridDim + b] = block b's share of V_j . w, j < k
__global__ __launch_bounds__(NT) void k_multidot(const double* __restrict__ V, long ld, int k,
                                                 const double* __restrict__ w, long n,
                                                 double* __restrict__ part) {
    __shared__ double red[NT / 64];
    for (int j0 = 0; j0 < k; j0 += KG) {
        switch (min(KG, k - j0)) {
            case 1: multidot_pass<1>(V, ld, j0, w, n, part, red); break;
            case 2: multidot_pass<2>(V, ld, j0, w, n, part, red); break;
            case 3: multidot_pass<3>(V, ld, j0, w, n, part, red); break;
            case 4: multidot_pass<4>(V, ld, j0, w, n, part, red); break;
            case 5: multidot_pass<5>(V, ld, j0, w, n, part, red); break;
            case 6: multidot_pass<6>(V, ld, j0, w, n, part, red); break;
            case 7: multidot_pass<7>(V, ld, j0, w, n, part, red); break;
            default: multidot_pass<8>(V, ld, j0, w, n, part, red); break;
        }
    }
}

// s + sum_{q < KK} sign * cf[j0 + q] * V_{j0+q}[i], added in order of q (loads unconditional)
template <int KK>
__device__ __forceinline__ double axpy_chunk(const double* __restrict__ V, long ld, int j0, long i,
                                             const double* cf, double sign, double s) {
    double v[KK];
#pragma unroll
    for (int q = 0; q < KK; ++q) v[q] = V[(long)(j0 + q) * ld + i];
#pragma unroll
    for (int q = 0; q < KK; ++q) s += sign * cf[j0 + q] * v[q];
    return s;
}

// s + sum_{j < k} sign * cf[j] * V_j[i], in order of j
__device__ __forceinline__ double axpy_all(const double* __restrict__ V, long ld, int k, long i, const double* cf,
                                           double sign, double s) {
    int j = 0;
    for (; j + KG <= k; j += KG) s = axpy_chunk<KG>(V, ld, j, i, cf, sign, s);
    switch (k - j) {
        case 1: return axpy_chunk<1>(V, ld, j, i, cf, sign, s);
        case 2: return axpy_chunk<2>(V, ld, j, i, cf, sign, s);
        case 3: return axpy_chunk<3>(V, ld, j, i, cf, sign, s);
        case 4: return axpy_chunk<4>(V, ld, j, i, cf, sign, s);
        case 5: return axpy_chunk<5>(V, ld, j, i, cf, sign, s);
        case 6: return axpy_chunk<6>(V, ld, j, i, cf, sign, s);
        case 7: return axpy_chunk<7>(V, ld, j, i, cf, sign, s);
        default: return s;
    }
}

// w <- w + sign * sum_j c_j V_j with c_j = sum_b coef_part[j * coef_n + b], k <= 64 (summed by
// every block in the same order; block 0 stores the c_j it used in coef_out).  With norm_part,
// also this block's share of ||w_new||^2.  assign: w starts from zero (not read).  With shift,
// sum(shift_part[0..shift_n)) * shift_scale is added to every w_i after the combination
// (the same additions k_shift would make afterwards).
__global__ __launch_bounds__(NT) void k_maxpy(const double* __restrict__ V, long ld, int k,
                                              const double* __restrict__ coef_part, int coef_n, double sign,
                                              double* __restrict__ w, long n, double* __restrict__ norm_part,
                                              double* __restrict__ coef_out, int assign,
                                              const double* __restrict__ shift_part, int shift_n,
                                              double shift_scale) {
    __shared__ double red[64 * (NT / 64)];
    __shared__ double cf[64];
    rows_sum_bcast(coef_part, k, coef_n, cf, red);
    if (coef_out && blockIdx.x == 0)
        for (int j = threadIdx.x; j < k; j += NT) coef_out[j] = cf[j];
    const double sh = shift_part ? shift_scale * sum_partials_bcast(shift_part, shift_n, red) : 0.0;
    double acc = 0.0;
    for (long i = blockIdx.x * (long)NT + threadIdx.x; i < n; i += (long)gridDim.x * NT) {
        double s = axpy_all(V, ld, k, i, cf, sign, assign ? 0.0 : w[i]);
        if (shift_part) s += sh;
        w[i] = s;
        acc += s * s;
    }
    if (norm_part) {
        const double t = block_sum_det(acc, red);
        if (threadIdx.x == 0) norm_part[blockIdx.x] = t;
    }
}

// One pass of Gram-Schmidt followed by the dots of the next one: w <- w + sign * sum_j c_j V_j
// exactly as k_maxpy, and this block's share of V_q . w_new (q < k <= KG) into
// dot_part[q * gridDim + b] exactly as k_multidot would compute it from the new w.
template <int KK>
__device__ __forceinline__ void maxpy_dot_body(const double* __restrict__ V, long ld, const double* cf, double sign,
                                               double* __restrict__ w, long n, double* __restrict__ dot_part,
                                               double* red) {
    double acc[KK];
#pragma unroll
    for (int q = 0; q < KK; ++q) acc[q] = 0.0;
    for (long i = blockIdx.x * (long)NT + threadIdx.x; i < n; i += (long)gridDim.x * NT) {
        double v[KK];
#pragma unroll
        for (int q = 0; q < KK; ++q) v[q] = V[(long)q * ld + i];
        double s = w[i];
#pragma unroll
        for (int j = 0; j < KK; ++j) s += sign * cf[j] * v[j];
        w[i] = s;
#pragma unroll
        for (int q = 0; q < KK; ++q) acc[q] += v[q] * s;
    }
#pragma unroll
    for (int q = 0; q < KK; ++q) {
        const double t = block_sum_det(acc[q], red);
        if (threadIdx.x == 0) dot_part[(long)q * gridDim.x + blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(NT) void k_maxpy_dot(const double* __restrict__ V, long ld, int k,
                                                  const double* __restrict__ coef_part, int coef_n, double sign,
                                                  double* __restrict__ w, long n, double* __restrict__ dot_part,
                                                  double* __restrict__ coef_out) {
    __shared__ double red[64 * (NT / 64)];
    __shared__ double cf[64];
    rows_sum_bcast(coef_part, k, coef_n, cf, red);
    if (coef_out && blockIdx.x == 0)
        for (int j = threadIdx.x; j < k; j += NT) coef_out[j] = cf[j];
    switch (k) {
        case 1: maxpy_dot_body<1>(V, ld, cf, sign, w, n, dot_part, red); break;
        case 2: maxpy_dot_body<2>(V, ld, cf, sign, w, n, dot_part, red); break;
        case 3: maxpy_dot_body<3>(V, ld, cf, sign, w, n, dot_part, red); break;
        case 4: maxpy_dot_body<4>(V, ld, cf, sign, w, n, dot_part, red); break;
        case 5: maxpy_dot_body<5>(V, ld, cf, sign, w, n, dot_part, red); break;
        case 6: maxpy_dot_body<6>(V, ld, cf, sign, w, n, dot_part, red); break;
        case 7: maxpy_dot_body<7>(V, ld, cf, sign, w, n, dot_part, red); break;
        case 8: maxpy_dot_body<8>(V, ld, cf, sign, w, n, dot_part, red); break;
        default: break;   // k is 1..KG (the launcher takes larger k apart)
    }
}

// w <- w / h with h = sqrt(sum(part[0..np))) (the Arnoldi normalisation, summed on the
// device); block 0 stores h in h_out.  w is left as it is when h is not positive.
__global__ __launch_bounds__(NT) void k_normalize(double* __restrict__ w, const double* __restrict__ part, int np,
                                                  long n, double* __restrict__ h_out) {
    __shared__ double red[NT / 64];
    const double h = sqrt(sum_partials_bcast(part, np, red));
    if (h_out && blockIdx.x == 0 && threadIdx.x == 0) *h_out = h;
    if (!(h > 0.0)) return;
    const double s = 1.0 / h;
    for (long i = blockIdx.x * (long)NT + threadIdx.x; i < n; i += (long)gridDim.x * NT) w[i] = s * w[i];
}

__global__ void k_axpby(double a, const double* __restrict__ x, double b, const double* __restrict__ y,
                        double* __restrict__ out, long n) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        out[i] = a * x[i] + (y ? b * y[i] : 0.0);
}

// x += scale * sum(part[0..np))
__global__ __launch_bounds__(256) void k_shift(double* __restrict__ x, const double* __restrict__ part, int np,
                                               double scale, long n) {
    __shared__ double red[4];
    const double v = scale * sum_partials_bcast(part, np, red);
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

hipError_t launch_dot(hipStream_t s, const double* x, const double* y, long n, double* partials) {
    hipLaunchKernelGGL(k_dot, dim3(kRedBlocks), dim3(NT), 0, s, x, y, n, partials);
    return hipGetLastError();
}

hipError_t launch_reduce_rows_n(hipStream_t s, const double* partials, int rows, int count, double* out,
                                double scale) {
    hipLaunchKernelGGL(k_reduce_rows, dim3(rows), dim3(NT), 0, s, partials, count, out, scale);
    return hipGetLastError();
}

hipError_t launch_multidot(hipStream_t s, const double* V, long ld, int k, const double* w, long n,
                           double* partials) {
    hipLaunchKernelGGL(k_multidot, dim3(kRedBlocks), dim3(NT), 0, s, V, ld, k, w, n, partials);
    return hipGetLastError();
}

hipError_t launch_maxpy(hipStream_t s, const double* V, long ld, int k, const double* coef_part, int coef_n,
                        double sign, double* w, long n, double* norm_part, double* coef_out, bool assign,
                        const double* shift_part, int shift_n, double shift_scale) {
    hipLaunchKernelGGL(k_maxpy, dim3(kRedBlocks), dim3(NT), 0, s, V, ld, k, coef_part, coef_n, sign, w, n,
                       norm_part, coef_out, assign ? 1 : 0, shift_part, shift_n, shift_scale);
    return hipGetLastError();
}

hipError_t launch_maxpy_dot(hipStream_t s, const double* V, long ld, int k, const double* coef_part, int coef_n,
                            double sign, double* w, long n, double* dot_part, double* coef_out) {
    if (k > KG) {   // beyond the fused pass: the two kernels
        hipError_t e = launch_maxpy(s, V, ld, k, coef_part, coef_n, sign, w, n, nullptr, coef_out);
        return e != hipSuccess ? e : launch_multidot(s, V, ld, k, w, n, dot_part);
    }
    hipLaunchKernelGGL(k_maxpy_dot, dim3(kRedBlocks), dim3(NT), 0, s, V, ld, k, coef_part, coef_n, sign, w, n,
                       dot_part, coef_out);
    return hipGetLastError();
}

hipError_t launch_normalize(hipStream_t s, double* w, const double* part, int np, long n, double* h_out) {
    hipLaunchKernelGGL(k_normalize, dim3(kRedBlocks), dim3(NT), 0, s, w, part, np, n, h_out);
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

hipError_t launch_shift(hipStream_t s, double* x, const double* part, int np, double scale, long n) {
    hipLaunchKernelGGL(k_shift, ew_grid(n), dim3(256), 0, s, x, part, np, scale, n);
    return hipGetLastError();
}

hipError_t launch_extrap(hipStream_t s, const double* phi, const double* prev, double ratio, double* out,
                         long n) {
    hipLaunchKernelGGL(k_extrap, ew_grid(n), dim3(256), 0, s, phi, prev, ratio, out, n);
    return hipGetLastError();
}

}  // namespace pfc
