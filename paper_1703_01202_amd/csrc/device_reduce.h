// Deterministic reductions for the library's kernels.
//
// A reducing kernel has a fixed grid; each block sums a fixed slice in a fixed order
// (shuffle tree, then its waves in order) and writes one partial per block.  The value is
// then formed, again in a fixed order, either on the host from the partials copied back,
// or inside the next kernel that needs it on the device, where every block sums the
// partials itself.  There is no floating-point atomic and no cross-block fence, and every
// result is bitwise reproducible run to run.
#pragma once

#include <hip/hip_runtime.h>

namespace pfc {

// Sum over the block, fixed order; valid in thread 0.
__device__ __forceinline__ double block_sum_det(double v, double* red) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
    return s;
}

// Sum of part[0..n) in a fixed order, returned to every thread of the block.
__device__ __forceinline__ double sum_partials_bcast(const double* __restrict__ part, int n, double* red) {
    __shared__ double bc;
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) acc += part[i];
    const double s = block_sum_det(acc, red);
    if (threadIdx.x == 0) bc = s;
    __syncthreads();
    return bc;
}

// out[j] = sum_i part[j * n + i] for every row j < rows, in a fixed order (thread-strided
// sums, wave shuffle tree, waves in order), into shared memory visible to the whole block.
// The rows are reduced side by side, so the block synchronises twice in all.
// red holds rows * (blockDim.x / 64) doubles.
__device__ __forceinline__ void rows_sum_bcast(const double* __restrict__ part, int rows, int n, double* out,
                                               double* red) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll 4
    for (int j = 0; j < rows; ++j) {
        double acc = 0.0;
        for (int i = threadIdx.x; i < n; i += blockDim.x) acc += part[(long)j * n + i];
        for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
        if (lane == 0) red[j * nw + wid] = acc;
    }
    __syncthreads();
    for (int j = threadIdx.x; j < rows; j += blockDim.x) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += red[j * nw + w];
        out[j] = s;
    }
    __syncthreads();
}

}  // namespace pfc
