// Learned Newton initial guess: a four-layer 3x3 periodic convolutional network with
// hand-written forward, backward and Adam kernels for gfx950 (C ABI in include/pfc_net.h).
//
// Layouts
//   input x      planar FP32 [2][HW]
//   activations  groups of four channels, [8][HW] x 16 bytes: the four values of a cell as
//                hi = bf16(a) and lo = bf16(a - hi) (hi0..hi3 then lo0..lo3), so that one
//                16-byte load gives both matrix-core operands; the value is hi + lo (exact
//                in FP32, |a - hi - lo| <= 2^-17 |a|); 32 cells of a group are 512 bytes
//   output y     FP32 [HW]
// The two 32 -> 32 layers are a dense contraction (K = 9 taps x 32 channels = 288) and run
// on the matrix cores: v_mfma_f32_32x32x16 bf16 with the 32 output channels as M, 32
// consecutive cells as N and (tap, 16 input channels) as K, once for the hi and once for
// the lo parts of the activations.  Both parts of each stored
// activation are multiplied by the bf16 weight, so the products carry ~16 significant bits
// of the activation and accumulate in FP32.  The split is made once, by the producing
// kernel.  The thin first (2 -> 32) and last (32 -> 1) layers and the weight gradients use
// FP32 FMA with the weights read as wave-uniform (scalar-register) operands.
// Reductions (loss, weight gradients) leave per-block partials summed in a fixed order.
#include <cmath>
#include <cstring>
#include <string>

#include "../../include/pfc_net.h"
#include "device_reduce.h"
#include "pfc_internal.h"

namespace pfc {
namespace {

constexpr int CIN = PFC_NET_CIN, WID = PFC_NET_WIDTH, NG = WID / 4;
constexpr int OFF_W1 = 0, OFF_B1 = 576, OFF_W2 = 608, OFF_B2 = 9824, OFF_W3 = 9856, OFF_B3 = 19072,
              OFF_W4 = 19104, OFF_B4 = 19392, OFF_U1 = 19393;
constexpr int NPARAM = PFC_NET_NPARAM;
static_assert(OFF_U1 + WID == NPARAM, "parameter layout");
constexpr int KSTEPS = 18;                 // 9 taps x 2 blocks of 16 input channels
constexpr int PACK = KSTEPS * 64;          // packed A operands (8 bf16 each) per layer and direction
constexpr int PACK4 = 2 * 64;              // packed A operands of the output layer's tap sums
constexpr int PACK1 = 2 * 64;              // packed A operands of the first layer (inference)
constexpr int PACK_ALL = 4 * PACK + PACK4 + PACK1;
constexpr int WG_BLOCKS = 256;             // fixed grid of the weight-gradient kernels
constexpr int WG_MAXOUT = WID * WID * 9 + WID;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));   // staging registers (a native vector stays in VGPRs)

__device__ __forceinline__ unsigned short f2bf(float f) {   // round to nearest, ties to even
    unsigned u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float((unsigned)h << 16); }
__device__ __forceinline__ int wrap1(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }
__device__ __forceinline__ int wrapm(int i, int n) { return ((i % n) + n) % n; }

// four activations -> hi/lo bf16 pairs in one 16-byte word (see the layout above); the
// conversions are gfx950's packed FP32 -> bf16 instruction (round to nearest, ties to even,
// the same rounding as f2bf for finite values)
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ unsigned pk_bf16(float a, float b) {
    const bf16x2 h = {(__bf16)a, (__bf16)b};
    return __builtin_bit_cast(unsigned, h);
}
__device__ __forceinline__ uint4 split4(float a0, float a1, float a2, float a3) {
    const unsigned h01 = pk_bf16(a0, a1), h23 = pk_bf16(a2, a3);
    const unsigned l01 = pk_bf16(a0 - __uint_as_float(h01 << 16), a1 - __uint_as_float(h01 & 0xFFFF0000u));
    const unsigned l23 = pk_bf16(a2 - __uint_as_float(h23 << 16), a3 - __uint_as_float(h23 & 0xFFFF0000u));
    return make_uint4(h01, h23, l01, l23);
}
__device__ __forceinline__ float4 join4(uint4 u) {
    return make_float4(__uint_as_float(u.x << 16) + __uint_as_float(u.z << 16),
                       __uint_as_float(u.x & 0xFFFF0000u) + __uint_as_float(u.z & 0xFFFF0000u),
                       __uint_as_float(u.y << 16) + __uint_as_float(u.w << 16),
                       __uint_as_float(u.y & 0xFFFF0000u) + __uint_as_float(u.w & 0xFFFF0000u));
}
__device__ __forceinline__ const uint4* grp(const float* base, long g, long HW, long p) {
    return reinterpret_cast<const uint4*>(base) + g * HW + p;
}
__device__ __forceinline__ uint4* grp(float* base, long g, long HW, long p) {
    return reinterpret_cast<uint4*>(base) + g * HW + p;
}

// tanh from one exponential: sign(z) (1 - 2 / (exp(2|z|) + 1)), the reciprocal taken by the
// hardware's approximate v_rcp_f32 (about 1 ulp) instead of a correctly rounded division;
// absolute error ~2e-7.  exp overflowing to inf gives 1 exactly.
__device__ __forceinline__ float tanh_fast(float z) {
    const float e = __expf(2.f * fabsf(z));
    return copysignf(1.f - 2.f * __builtin_amdgcn_rcpf(e + 1.f), z);
}

__device__ __forceinline__ bool is_weight_index(int i) {
    return i < OFF_B1 || (i >= OFF_W2 && i < OFF_B2) || (i >= OFF_W3 && i < OFF_B3) || (i >= OFF_W4 && i < OFF_B4);
}

// q = parameters with the convolution weights rounded to bf16; pack = matrix-core A operands
// of the inner layers: set 0/1 layer 2 forward/backward, set 2/3 layer 3.  Entry
// [set][s][lane][e], step s = tap * 2 + j, row m = lane % 32, k = 16 j + 8 (lane / 32) + e:
//   forward  A[m = out ch][k = in ch] = W[m][k][tap]
//   backward A[m = in ch][k = out ch] = W[k][m][8 - tap]  (adjoint: swap channels, mirror taps)
// Then the output layer's operand [j][lane][e] (j = 0, 1), row m = tap (zero for m >= 9):
//   A[m][k] = W4[c(k)][m],  k = 16 j + 8 h + e,  c(k) = 16 j + 8 (e / 4) + 4 h + e % 4,  h = lane / 32,
// the channel order in which a lane of the inner layers' accumulator holds its outputs.
// Last the first layer's operand [j][lane][e], row m = out channel, k = 16 j + 8 h + e:
//   A[m][k] = W1[m][k % 2][k / 2] for k < 18 (tap k / 2, input channel k % 2), zero beyond.
__global__ void k_prepare(const float* __restrict__ theta, float* __restrict__ q, unsigned short* __restrict__ pack) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < NPARAM) q[i] = is_weight_index(i) ? bf2f(f2bf(theta[i])) : theta[i];
    if (i < 4 * PACK * 8) {
        const int set = i / (PACK * 8), r = i % (PACK * 8);
        const int st = r / 512, lane = (r / 8) % 64, e = r % 8;
        const int tap = st / 2, j = st % 2;
        const int m = lane % 32, k = 16 * j + 8 * (lane / 32) + e;
        const int woff = set < 2 ? OFF_W2 : OFF_W3;
        const int idx = (set & 1) ? woff + (k * WID + m) * 9 + (8 - tap) : woff + (m * WID + k) * 9 + tap;
        pack[i] = f2bf(theta[idx]);
    } else if (i < (4 * PACK + PACK4) * 8) {
        const int r = i - 4 * PACK * 8;
        const int j = r / 512, lane = (r / 8) % 64, e = r % 8;
        const int m = lane % 32, h = lane / 32;
        const int c = 16 * j + 8 * (e / 4) + 4 * h + e % 4;
        pack[i] = m < 9 ? f2bf(theta[OFF_W4 + c * 9 + m]) : (unsigned short)0;
    } else if (i < PACK_ALL * 8) {
        const int r = i - (4 * PACK + PACK4) * 8;
        const int j = r / 512, lane = (r / 8) % 64, e = r % 8;
        const int m = lane % 32, k = 16 * j + 8 * (lane / 32) + e;
        pack[i] = k < 2 * 9 ? f2bf(theta[OFF_W1 + (m * CIN + k % 2) * 9 + k / 2]) : (unsigned short)0;
    }
}

// layer 1 at cell (y, x): the 32 channels of a1 = tanh(conv(x; W1) + b1) as 8 split groups
__device__ __forceinline__ void layer1_cell(const float* __restrict__ x, const float* __restrict__ q,
                                            const float* __restrict__ b1, long HW, int ny, int nx, int y, int xx,
                                            uint4* out) {
    float in[CIN][9];
#pragma unroll
    for (int dy = 0; dy < 3; ++dy) {
        const long row = (long)wrap1(y + dy - 1, ny) * nx;
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
            const long qi = row + wrap1(xx + dx - 1, nx);
#pragma unroll
            for (int c = 0; c < CIN; ++c) in[c][dy * 3 + dx] = x[c * HW + qi];
        }
    }
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        float o[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int co = 4 * g + j;
            float z = b1[co];
#pragma unroll
            for (int c = 0; c < CIN; ++c)
#pragma unroll
                for (int t = 0; t < 9; ++t) z += q[OFF_W1 + (co * CIN + c) * 9 + t] * in[c][t];
            o[j] = tanh_fast(z);
        }
        out[g] = split4(o[0], o[1], o[2], o[3]);
    }
}

// layer 1: a1 = tanh(conv(x; W1) + b1c), x planar [2][HW], a1 grouped and split; b1c the
// bias with the step-size term (k_cond_bias)
__global__ __launch_bounds__(256) void k_in_fwd(const float* __restrict__ x, const float* __restrict__ q,
                                                const float* __restrict__ b1c, float* __restrict__ a1, int ny,
                                                int nx) {
    const long HW = (long)ny * nx;
    const long p = blockIdx.x * (long)blockDim.x + threadIdx.x;   // one cell per thread
    if (p >= HW) return;
    const int y = (int)(p / nx), xx = (int)(p - (long)y * nx);
    uint4 o[NG];
    layer1_cell(x, q, b1c, HW, ny, nx, y, xx, o);
#pragma unroll
    for (int g = 0; g < NG; ++g) *grp(a1, g, HW, p) = o[g];
}

// Block tiles of CT_X x CT_Y cells; the tile and its one-cell periodic halo are staged in
// LDS as [row][channel group][column] 16-byte groups, so a wave's 32 lanes read 512
// contiguous bytes per operand and global memory is read once per tile.
constexpr int CT_X = 32, CT_Y = 8, CT_R = CT_Y + 2, CT_C = CT_X + 2;

constexpr int ST_N = CT_R * NG * CT_C;        // 16-byte groups of a staged tile
constexpr int ST_IT = (ST_N + 255) / 256;     // per thread of a 256-thread block

// Halo staging in two phases: each thread issues its ST_IT global loads into registers
// (tile_load), and only then writes them to LDS (tile_store), so the whole tile is in flight
// at once; a persistent block loads its next tile while it computes the current one.  The
// registers are a native vector type, which the compiler keeps in VGPRs (an array of the
// HIP uint4 class was left in scratch memory).
// Grids of at least CT_R rows and CT_C columns: every halo index is within [-n, 2n), one
// select each way wraps it (no division, no branch, so the unrolled loads stay in registers).
__device__ __forceinline__ void tile_load(u32x4 (&v)[ST_IT], const float* __restrict__ in, long HW, int ny, int nx,
                                          int y0, int x0) {
#pragma unroll
    for (int k = 0; k < ST_IT; ++k) {
        const int e = threadIdx.x + 256 * k;
        const int c = e % CT_C, g = (e / CT_C) % NG, r = e / (CT_C * NG);
        int yy = y0 + r - 1, xx = x0 + c - 1;
        yy += yy < 0 ? ny : 0;
        yy -= yy >= ny ? ny : 0;
        xx += xx < 0 ? nx : 0;
        xx -= xx >= nx ? nx : 0;
        if (k < ST_IT - 1 || e < ST_N) v[k] = *reinterpret_cast<const u32x4*>(grp(in, g, HW, (long)yy * nx + xx));
    }
}
// Any grid size, one load at a time (small grids only).
__device__ __forceinline__ void stage_tile(uint4 (*sm)[NG][CT_C], const float* __restrict__ in, long HW, int ny,
                                           int nx, int y0, int x0) {
    const bool one_wrap = ny >= CT_R && nx >= CT_C;
    for (int e = threadIdx.x; e < CT_R * NG * CT_C; e += blockDim.x) {
        const int c = e % CT_C, g = (e / CT_C) % NG, r = e / (CT_C * NG);
        const int yy = one_wrap ? wrap1(y0 + r - 1, ny) : wrapm(y0 + r - 1, ny);
        const int xx = one_wrap ? wrap1(x0 + c - 1, nx) : wrapm(x0 + c - 1, nx);
        sm[r][g][c] = *grp(in, g, HW, (long)yy * nx + xx);
    }
}
__device__ __forceinline__ void tile_store(uint4 (*sm)[NG][CT_C], const u32x4 (&v)[ST_IT]) {
    u32x4* flat = reinterpret_cast<u32x4*>(&sm[0][0][0]);   // flat index e = (r * NG + g) * CT_C + c
#pragma unroll
    for (int k = 0; k < ST_IT; ++k) {
        const int e = threadIdx.x + 256 * k;
        if (e < ST_N) flat[e] = v[k];
    }
}

// One block tile of an inner layer from the staged halo tile sm: the matrix-core product
// and the MODE's epilogue (see conv32_body).
template <int MODE>
__device__ __forceinline__ void conv_tile(const uint4 (*sm)[NG][CT_C], const bf16x8 (&A)[KSTEPS],
                                          const bf16x8 (&A4)[2], const float* __restrict__ bias,
                                          const float* __restrict__ aux, float* __restrict__ out, long HW, int ny,
                                          int nx, int x0, int y0) {
    const int lane = threadIdx.x & 63, half = lane >> 5, col = lane & 31, wv = threadIdx.x >> 6;
    const int ly0 = 2 * wv;                 // this wave's rows ly0, ly0 + 1 (CT_Y = 8)
    f32x16 acc2[2] = {{}, {}};
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int dx = 0; dx < 3; ++dx)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                // channels 16 j + 8 half + 0..7 = groups 4 j + 2 half and the next one
                const uint4 u0 = sm[ly0 + r][4 * j + 2 * half][col + dx];
                const uint4 u1 = sm[ly0 + r][4 * j + 2 * half + 1][col + dx];
                const bf16x8 hi = __builtin_bit_cast(bf16x8, make_uint4(u0.x, u0.y, u1.x, u1.y));
                const bf16x8 lo = __builtin_bit_cast(bf16x8, make_uint4(u0.z, u0.w, u1.z, u1.w));
                if (r <= 2) {                // row ly0, tap dy = r
                    const int s = (r * 3 + dx) * 2 + j;
                    acc2[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[s], hi, acc2[0], 0, 0, 0);
                    acc2[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[s], lo, acc2[0], 0, 0, 0);
                }
                if (r >= 1) {                // row ly0 + 1, tap dy = r - 1
                    const int s = ((r - 1) * 3 + dx) * 2 + j;
                    acc2[1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[s], hi, acc2[1], 0, 0, 0);
                    acc2[1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[s], lo, acc2[1], 0, 0, 0);
                }
            }
#pragma unroll
    for (int rr = 0; rr < 2; ++rr) {
        const f32x16& acc = acc2[rr];
        const int y = y0 + ly0 + rr, x = x0 + col;
        const bool inside = y < ny && x < nx;
        const long p = (long)y * nx + x;
        // lane holds cell p and output channels 8 (r / 4) + 4 half + r % 4, r = 0..15
        if (MODE == 2) {
            float a[16];
#pragma unroll
            for (int q4 = 0; q4 < 4; ++q4)
#pragma unroll
                for (int e = 0; e < 4; ++e) a[4 * q4 + e] = tanh_fast(acc[4 * q4 + e] + bias[4 * (2 * q4 + half) + e]);
            // B operand j holds a[8 j .. 8 j + 7], the channel order the pack4 rows assume;
            // every lane takes part in the product, only cells of the grid are stored
            f32x16 d = {};
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const uint4 u0 = split4(a[8 * j], a[8 * j + 1], a[8 * j + 2], a[8 * j + 3]);
                const uint4 u1 = split4(a[8 * j + 4], a[8 * j + 5], a[8 * j + 6], a[8 * j + 7]);
                const bf16x8 hi = __builtin_bit_cast(bf16x8, make_uint4(u0.x, u0.y, u1.x, u1.y));
                const bf16x8 lo = __builtin_bit_cast(bf16x8, make_uint4(u0.z, u0.w, u1.z, u1.w));
                d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A4[j], hi, d, 0, 0, 0);
                d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A4[j], lo, d, 0, 0, 0);
            }
            // d[i] is tap row 8 (i / 4) + 4 half + i % 4: taps 0-3 and 8 (half 0), 4-7 (half 1)
            if (inside) {
#pragma unroll
                for (int i = 0; i < 4; ++i) out[(4 * half + i) * HW + p] = d[i];
                if (half == 0) out[8 * HW + p] = d[4];
            }
            continue;
        }
        if (!inside) continue;
#pragma unroll
        for (int q4 = 0; q4 < 4; ++q4) {
            const int cg = 2 * q4 + half;
            float v[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) v[e] = acc[4 * q4 + e];
            if (MODE == 0) {
#pragma unroll
                for (int e = 0; e < 4; ++e) v[e] = tanh_fast(v[e] + bias[4 * cg + e]);
            } else {
                const float4 a = join4(*grp(aux, cg, HW, p));
                v[0] *= 1.f - a.x * a.x;
                v[1] *= 1.f - a.y * a.y;
                v[2] *= 1.f - a.z * a.z;
                v[3] *= 1.f - a.w * a.w;
            }
            *grp(out, cg, HW, p) = split4(v[0], v[1], v[2], v[3]);
        }
    }
}
static_assert(CT_Y == 8, "conv_tile gives each of its 4 waves two rows");

// inner layers on the matrix cores.  MODE 0: out = tanh(conv(in) + bias) (forward);
// MODE 1: out = conv(in) * (1 - aux^2) (backward through the previous tanh, aux = its output);
// MODE 2: the last inner layer of an inference pass: a = tanh(conv(in) + bias) stays in
// registers and the output layer's per-tap sums s_t(p) = sum_c W4[c][t] a[c](p) are written
// instead, out = planar FP32 [9][HW] (a 32x32x16 product with the taps as rows, pack4).
// Each of the 4 waves computes two rows of 32 cells x 32 output channels of a block tile,
// reading each of the 4 input rows it needs once for both.  Persistent blocks walk a
// tiles with a stride of the grid size (so the tiles in work at any time form one band of the
// image), with the 18 A operands in registers, loading the next tile's halo while they
// compute the current one.
template <int MODE>
__device__ __forceinline__ void conv32_body(const float* __restrict__ in, const bf16x8* __restrict__ pack,
                                            const float* __restrict__ bias, const float* __restrict__ aux,
                                            const bf16x8* __restrict__ pack4, float* __restrict__ out, int ny,
                                            int nx) {
    __shared__ uint4 sm[CT_R][NG][CT_C];
    const int lane = threadIdx.x & 63;
    const long HW = (long)ny * nx;
    const int ntx = (nx + CT_X - 1) / CT_X, nty = (ny + CT_Y - 1) / CT_Y;
    const int ntiles = ntx * nty;
    bf16x8 A[KSTEPS];
#pragma unroll
    for (int s = 0; s < KSTEPS; ++s) A[s] = pack[s * 64 + lane];
    bf16x8 A4[2];
    if (MODE == 2) {
        A4[0] = pack4[lane];
        A4[1] = pack4[64 + lane];
    }
    const bool big = ny >= CT_R && nx >= CT_C;   // block-uniform: two-phase staging applies
    u32x4 pre[ST_IT];
    if (big && (int)blockIdx.x < ntiles) {
        const int ty = blockIdx.x / ntx;
        tile_load(pre, in, HW, ny, nx, ty * CT_Y, (blockIdx.x - ty * ntx) * CT_X);
    }
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int ty = tile / ntx, tx = tile - ty * ntx;
        const int x0 = tx * CT_X, y0 = ty * CT_Y;
        __syncthreads();                        // LDS reads of the previous tile are done
        if (big) {
            tile_store(sm, pre);
            __syncthreads();
            const int t1 = tile + gridDim.x;    // next tile's halo, in flight during the compute
            if (t1 < ntiles) {
                const int ty1 = t1 / ntx;
                tile_load(pre, in, HW, ny, nx, ty1 * CT_Y, (t1 - ty1 * ntx) * CT_X);
            }
        } else {
            stage_tile(sm, in, HW, ny, nx, y0, x0);
            __syncthreads();
        }
        conv_tile<MODE>(sm, A, A4, bias, aux, out, HW, ny, nx, x0, y0);
    }
}

#define CONV32_ARGS                                                                                        \
    const float *__restrict__ in, const bf16x8 *__restrict__ pack, const float *__restrict__ bias,          \
        const float *__restrict__ aux, const bf16x8 *__restrict__ pack4, float *__restrict__ out, int ny, int nx
// 43.5 KB of LDS per block.  The next tile's loads are in flight during the compute, so two
// blocks per CU (with registers for the prefetch, the 18 A operands and both accumulators)
// keep the loads going; three would spill.
constexpr int CONV_OCC = 2;
__global__ __launch_bounds__(256, CONV_OCC) void k_conv32_fwd(CONV32_ARGS) {
    conv32_body<0>(in, pack, bias, aux, pack4, out, ny, nx);
}
__global__ __launch_bounds__(256, CONV_OCC) void k_conv32_bwd(CONV32_ARGS) {
    conv32_body<1>(in, pack, bias, aux, pack4, out, ny, nx);
}
__global__ __launch_bounds__(256, CONV_OCC) void k_conv32_taps(CONV32_ARGS) {
    conv32_body<2>(in, pack, bias, aux, pack4, out, ny, nx);
}

// Layers 1 and 2 of an inference pass in one kernel.  A block stages the network input x
// of its tile with a two-cell halo (12 x 36 cells, both channels as one 8-byte pair), forms
// layer 1 on the 10 x 34 halo tile that layer 2 needs directly into LDS, and then runs
// layer 2 as k_conv32_fwd does; a1 never leaves the chip.  Layer 1 on the matrix cores:
// rows = 32 output channels, columns = 32 halo cells, K = 18 (9 taps x 2 channels, padded
// to two steps of 16) with x split into hi + lo bfloat16 parts like the activations.
constexpr int XS_R = CT_R + 2, XS_C = CT_C + 2, XS_N = XS_R * XS_C;
constexpr int XS_IT = (XS_N + 255) / 256;
constexpr int L1_CELLS = CT_R * CT_C, L1_CHUNKS = (L1_CELLS + 31) / 32;
typedef float f32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ void xs_load(f32x2 (&v)[XS_IT], const float* __restrict__ x, long HW, int ny, int nx,
                                        int y0, int x0) {
#pragma unroll
    for (int k = 0; k < XS_IT; ++k) {
        const int e = threadIdx.x + 256 * k;
        if (e < XS_N) {
            const int r = e / XS_C, c = e - r * XS_C;
            const long q = (long)wrapm(y0 - 2 + r, ny) * nx + wrapm(x0 - 2 + c, nx);
            v[k] = f32x2{x[q], x[HW + q]};
        }
    }
}

__device__ __forceinline__ bf16x8 pk8(const float (&b)[8]) {
    return __builtin_bit_cast(bf16x8, make_uint4(pk_bf16(b[0], b[1]), pk_bf16(b[2], b[3]), pk_bf16(b[4], b[5]),
                                                 pk_bf16(b[6], b[7])));
}

// a1 = tanh(conv(x; W1) + b1) on the halo tile, into sm; wave wv takes chunks wv, wv + 4, ...
// of 32 halo cells in row-major order (the last chunk is partial).  bl holds this lane's 16
// bias values, b1[4 (2 q4 + half) + e] at 4 q4 + e, loaded once per kernel.
__device__ __forceinline__ void layer1_to_lds(uint4 (*sm)[NG][CT_C], const f32x2 (*xs)[XS_C],
                                              const bf16x8 (&A1)[2], const float (&bl)[16]) {
    const int lane = threadIdx.x & 63, half = lane >> 5, col = lane & 31, wv = threadIdx.x >> 6;
    for (int k = wv; k < L1_CHUNKS; k += 4) {
        const int q0 = 32 * k + col;
        const bool ok = q0 < L1_CELLS;
        const int q = ok ? q0 : L1_CELLS - 1;
        const int r = q / CT_C, c = q - r * CT_C;
        // B operands: step 0 holds taps 4 half .. 4 half + 3, step 1 tap 8 (half 0), else zero
        float b0[8], b1v[8];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int t = 4 * half + i;
            const f32x2 v = xs[r + t / 3][c + t % 3];
            b0[2 * i] = v.x;
            b0[2 * i + 1] = v.y;
        }
        const f32x2 v8 = xs[r + 2][c + 2];
        b1v[0] = half == 0 ? v8.x : 0.f;
        b1v[1] = half == 0 ? v8.y : 0.f;
#pragma unroll
        for (int e = 2; e < 8; ++e) b1v[e] = 0.f;
        float l0[8], l1[8];
        const bf16x8 h0 = pk8(b0), h1 = pk8(b1v);
        const uint4 uh0 = __builtin_bit_cast(uint4, h0), uh1 = __builtin_bit_cast(uint4, h1);
        const unsigned w0[4] = {uh0.x, uh0.y, uh0.z, uh0.w}, w1[4] = {uh1.x, uh1.y, uh1.z, uh1.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            l0[2 * e] = b0[2 * e] - __uint_as_float(w0[e] << 16);
            l0[2 * e + 1] = b0[2 * e + 1] - __uint_as_float(w0[e] & 0xFFFF0000u);
            l1[2 * e] = b1v[2 * e] - __uint_as_float(w1[e] << 16);
            l1[2 * e + 1] = b1v[2 * e + 1] - __uint_as_float(w1[e] & 0xFFFF0000u);
        }
        f32x16 d = {};
        d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A1[0], h0, d, 0, 0, 0);
        d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A1[0], pk8(l0), d, 0, 0, 0);
        d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A1[1], h1, d, 0, 0, 0);
        d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A1[1], pk8(l1), d, 0, 0, 0);
        // lane holds halo cell q and channels 8 (i / 4) + 4 half + i % 4
#pragma unroll
        for (int q4 = 0; q4 < 4; ++q4) {
            const int cg = 2 * q4 + half;
            float v[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) v[e] = tanh_fast(d[4 * q4 + e] + bl[4 * q4 + e]);
            if (ok) sm[r][cg][c] = split4(v[0], v[1], v[2], v[3]);
        }
    }
}

// x planar FP32 [2][HW] -> a2 (grouped, split); pack: layer 2 forward, pack1: layer 1
__global__ __launch_bounds__(256, CONV_OCC) void k_conv12_fwd(const float* __restrict__ x,
                                                             const bf16x8* __restrict__ pack1,
                                                             const float* __restrict__ b1,
                                                             const bf16x8* __restrict__ pack,
                                                             const float* __restrict__ b2, float* __restrict__ out,
                                                             int ny, int nx) {
    __shared__ uint4 sm[CT_R][NG][CT_C];
    __shared__ f32x2 xs[XS_R][XS_C];
    const int lane = threadIdx.x & 63;
    const long HW = (long)ny * nx;
    const int ntx = (nx + CT_X - 1) / CT_X, nty = (ny + CT_Y - 1) / CT_Y;
    const int ntiles = ntx * nty;
    bf16x8 A[KSTEPS];
#pragma unroll
    for (int s = 0; s < KSTEPS; ++s) A[s] = pack[s * 64 + lane];
    const bf16x8 A1[2] = {pack1[lane], pack1[64 + lane]};
    const bf16x8 A4[2] = {};
    float bl[16];
#pragma unroll
    for (int q4 = 0; q4 < 4; ++q4)
#pragma unroll
        for (int e = 0; e < 4; ++e) bl[4 * q4 + e] = b1[4 * (2 * q4 + (lane >> 5)) + e];
    f32x2 pre[XS_IT];
    if ((int)blockIdx.x < ntiles) {
        const int ty = blockIdx.x / ntx;
        xs_load(pre, x, HW, ny, nx, ty * CT_Y, (blockIdx.x - ty * ntx) * CT_X);
    }
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int ty = tile / ntx, tx = tile - ty * ntx;
        const int x0 = tx * CT_X, y0 = ty * CT_Y;
        __syncthreads();                        // LDS reads of the previous tile are done
#pragma unroll
        for (int k = 0; k < XS_IT; ++k) {
            const int e = threadIdx.x + 256 * k;
            if (e < XS_N) (&xs[0][0])[e] = pre[k];
        }
        __syncthreads();
        const int t1 = tile + gridDim.x;
        if (t1 < ntiles) {
            const int ty1 = t1 / ntx;
            xs_load(pre, x, HW, ny, nx, ty1 * CT_Y, (t1 - ty1 * ntx) * CT_X);
        }
        layer1_to_lds(sm, xs, A1, bl);
        __syncthreads();
        conv_tile<0>(sm, A, A4, b2, nullptr, out, HW, ny, nx, x0, y0);
    }
}

// layer 4: y = conv(a3; W4) + b4, one cell per thread of a block tile staged in LDS
__global__ __launch_bounds__(256) void k_out_fwd(const float* __restrict__ a3, const float* __restrict__ q,
                                                 float* __restrict__ yout, int ny, int nx) {
    __shared__ uint4 sm[CT_R][NG][CT_C];
    const long HW = (long)ny * nx;
    const int ntx = (nx + CT_X - 1) / CT_X;
    const int ty = blockIdx.x / ntx, tx = blockIdx.x - ty * ntx;
    const int x0 = tx * CT_X, y0 = ty * CT_Y;
    if (ny >= CT_R && nx >= CT_C) {
        u32x4 v[ST_IT];
        tile_load(v, a3, HW, ny, nx, y0, x0);
        tile_store(sm, v);
    } else {
        stage_tile(sm, a3, HW, ny, nx, y0, x0);
    }
    __syncthreads();
    const int ly = threadIdx.x / CT_X, lx = threadIdx.x % CT_X;
    const int y = y0 + ly, x = x0 + lx;
    if (y >= ny || x >= nx) return;
    float acc = q[OFF_B4];
#pragma unroll
    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
            const int t = dy * 3 + dx;
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                const float4 v = join4(sm[ly + dy][g][lx + dx]);
                acc += q[OFF_W4 + (4 * g) * 9 + t] * v.x + q[OFF_W4 + (4 * g + 1) * 9 + t] * v.y +
                       q[OFF_W4 + (4 * g + 2) * 9 + t] * v.z + q[OFF_W4 + (4 * g + 3) * 9 + t] * v.w;
            }
        }
    yout[(long)y * nx + x] = acc;
}

// layer 4 of an inference pass from the per-tap sums: y(p) = b4 + sum_t s_t(p + off(t)),
// off(t) = (t / 3 - 1, t % 3 - 1).  Writes y, or X = phi + s_o y when X is given, and then
// with diff_part also this block's share of sum_p (phi - X)(p) (grid-stride over a fixed grid).
__global__ __launch_bounds__(256) void k_out_sum(const float* __restrict__ s, const float* __restrict__ q, int ny,
                                                 int nx, float* __restrict__ yout, const double* __restrict__ phi,
                                                 double s_o, double* __restrict__ X, double* __restrict__ diff_part) {
    __shared__ double red[4];
    const long HW = (long)ny * nx;
    double dsum = 0.0;
    for (long p = blockIdx.x * (long)blockDim.x + threadIdx.x; p < HW; p += (long)gridDim.x * blockDim.x) {
        const int y = (int)(p / nx), xx = (int)(p - (long)y * nx);
        float acc = q[OFF_B4];
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
            const long row = (long)wrap1(y + dy - 1, ny) * nx;
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) acc += s[(dy * 3 + dx) * HW + row + wrap1(xx + dx - 1, nx)];
        }
        if (X) {
            const double f = phi[p], xv = f + s_o * (double)acc;
            X[p] = xv;
            dsum += f - xv;
        } else {
            yout[p] = acc;
        }
    }
    if (diff_part) {
        const double t = block_sum_det(dsum, red);
        if (threadIdx.x == 0) diff_part[blockIdx.x] = t;
    }
}

// dy = scale * 2 (y - t) / HW and per-block partials of sum (y - t)^2
__global__ __launch_bounds__(256) void k_loss(const float* __restrict__ y, const float* __restrict__ t,
                                              float* __restrict__ dy, long HW, float gmul, double* __restrict__ part) {
    __shared__ double red[4];
    double acc = 0.0;
    for (long p = blockIdx.x * (long)blockDim.x + threadIdx.x; p < HW; p += (long)gridDim.x * blockDim.x) {
        const float d = y[p] - t[p];
        dy[p] = gmul * d;
        acc += (double)d * (double)d;
    }
    const double s = block_sum_det(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// backward through layer 4 and the tanh of layer 3:
// g3[c](p) = (1 - a3[c](p)^2) sum_tap W4[c][tap] dy(p - off(tap))
__global__ __launch_bounds__(256) void k_out_bwd(const float* __restrict__ dy, const float* __restrict__ q,
                                                 const float* __restrict__ a3, float* __restrict__ g3, int ny,
                                                 int nx) {
    const long HW = (long)ny * nx;
    const long p = blockIdx.x * (long)blockDim.x + threadIdx.x;   // one cell per thread
    if (p >= HW) return;
    const int y = (int)(p / nx), xx = (int)(p - (long)y * nx);
    float d[9];   // d[t'] = dy(p + off(t')), paired with the mirrored tap 8 - t'
#pragma unroll
    for (int dyo = 0; dyo < 3; ++dyo)
#pragma unroll
        for (int dxo = 0; dxo < 3; ++dxo)
            d[dyo * 3 + dxo] = dy[(long)wrap1(y + dyo - 1, ny) * nx + wrap1(xx + dxo - 1, nx)];
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        const float4 a = join4(*grp(a3, g, HW, p));
        float r[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int c = 4 * g + j;
            float s = 0.f;
#pragma unroll
            for (int t = 0; t < 9; ++t) s += q[OFF_W4 + c * 9 + (8 - t)] * d[t];
            r[j] = s;
        }
        r[0] *= 1.f - a.x * a.x;
        r[1] *= 1.f - a.y * a.y;
        r[2] *= 1.f - a.z * a.z;
        r[3] *= 1.f - a.w * a.w;
        *grp(g3, g, HW, p) = split4(r[0], r[1], r[2], r[3]);
    }
}

// Weight and bias gradient of one layer, per-block partials:
//   dW[o][c][tap] = sum_p g[o](p) a[c](p + off(tap)),  db[o] = sum_p g[o](p)
// G output channels (32: grouped layout, 1: plain), A input channels (32: grouped, 2: planar).
// A block walks tiles of 64 cells of one row; thread t owns channel o and CB input
// channels for all 9 taps over a contiguous share of the tile's cells (NPH shares).
template <int G, int A>
__global__ __launch_bounds__(256) void k_wgrad(const float* __restrict__ g, const float* __restrict__ a, int ny,
                                               int nx, float* __restrict__ part) {
    constexpr int CB = A == 32 ? 4 : 2;
    constexpr int NPAIR = G * (A / CB);
    constexpr int NPH = 256 / NPAIR;
    constexpr int XS = 64 / NPH;
    constexpr int NO = G * A * 9;
    static_assert(NPAIR * NPH == 256 && XS * NPH == 64, "thread mapping");
    __shared__ float gs[G][65];
    __shared__ float as_[A][3][67];
    __shared__ float red[NPH > 1 ? NPH * NPAIR * (CB * 9 + 1) : 1];
    const int t = threadIdx.x;
    const int pair = t % NPAIR, ph = t / NPAIR;
    const int o = pair / (A / CB), cb = (pair % (A / CB)) * CB;
    const long HW = (long)ny * nx;
    const int ntx = (nx + 63) / 64;
    const long ntiles = (long)ny * ntx;
    float acc[CB][9];
#pragma unroll
    for (int i = 0; i < CB; ++i)
#pragma unroll
        for (int k = 0; k < 9; ++k) acc[i][k] = 0.f;
    float bacc = 0.f;
    for (long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int y = (int)(tile / ntx), x0 = (int)(tile - (long)y * ntx) * 64;
        __syncthreads();
        if (G == 32) {   // one 16-byte group (4 channels of a cell) per thread
            for (int e = t; e < (G / 4) * 64; e += 256) {
                const int xl = e % 64, gg = e / 64, x = x0 + xl;
                float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
                if (x < nx) v = join4(*grp(g, gg, HW, (long)y * nx + x));
                gs[4 * gg][xl] = v.x;
                gs[4 * gg + 1][xl] = v.y;
                gs[4 * gg + 2][xl] = v.z;
                gs[4 * gg + 3][xl] = v.w;
            }
        } else {
            for (int e = t; e < 64; e += 256) {
                const int x = x0 + e;
                gs[0][e] = x < nx ? g[(long)y * nx + x] : 0.f;
            }
        }
        if (A == 32) {
            for (int e = t; e < (A / 4) * 3 * 66; e += 256) {
                const int xl = e % 66, r = (e / 66) % 3, gg = e / 198;
                const long pi = (long)wrapm(y + r - 1, ny) * nx + wrapm(x0 + xl - 1, nx);
                const float4 v = join4(*grp(a, gg, HW, pi));
                as_[4 * gg][r][xl] = v.x;
                as_[4 * gg + 1][r][xl] = v.y;
                as_[4 * gg + 2][r][xl] = v.z;
                as_[4 * gg + 3][r][xl] = v.w;
            }
        } else {
            for (int e = t; e < A * 3 * 66; e += 256) {
                const int xl = e % 66, r = (e / 66) % 3, c = e / 198;
                as_[c][r][xl] = a[(long)c * HW + (long)wrapm(y + r - 1, ny) * nx + wrapm(x0 + xl - 1, nx)];
            }
        }
        __syncthreads();
        for (int xl = ph * XS; xl < (ph + 1) * XS; ++xl) {
            const float gv = gs[o][xl];
            bacc += gv;
#pragma unroll
            for (int i = 0; i < CB; ++i)
#pragma unroll
                for (int r = 0; r < 3; ++r)
#pragma unroll
                    for (int d = 0; d < 3; ++d) acc[i][r * 3 + d] += gv * as_[cb + i][r][xl + d];
        }
    }
    float* dst = part + (long)blockIdx.x * (NO + G);
    if (NPH == 1) {
#pragma unroll
        for (int i = 0; i < CB; ++i)
#pragma unroll
            for (int k = 0; k < 9; ++k) dst[(o * A + cb + i) * 9 + k] = acc[i][k];
        if (cb == 0) dst[NO + o] = bacc;
        return;
    }
    __syncthreads();
    float* mine = red + ((long)ph * NPAIR + pair) * (CB * 9 + 1);
#pragma unroll
    for (int i = 0; i < CB; ++i)
#pragma unroll
        for (int k = 0; k < 9; ++k) mine[i * 9 + k] = acc[i][k];
    mine[CB * 9] = bacc;
    __syncthreads();
    for (int e = t; e < NPAIR * (CB * 9 + 1); e += 256) {
        const int pr = e / (CB * 9 + 1), k = e % (CB * 9 + 1);
        float s = 0.f;
        for (int h = 0; h < NPH; ++h) s += red[((long)h * NPAIR + pr) * (CB * 9 + 1) + k];
        const int oo = pr / (A / CB), cc = (pr % (A / CB)) * CB;
        if (k < CB * 9)
            dst[(oo * A + cc + k / 9) * 9 + k % 9] = s;
        else if (cc == 0)
            dst[NO + oo] = s;
    }
}

// grad[off + k] (+)= sum_b part[b][k], k < n, blocks in order
__global__ void k_wreduce(const float* __restrict__ part, int nblocks, int n, float* __restrict__ grad, int accumulate) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    float s = 0.f;
    for (int b = 0; b < nblocks; ++b) s += part[(long)b * n + k];
    grad[k] = accumulate ? grad[k] + s : s;
}

// Gradient of the step-size weights u1: z_1 depends on b1 + c u1, so d/du1 = c d/db1.  The
// layer-1 bias partials (entries koff..koff+WID of each block's row of n) are summed in the
// order k_wreduce sums them.
__global__ void k_ureduce(const float* __restrict__ part, int nblocks, int n, int koff, float c,
                          float* __restrict__ grad, int accumulate) {
    const int k = threadIdx.x;
    if (k >= WID) return;
    float s = 0.f;
    for (int b = 0; b < nblocks; ++b) s += part[(long)b * n + koff + k];
    grad[k] = accumulate ? grad[k] + c * s : c * s;
}

// b1c = b1 + c u1: layer 1's bias with the constant step-size plane folded in (its 3x3 taps
// sum to u1, so over a constant plane c the convolution adds c u1)
__global__ void k_cond_bias(const float* __restrict__ q, float c, float* __restrict__ b1c) {
    const int k = threadIdx.x;
    if (k < WID) b1c[k] = q[OFF_B1 + k] + c * q[OFF_U1 + k];
}

__global__ void k_adam(float* __restrict__ theta, const float* __restrict__ grad, float* __restrict__ m,
                       float* __restrict__ v, int n, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float g = grad[i];
    const float mi = b1 * m[i] + (1.f - b1) * g;
    const float vi = b2 * v[i] + (1.f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    theta[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

// solver side: network input planes and the guess
// x[0] = (phi - mean)/s_a, x[1] = ratio (phi - prev) * inv_x1; every block sums the mean's
// partials in the same order
__global__ __launch_bounds__(256) void k_net_input(const double* __restrict__ phi, const double* __restrict__ prev,
                                                   long n, double ratio, double inv_sa, double inv_x1,
                                                   const double* __restrict__ sum_part, int np,
                                                   float* __restrict__ x) {
    __shared__ double red[4];
    const double mean = sum_partials_bcast(sum_part, np, red) / (double)n;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const double f = phi[i];
        x[i] = (float)((f - mean) * inv_sa);
        x[n + i] = (float)(ratio * (f - prev[i]) * inv_x1);
    }
}

inline unsigned cell_grid(long n) { return (unsigned)((n + 255) / 256); }   // one cell per thread

inline unsigned grid_for(long n, int per = 256, unsigned cap = 4096) {
    const long b = (n + per - 1) / per;
    return (unsigned)(b < 1 ? 1 : (b > cap ? cap : b));
}

}  // namespace
}  // namespace pfc

using namespace pfc;

struct pfc_net {
    hipStream_t stream = nullptr;
    float* d_theta = nullptr;   // master parameters
    float* d_q = nullptr;       // rounded weights + biases
    float* d_b1c = nullptr;     // layer-1 bias with the step-size term, b1 + c u1
    unsigned short* d_pack = nullptr;
    float* d_grad = nullptr;
    float* d_m = nullptr;
    float* d_v = nullptr;
    float* d_wpart = nullptr;   // weight-gradient partials
    double* d_lpart = nullptr;  // loss partials
    double* h_lpart = nullptr;
    long cap = 0;               // cells the activation buffers hold
    float *a1 = nullptr, *a2 = nullptr, *a3 = nullptr, *b1 = nullptr, *b2 = nullptr, *y = nullptr, *dy = nullptr;
    long step = 0;
    int conv_res = 0;           // conv32 blocks resident on the device at once
    bool prepared = false;
    std::string err;
};

namespace {

#define NETCHK(expr)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess) {                                                          \
            net->err = std::string(#expr) + ": " + hipGetErrorString(e_);                \
            return PFC_EHIP;                                                             \
        }                                                                                \
    } while (0)

void free_acts(pfc_net* net) {
    float* bufs[] = {net->a1, net->a2, net->a3, net->b1, net->b2, net->y, net->dy};
    for (float* p : bufs)
        if (p) (void)hipFree(p);
    net->a1 = net->a2 = net->a3 = net->b1 = net->b2 = net->y = net->dy = nullptr;
    net->cap = 0;
}

pfc_status ensure(pfc_net* net, long HW) {
    if (HW <= net->cap) return PFC_OK;
    if (hipDeviceSynchronize() != hipSuccess) {   // earlier launches may still use the buffers
        net->err = "stream synchronisation failed";
        return PFC_EHIP;
    }
    free_acts(net);
    const size_t big = sizeof(float) * (size_t)WID * HW, small = sizeof(float) * (size_t)HW;
    float** bigs[] = {&net->a1, &net->a2, &net->a3, &net->b1, &net->b2};
    for (float** p : bigs)
        if (hipMalloc((void**)p, big) != hipSuccess) {
            free_acts(net);
            net->err = "out of device memory for activations";
            return PFC_ENOMEM;
        }
    if (hipMalloc((void**)&net->y, small) != hipSuccess || hipMalloc((void**)&net->dy, small) != hipSuccess) {
        free_acts(net);
        net->err = "out of device memory for activations";
        return PFC_ENOMEM;
    }
    net->cap = HW;
    return PFC_OK;
}

pfc_status prepare(pfc_net* net, hipStream_t s) {
    if (net->prepared) return PFC_OK;
    hipLaunchKernelGGL(k_prepare, dim3((PACK_ALL * 8 + 255) / 256), dim3(256), 0, s, net->d_theta, net->d_q,
                       net->d_pack);
    NETCHK(hipGetLastError());
    net->prepared = true;
    return PFC_OK;
}

const bf16x8* pack_of(const pfc_net* net, int set) {
    return reinterpret_cast<const bf16x8*>(net->d_pack) + (long)set * PACK;
}
const bf16x8* pack1_of(const pfc_net* net) { return reinterpret_cast<const bf16x8*>(net->d_pack) + 4 * PACK + PACK4; }

unsigned tile_count(int ny, int nx) { return (unsigned)(((nx + CT_X - 1) / CT_X) * ((ny + CT_Y - 1) / CT_Y)); }

unsigned conv_grid(const pfc_net* net, int ny, int nx) {   // persistent: one block per resident slot
    const unsigned t = tile_count(ny, nx);
    return t < (unsigned)net->conv_res ? t : (unsigned)net->conv_res;
}

// forward pass on stream s: activations a1..a3 (kept for a backward pass), output in y_out
// the four layers on stream s with activations in a1..a3 (parameters already prepared)
pfc_status forward_into(pfc_net* net, hipStream_t s, const float* x, int ny, int nx, float* y_out, float* a1,
                        float* a2, float* a3) {
    const long HW = (long)ny * nx;
    hipLaunchKernelGGL(k_in_fwd, dim3(cell_grid(HW)), dim3(256), 0, s, x, net->d_q, net->d_b1c, a1, ny, nx);
    hipLaunchKernelGGL(k_conv32_fwd, dim3(conv_grid(net, ny, nx)), dim3(256), 0, s, a1, pack_of(net, 0),
                       net->d_q + OFF_B2, nullptr, nullptr, a2, ny, nx);
    hipLaunchKernelGGL(k_conv32_fwd, dim3(conv_grid(net, ny, nx)), dim3(256), 0, s, a2, pack_of(net, 2),
                       net->d_q + OFF_B3, nullptr, nullptr, a3, ny, nx);
    hipLaunchKernelGGL(k_out_fwd, dim3(tile_count(ny, nx)), dim3(256), 0, s, a3, net->d_q, y_out, ny, nx);
    NETCHK(hipGetLastError());
    return PFC_OK;
}

// inference pass on stream s, three kernels: layers 1-2 (a1 stays in LDS) into a2 (32 HW
// floats), layer 3 with the output layer's per-tap sums into taps (9 HW floats; a3 is never
// stored), and the output sum.  b1c: layer 1's conditioned bias.  Output y_out, or
// X = phi + s_o y when X is given.
pfc_status infer_into(pfc_net* net, hipStream_t s, const float* x, const float* b1c, int ny, int nx, float* a2,
                      float* taps, float* y_out, const double* phi, double s_o, double* X,
                      double* diff_part = nullptr) {
    const long HW = (long)ny * nx;
    hipLaunchKernelGGL(k_conv12_fwd, dim3(conv_grid(net, ny, nx)), dim3(256), 0, s, x, pack1_of(net), b1c,
                       pack_of(net, 0), net->d_q + OFF_B2, a2, ny, nx);
    hipLaunchKernelGGL(k_conv32_taps, dim3(conv_grid(net, ny, nx)), dim3(256), 0, s, a2, pack_of(net, 2),
                       net->d_q + OFF_B3, nullptr, pack_of(net, 4), taps, ny, nx);
    const dim3 sum_grid = diff_part ? dim3(kRedBlocks) : dim3(cell_grid(HW));
    hipLaunchKernelGGL(k_out_sum, sum_grid, dim3(256), 0, s, taps, net->d_q, ny, nx, y_out, phi, s_o, X,
                       diff_part);
    NETCHK(hipGetLastError());
    return PFC_OK;
}

// forward pass on stream s with the network's own activation buffers (kept for a backward pass)
pfc_status forward_impl(pfc_net* net, hipStream_t s, const float* x, double cond, int ny, int nx, float* y_out) {
    pfc_status st = ensure(net, (long)ny * nx);
    if (st != PFC_OK) return st;
    st = prepare(net, s);
    if (st != PFC_OK) return st;
    hipLaunchKernelGGL(k_cond_bias, dim3(1), dim3(64), 0, s, net->d_q, (float)cond, net->d_b1c);
    return forward_into(net, s, x, ny, nx, y_out, net->a1, net->a2, net->a3);
}

template <int G, int A>
pfc_status wgrad(pfc_net* net, const float* g, const float* a, int ny, int nx, int off, int accumulate) {
    constexpr int n = G * A * 9 + G;
    hipLaunchKernelGGL((k_wgrad<G, A>), dim3(WG_BLOCKS), dim3(256), 0, net->stream, g, a, ny, nx, net->d_wpart);
    hipLaunchKernelGGL(k_wreduce, dim3((n + 255) / 256), dim3(256), 0, net->stream, net->d_wpart, WG_BLOCKS, n,
                       net->d_grad + off, accumulate);
    NETCHK(hipGetLastError());
    return PFC_OK;
}

}  // namespace

namespace pfc {
// for the solver: learned initial guess X = phi + out_scale net(x(phi, prev); c), before the
// mass shift; sum_part holds np partial sums of phi
pfc_status net_guess(pfc_net* net, hipStream_t s, const double* phi, const double* prev, int ny, int nx,
                     double ratio, double cond, double inv_sa, double inv_x1, double out_scale,
                     const double* sum_part, int np, const NetWork& w, double* X, double* diff_part) {
    const long n = (long)ny * nx;
    if (!net->prepared) {
        net->err = "network parameters changed since pfc_attach_net: attach it again";
        return PFC_EINVAL;
    }
    hipLaunchKernelGGL(k_cond_bias, dim3(1), dim3(64), 0, s, net->d_q, (float)cond, w.b1c);
    hipLaunchKernelGGL(k_net_input, dim3(grid_for(n)), dim3(256), 0, s, phi, prev, n, ratio, inv_sa, inv_x1,
                       sum_part, np, w.x);
    static_assert(kNetWorkFloats == WID + 9, "inference workspace: a2, then the tap sums");
    return infer_into(net, s, w.x, w.b1c, ny, nx, w.a, w.a + (size_t)WID * n, nullptr, phi, out_scale, X,
                      diff_part);
}

pfc_status net_prepare(pfc_net* net) {
    pfc_status st = prepare(net, net->stream);
    if (st != PFC_OK) return st;
    NETCHK(hipStreamSynchronize(net->stream));
    return PFC_OK;
}

const char* net_error(const pfc_net* net) { return net->err.c_str(); }
}  // namespace pfc

extern "C" {

pfc_status pfc_net_create(void* stream, pfc_net** out) {
    if (!out) return PFC_EINVAL;
    *out = nullptr;
    pfc_net* net = new pfc_net();
    net->stream = (hipStream_t)stream;
    bool ok = hipMalloc((void**)&net->d_theta, sizeof(float) * NPARAM) == hipSuccess &&
              hipMalloc((void**)&net->d_q, sizeof(float) * NPARAM) == hipSuccess &&
              hipMalloc((void**)&net->d_b1c, sizeof(float) * WID) == hipSuccess &&
              hipMalloc((void**)&net->d_pack, sizeof(unsigned short) * PACK_ALL * 8) == hipSuccess &&
              hipMalloc((void**)&net->d_grad, sizeof(float) * NPARAM) == hipSuccess &&
              hipMalloc((void**)&net->d_m, sizeof(float) * NPARAM) == hipSuccess &&
              hipMalloc((void**)&net->d_v, sizeof(float) * NPARAM) == hipSuccess &&
              hipMalloc((void**)&net->d_wpart, sizeof(float) * (size_t)WG_BLOCKS * WG_MAXOUT) == hipSuccess &&
              hipMalloc((void**)&net->d_lpart, sizeof(double) * kRedBlocks) == hipSuccess &&
              hipHostMalloc((void**)&net->h_lpart, sizeof(double) * kRedBlocks) == hipSuccess;
    if (ok) {
        ok = hipMemset(net->d_theta, 0, sizeof(float) * NPARAM) == hipSuccess &&
             hipMemset(net->d_grad, 0, sizeof(float) * NPARAM) == hipSuccess &&
             hipMemset(net->d_m, 0, sizeof(float) * NPARAM) == hipSuccess &&
             hipMemset(net->d_v, 0, sizeof(float) * NPARAM) == hipSuccess && hipDeviceSynchronize() == hipSuccess;
    }
    if (ok) {   // the persistent conv kernels share launch bounds; the fused one has more LDS
        int dev = 0, cus = 0, occ = 0, occ12 = 0;
        ok = hipGetDevice(&dev) == hipSuccess &&
             hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
             hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_conv32_fwd, 256, 0) == hipSuccess &&
             hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ12, k_conv12_fwd, 256, 0) == hipSuccess;
        occ = occ12 < occ ? occ12 : occ;
        net->conv_res = (occ < 1 ? 1 : occ) * (cus < 1 ? 1 : cus);
    }
    if (!ok) {
        pfc_net_destroy(net);
        return PFC_ENOMEM;
    }
    *out = net;
    return PFC_OK;
}

void pfc_net_destroy(pfc_net* net) {
    if (!net) return;
    free_acts(net);
    void* ptrs[] = {net->d_theta, net->d_q, net->d_b1c, net->d_pack, net->d_grad, net->d_m, net->d_v,
                    net->d_wpart, net->d_lpart};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (net->h_lpart) (void)hipHostFree(net->h_lpart);
    delete net;
}

const char* pfc_net_last_error(const pfc_net* net) { return net ? net->err.c_str() : "null network"; }

pfc_status pfc_net_set_params(pfc_net* net, const float* host_params) {
    if (!net || !host_params) return PFC_EINVAL;
    NETCHK(hipMemcpyAsync(net->d_theta, host_params, sizeof(float) * NPARAM, hipMemcpyHostToDevice, net->stream));
    NETCHK(hipMemsetAsync(net->d_m, 0, sizeof(float) * NPARAM, net->stream));
    NETCHK(hipMemsetAsync(net->d_v, 0, sizeof(float) * NPARAM, net->stream));
    NETCHK(hipStreamSynchronize(net->stream));
    net->step = 0;
    net->prepared = false;
    return PFC_OK;
}

pfc_status pfc_net_get_params(pfc_net* net, float* host_params) {
    if (!net || !host_params) return PFC_EINVAL;
    NETCHK(hipMemcpyAsync(host_params, net->d_theta, sizeof(float) * NPARAM, hipMemcpyDeviceToHost, net->stream));
    NETCHK(hipStreamSynchronize(net->stream));
    return PFC_OK;
}

pfc_status pfc_net_forward(pfc_net* net, const float* x, double cond, int ny, int nx, float* y) {
    if (!net) return PFC_EINVAL;
    if (!x || !y || ny < 3 || nx < 3 || !std::isfinite(cond)) {
        net->err = "bad argument";
        return PFC_EINVAL;
    }
    pfc_status st = ensure(net, (long)ny * nx);
    if (st != PFC_OK) return st;
    st = prepare(net, net->stream);
    if (st != PFC_OK) return st;
    hipLaunchKernelGGL(k_cond_bias, dim3(1), dim3(64), 0, net->stream, net->d_q, (float)cond, net->d_b1c);
    return infer_into(net, net->stream, x, net->d_b1c, ny, nx, net->a2, net->a3, y, nullptr, 0.0, nullptr);
}

pfc_status pfc_net_gradient(pfc_net* net, const float* x, double cond, const float* t, int ny, int nx, double scale,
                            int accumulate, double* loss) {
    if (!net) return PFC_EINVAL;
    if (!x || !t || ny < 3 || nx < 3 || !std::isfinite(cond)) {
        net->err = "bad argument";
        return PFC_EINVAL;
    }
    const long HW = (long)ny * nx;
    hipStream_t s = net->stream;
    pfc_status st = ensure(net, HW);
    if (st != PFC_OK) return st;
    st = forward_impl(net, s, x, cond, ny, nx, net->y);
    if (st != PFC_OK) return st;
    hipLaunchKernelGGL(k_loss, dim3(kRedBlocks), dim3(256), 0, s, net->y, t, net->dy, HW,
                       (float)(2.0 * scale / (double)HW), net->d_lpart);
    NETCHK(hipGetLastError());
    // layer 4
    if ((st = wgrad<1, WID>(net, net->dy, net->a3, ny, nx, OFF_W4, accumulate)) != PFC_OK) return st;
    hipLaunchKernelGGL(k_out_bwd, dim3(cell_grid(HW)), dim3(256), 0, s, net->dy, net->d_q, net->a3, net->b1, ny, nx);
    // layer 3: g3 in b1
    if ((st = wgrad<WID, WID>(net, net->b1, net->a2, ny, nx, OFF_W3, accumulate)) != PFC_OK) return st;
    hipLaunchKernelGGL(k_conv32_bwd, dim3(conv_grid(net, ny, nx)), dim3(256), 0, s, net->b1, pack_of(net, 3), nullptr, net->a2,
                       nullptr, net->b2, ny, nx);
    // layer 2: g2 in b2
    if ((st = wgrad<WID, WID>(net, net->b2, net->a1, ny, nx, OFF_W2, accumulate)) != PFC_OK) return st;
    hipLaunchKernelGGL(k_conv32_bwd, dim3(conv_grid(net, ny, nx)), dim3(256), 0, s, net->b2, pack_of(net, 1), nullptr, net->a1,
                       nullptr, net->b1, ny, nx);
    // layer 1: g1 in b1; then u1 from layer 1's bias partials, still in d_wpart
    if ((st = wgrad<WID, CIN>(net, net->b1, x, ny, nx, OFF_W1, accumulate)) != PFC_OK) return st;
    hipLaunchKernelGGL(k_ureduce, dim3(1), dim3(64), 0, s, net->d_wpart, WG_BLOCKS, WID * CIN * 9 + WID,
                       WID * CIN * 9, (float)cond, net->d_grad + OFF_U1, accumulate);
    NETCHK(hipGetLastError());
    if (loss) {
        NETCHK(hipMemcpyAsync(net->h_lpart, net->d_lpart, sizeof(double) * kRedBlocks, hipMemcpyDeviceToHost, s));
        NETCHK(hipStreamSynchronize(s));
        double sum = 0.0;
        for (int i = 0; i < kRedBlocks; ++i) sum += net->h_lpart[i];
        *loss = sum / (double)HW;
    }
    return PFC_OK;
}

pfc_status pfc_net_get_gradient(pfc_net* net, float* host_grad) {
    if (!net || !host_grad) return PFC_EINVAL;
    NETCHK(hipMemcpyAsync(host_grad, net->d_grad, sizeof(float) * NPARAM, hipMemcpyDeviceToHost, net->stream));
    NETCHK(hipStreamSynchronize(net->stream));
    return PFC_OK;
}

pfc_status pfc_net_adam(pfc_net* net, double lr, double beta1, double beta2, double eps) {
    if (!net) return PFC_EINVAL;
    if (!(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0)) {
        net->err = "bad Adam hyper-parameters";
        return PFC_EINVAL;
    }
    net->step++;
    const double c1 = 1.0 / (1.0 - std::pow(beta1, (double)net->step));
    const double c2 = 1.0 / (1.0 - std::pow(beta2, (double)net->step));
    hipLaunchKernelGGL(k_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, net->stream, net->d_theta, net->d_grad,
                       net->d_m, net->d_v, NPARAM, (float)lr, (float)beta1, (float)beta2, (float)eps, (float)c1,
                       (float)c2);
    NETCHK(hipGetLastError());
    net->prepared = false;
    return PFC_OK;
}

}  // extern "C"
