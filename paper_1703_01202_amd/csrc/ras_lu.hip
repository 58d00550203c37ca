// Restricted additive Schwarz with exact subdomain solves (Sec. 4: the subdomain problems
// may be solved directly by a sparse LU factorisation), 2-D.
//
// In the natural order of an ex x ey box the subdomain matrix A_k (Eq. (25)/(26)) is
// block banded: blocks are box rows of W = ex cells, and block (I, J) is nonzero for
// |I - J| <= 3 (the stencil reaches three rows).  Block Gaussian elimination without
// pivoting keeps that band and gives the exact factorisation A = Lh D Uh with
//     S_KK   = A_KK after the updates of steps < K      (D = diag(S_KK)),
//     Lh(I,K) = A(I,K) S_KK^-1,  Uh(K,J) = S_KK^-1 A(K,J),  A(I,J) -= A(I,K) S_KK^-1 A(K,J),
// for |I - K|, |J - K| <= 3.  S_KK^-1 is formed by Gauss-Jordan elimination in LDS.
// The solve needs no triangular solve inside a block:
//     forward:  z_I = r_I - sum_{K=I-3}^{I-1} Lh(I,K) z_K
//     backward: x_I = S_II^-1 z_I - sum_{J=I+1}^{I+3} Uh(I,J) x_J
// Each block row stores [Lh(I,I-3..I-1) | S_II^-1 | -Uh(I,I+1..I+3)] (7 W^2 values), each
// W x W block column-major, so each half sweep is one dense product per block row whose
// input is a contiguous slice of the box vector.
// Elimination without pivoting is exact here because the symmetric part of the Jacobian
// is positive definite for the step sizes used (its Fourier symbol at a uniform state is
// 1/dt + kappa((1-kappa)^2 - gamma + 2c)/2 > 0); a zero pivot is reported.
#include "device_reduce.h"
#include "pfc_internal.h"

namespace pfc {
namespace {

constexpr int kSmallW = 36;        // boxes up to this width factor entirely in LDS

struct LuBox {
    int W, H;                  // block size (box x extent), block rows (box y extent)
    int subx, ownx, owny, ov;
    int nx, ny;
    int idx7[49];              // stencil index of offset (dx, dy), (dy+3)*7 + dx+3, or -1
};

__device__ __forceinline__ int wrapg(int i, int n) {
    i %= n;
    return i < 0 ? i + n : i;
}

// window slot of block (I, J) in the 16-block workspace
__device__ __forceinline__ double* slot(double* win, int I, int J, int W) {
    return win + (long)(((I & 3) * 4) + (J & 3)) * W * W;
}

// Stencil coefficients of the Jacobian by offset, (dy+3)*7 + dx+3, staged in LDS once per
// kernel (kconst and d1; zero outside the stencil).
struct LdsStencil {
    double k[49];
    double d1[49];
};

__device__ void stage_stencil(LdsStencil* t, const LuBox& b, const StencilTable& st) {
    for (int o = threadIdx.x; o < 49; o += blockDim.x) {
        const int s = b.idx7[o];
        t->k[o] = s >= 0 ? st.kconst[s] : 0.0;
        t->d1[o] = s >= 0 ? st.d1[s] : 0.0;
    }
}

// Block (I, J) of A_k into dst (row-major).  crow holds c along box row J (W values).  With a
// variable mobility (uu: u = (Phi + phi)/2, else null) the spatial part of row (I, p) is scaled
// by its node mobility 1 - u^2, as subdomain_entry says.  Entries first, first + stride, ...
// (by default every thread of the block).
__device__ void assemble_block(double* dst, int I, int J, const LuBox& b, const LdsStencil* t,
                               const double* crow, const double* __restrict__ uu, int ox, int oy, double inv_dt,
                               int first = -1, int stride = 0) {
    const int W = b.W, dy = J - I;
    const long grow = (long)wrapg(oy + I, b.ny) * b.nx;
    if (first < 0) {
        first = threadIdx.x;
        stride = blockDim.x;
    }
    for (int e = first; e < W * W; e += stride) {
        const int p = e / W, q = e - p * W;
        const int dx = q - p;
        double v = 0.0;
        if (abs(dx) + abs(dy) <= 3) {
            const int o = (dy + 3) * 7 + dx + 3;
            v = t->k[o] - t->d1[o] * crow[q];
            if (uu) {
                const double u = uu[grow + wrapg(ox + p, b.nx)];
                const double d = o == 24 ? inv_dt : 0.0;
                v = d + (1.0 - u * u) * (v - d);
            }
        }
        dst[e] = v;
    }
}

// As assemble_block, with c read from the field cc itself (box row J) instead of an LDS row.
__device__ void assemble_block_field(double* dst, int I, int J, const LuBox& b, const LdsStencil* t,
                                     const double* __restrict__ cc, const double* __restrict__ uu, int ox, int oy,
                                     double inv_dt) {
    const int W = b.W, dy = J - I;
    const long grow = (long)wrapg(oy + I, b.ny) * b.nx;
    const long crow = (long)wrapg(oy + J, b.ny) * b.nx;
    for (int e = threadIdx.x; e < W * W; e += blockDim.x) {
        const int p = e / W, q = e - p * W;
        const int dx = q - p;
        double v = 0.0;
        if (abs(dx) + abs(dy) <= 3) {
            const int o = (dy + 3) * 7 + dx + 3;
            v = t->k[o] - t->d1[o] * cc[crow + wrapg(ox + q, b.nx)];
            if (uu) {
                const double u = uu[grow + wrapg(ox + p, b.nx)];
                const double d = o == 24 ? inv_dt : 0.0;
                v = d + (1.0 - u * u) * (v - d);
            }
        }
        dst[e] = v;
    }
}

// c along box row J into the LDS ring slot J % 8 (W <= 72 values per slot).
__device__ void load_c_row(double* ring, int J, const LuBox& b, const double* __restrict__ cc, int ox, int oy) {
    const long row = (long)wrapg(oy + J, b.ny) * b.nx;
    for (int q = threadIdx.x; q < b.W; q += blockDim.x) ring[(J & 7) * 72 + q] = cc[row + wrapg(ox + q, b.nx)];
}

// Inverse of the W x W block in G0 by Gauss-Jordan elimination without pivoting, taking
// the pivots four at a time: for the pivot block K = {k0..k0+3} with P = a(K,K),
//     a'(K,K) = P^-1,            a'(K,j) = P^-1 a(K,j),
//     a'(i,K) = -a(i,K) P^-1,    a'(i,j) = a(i,j) - a(i,K) a'(K,j)      (i, j not in K),
// which is four scalar Gauss-Jordan steps done at once.  First the threads of the first W
// columns each invert the 4 x 4 pivot block in registers (scalar Gauss-Jordan, same pivots)
// and write their column of the new pivot rows a'(K, :); after a barrier every other entry
// takes four products with those rows (a'(i,K) = -a(i,K) a'(K,K)).  The matrix is double-
// buffered through G1, two barriers per pivot block.  A last block narrower than four is
// padded with the identity.  Returns the buffer holding the inverse.
__device__ double* gauss_jordan(double* G0, double* G1, int W, int* flag) {
    const int tid = threadIdx.x, nt = blockDim.x;
    double* a = G0;
    double* o = G1;
    for (int k0 = 0; k0 < W; k0 += 4) {
        const int bs = min(4, W - k0);
        if (tid < W) {                               // column j = tid of the pivot rows
            double P[4][4];
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    P[r][c] = (r < bs && c < bs) ? a[(k0 + r) * W + k0 + c] : (r == c ? 1.0 : 0.0);
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {         // in-register Gauss-Jordan of P
                const double piv = P[kk][kk];
                if (tid == 0 && (!(piv != 0.0) || !isfinite(piv))) *flag = 1;
                const double ip = 1.0 / piv;
                double rowk[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) rowk[c] = (c == kk) ? ip : P[kk][c] * ip;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if (r == kk) continue;
                    const double f = P[r][kk];
#pragma unroll
                    for (int c = 0; c < 4; ++c) P[r][c] = (c == kk ? 0.0 : P[r][c]) - f * rowk[c];
                }
#pragma unroll
                for (int c = 0; c < 4; ++c) P[kk][c] = rowk[c];
            }
            const int j = tid, cj = j - k0;
            double aKj[4];
#pragma unroll
            for (int s = 0; s < 4; ++s) aKj[s] = (s < bs) ? a[(k0 + s) * W + j] : 0.0;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                if (r >= bs) break;
                double v;
                if (cj >= 0 && cj < bs) {            // a'(K,K) = P^-1
                    v = 0.0;
#pragma unroll
                    for (int c = 0; c < 4; ++c)
                        if (c == cj) v = P[r][c];
                } else {                             // a'(K,j) = P^-1 a(K,j)
                    v = 0.0;
#pragma unroll
                    for (int s = 0; s < 4; ++s) v += P[r][s] * aKj[s];
                }
                o[(k0 + r) * W + j] = v;
            }
        }
        __syncthreads();
        for (int e = tid; e < W * W; e += nt) {
            const int i = e / W, j = e - i * W;
            if (i >= k0 && i < k0 + bs) continue;    // the pivot rows, written above
            const bool jK = j >= k0 && j < k0 + bs;
            double v = jK ? 0.0 : a[e];
#pragma unroll
            for (int s = 0; s < 4; ++s)
                if (s < bs) v -= a[i * W + k0 + s] * o[(k0 + s) * W + j];
            o[e] = v;
        }
        __syncthreads();
        double* t = a;
        a = o;
        o = t;
    }
    return a;
}

// Dense W x W product on one 4 x 4 register tile, operands in LDS (row-major, ld = W);
// tile t covers rows 4*(t / nq).., columns 4*(t % nq).., indices clamped at the edge.
template <int WMAX>
__device__ __forceinline__ void tile_product(const double* A, const double* B, int W, int tile,
                                             double acc[4][4], int* p0, int* q0) {
    const int nq = (W + 3) / 4;
    *p0 = 4 * (tile / nq);
    *q0 = 4 * (tile - (tile / nq) * nq);
    int pr[4], qc[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        pr[a] = min(*p0 + a, W - 1);
        qc[a] = min(*q0 + a, W - 1);
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[a][c] = 0.0;
    constexpr int UNR = WMAX <= 24 ? 2 : 4;   // the W <= 24 kernel runs four workgroups per CU (128 VGPRs)
#pragma unroll UNR
    for (int m = 0; m < W; ++m) {
        {
            double av[4], bv[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) av[a] = A[pr[a] * W + m];
#pragma unroll
            for (int c = 0; c < 4; ++c) bv[c] = B[m * W + qc[c]];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[a][c] += av[a] * bv[c];
        }
    }
}

// Boxes of width W <= kSmallW: the blocks of a step are staged in LDS:
//   G0, G1 (Gauss-Jordan; after it the one not holding S^-1 takes Uh(K,K+1)),
//   A(K+1..K+2, K) -> Pa[2], A(K, K+1..K+2) -> Pu[2], and Uh(K,K+2):
//   7 W^2 doubles, four workgroups per CU at W = 24.  Lh goes from registers straight to the
//   factors, and the Schur updates take the form A(I,J) -= A(I,K) Uh(K,J) (equal to
//   Lh(I,K) A(K,J)), so neither Lh nor A(K,J) has to stay in LDS.
// The blocks at distance 3, A(K+3, K) and A(K, K+3), are diagonal (the stencil reaches three
// rows only straight up and down) and no elimination step updates them (a step K' updates
// blocks within distance 3 of K' on both sides).  So Lh(K+3, K) = diag(dA) S^-1 and
// Uh(K, K+3) = S^-1 diag(dB) are scalings of S^-1, and the Schur terms that involve them are
// scalings too: 8 dense W x W products per step instead of 15.
template <typename T, int WMAX>
__global__ __launch_bounds__(256, WMAX <= 24 ? 4 : 3) void k_lu_factor_lds(const double* __restrict__ cc, double* __restrict__ work,
                                                       T* __restrict__ fac, int* __restrict__ flag, LuBox b,
                                                       StencilTable st, const double* __restrict__ uu) {
    extern __shared__ double lds[];
    const int W = b.W, H = b.H, WW = W * W;
    double* G0 = lds;
    double* G1 = lds + WW;
    double* Pa = lds + 2 * WW;
    double* Pu = lds + 4 * WW;   // A(K, K+1..K+2) as staged
    const int k = blockIdx.x;
    const int ox = (k % b.subx) * b.ownx - b.ov, oy = (k / b.subx) * b.owny - b.ov;
    double* win = work + (long)k * 16 * WW;
    T* out = fac + (long)k * H * 7 * WW;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int nq = (W + 3) / 4;
    const int ntile = nq * nq;
    __shared__ LdsStencil sst;
    __shared__ double cring[8 * 72];        // c along the box rows entering the window
    __shared__ double dA[WMAX], dB[WMAX];   // diagonals of A(K+3, K) and A(K, K+3)
    stage_stencil(&sst, b, st);
    for (int J = 0; J < 5 && J < H; ++J) load_c_row(cring, J, b, cc, ox, oy);
    __syncthreads();

    for (int I = 0; I < 4 && I < H; ++I)
        for (int J = 0; J < 4 && J < H; ++J)
            assemble_block(slot(win, I, J, W), I, J, b, &sst, cring + (J & 7) * 72, uu, ox, oy, st.inv_dt);
    __syncthreads();

    for (int K = 0; K < H; ++K) {
        const int nI = min(3, H - 1 - K);
        const int nd = min(nI, 2);          // dense neighbour blocks on each side
        T* rowK = out + (long)K * 7 * WW;
        for (int e = tid; e < WW; e += nt) G0[e] = slot(win, K, K, W)[e];
        for (int e = tid; e < nd * WW; e += nt) {
            const int bi = e / WW, r = e - bi * WW;
            Pa[bi * WW + r] = slot(win, K + 1 + bi, K, W)[r];
            Pu[bi * WW + r] = slot(win, K, K + 1 + bi, W)[r];
        }
        if (nI == 3)
            for (int q = tid; q < W; q += nt) {
                dA[q] = slot(win, K + 3, K, W)[q * W + q];
                dB[q] = slot(win, K, K + 3, W)[q * W + q];
            }
        __syncthreads();
        const double* Sinv = gauss_jordan(G0, G1, W, flag);
        // Lh(I,K) = A(I,K) S^-1, I = K+1, K+2, tile by tile to the factors of row I (column
        // block 2 - bi), with A(I, K+3) -= Lh(I,K) diag(dB) applied from the same registers.
        // Uh(K,K+1) = S^-1 A(K,K+1) goes to the Gauss-Jordan buffer that does not hold S^-1,
        // Uh(K,K+2) = S^-1 A(K,K+2) to a buffer of its own, both in the same pass as Lh.
        double* Uh0 = Sinv == G0 ? G1 : G0;
        double* Uh1 = lds + 6 * WW;
        const int nprod = nd + 1 + (nd == 2 ? 1 : 0);
        // Block row and column K + 4 enter the window in the slots of row and column K, which
        // are staged and no longer read: the threads past the last product tile assemble them
        // during this pass (at the end of the step if too few are left over).
        const int N4 = K + 4;
        const int idle0 = nprod * ntile;
        const bool early = N4 < H && idle0 + 64 <= nt;
        for (int t = tid; t < nprod * ntile; t += nt) {
            const int b = t / ntile, tile = t - b * ntile;
            double acc[4][4];
            int p0, q0;
            if (b < nd) {
                tile_product<WMAX>(Pa + b * WW, Sinv, W, tile, acc, &p0, &q0);
                T* dst = out + (long)(K + 1 + b) * 7 * WW + (2 - b) * WW;
                double* C3 = nI == 3 ? slot(win, K + 1 + b, K + 3, W) : nullptr;
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int c = 0; c < 4; ++c)
                        if (p0 + a < W && q0 + c < W) {
                            dst[(q0 + c) * W + p0 + a] = (T)acc[a][c];
                            if (C3) C3[(p0 + a) * W + q0 + c] -= acc[a][c] * dB[q0 + c];
                        }
            } else {
                const int bj = b - nd;                 // Uh(K, K+1+bj)
                double* U = bj == 0 ? Uh0 : Uh1;
                tile_product<WMAX>(Sinv, Pu + bj * WW, W, tile, acc, &p0, &q0);
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int c = 0; c < 4; ++c)
                        if (p0 + a < W && q0 + c < W) U[(p0 + a) * W + q0 + c] = acc[a][c];
            }
        }
        if (early && tid >= idle0) {
            for (int J = K + 1; J <= N4; ++J)
                assemble_block(slot(win, N4, J, W), N4, J, b, &sst, cring + (J & 7) * 72, uu, ox, oy, st.inv_dt,
                               tid - idle0, nt - idle0);
            for (int I = K + 1; I < N4; ++I)
                assemble_block(slot(win, I, N4, W), I, N4, b, &sst, cring + (N4 & 7) * 72, uu, ox, oy, st.inv_dt,
                               tid - idle0, nt - idle0);
        }
        __syncthreads();
        const double* Uh[2] = {Uh0, Uh1};
        // block row K: S^-1 and -Uh(K, K+1..K+3) (zero past the box; Lh blocks before it zero);
        // Lh(K+3, K) = diag(dA) S^-1 into column block 0 of row K+3.  e = q * W + p: coalesced
        // column-major stores.
        for (int e = tid; e < WW; e += nt) {
            const int q = e / W, p = e - q * W, rm = p * W + q;
            const double sv = Sinv[rm];
            rowK[3 * WW + e] = (T)sv;
            for (int bj = 0; bj < 3; ++bj) {
                const double u = bj < nd ? Uh[bj][rm] : (bj < nI ? sv * dB[q] : 0.0);
                rowK[4 * WW + bj * WW + e] = (T)(-u);
            }
            if (K < 3)
                for (int cb = 0; cb < 3 - K; ++cb) rowK[cb * WW + e] = (T)0.0;
            if (nI == 3) out[(long)(K + 3) * 7 * WW + e] = (T)(dA[p] * sv);
        }
        // Schur complement A(I,J) -= A(I,K) Uh(K,J): dense for I, J = K+1, K+2.  (The C tile is
        // read after the product: held through it, beside the product's own tile, it would
        // not fit the 128 registers of four workgroups per CU.) ...
        const int nsch = nd * nd * ntile;
        for (int t = tid; t < nsch; t += nt) {
            const int blk = t / ntile, tile = t - blk * ntile;
            const int bi = blk / nd, bj = blk - bi * nd;
            double* C = slot(win, K + 1 + bi, K + 1 + bj, W);
            double acc[4][4];
            int p0, q0;
            tile_product<WMAX>(Pa + bi * WW, Uh[bj], W, tile, acc, &p0, &q0);
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    if (p0 + a < W && q0 + c < W) C[(p0 + a) * W + q0 + c] -= acc[a][c];
        }
        // ... and the scalings where a distance-3 block takes part (A(I, K+3) -= Lh(I,K) diag(dB)
        // was applied with Lh above):
        //   A(K+3, J) -= diag(dA) Uh(K,J), A(K+3, K+3) -= diag(dA) S^-1 diag(dB)
        if (nI == 3)
            for (int e = tid; e < 3 * WW; e += nt) {
                const int c3 = e / WW, rm = e - c3 * WW, p = rm / W, q = rm - p * W;
                if (c3 < 2)
                    slot(win, K + 3, K + 1 + c3, W)[rm] -= dA[p] * Uh[c3][rm];
                else
                    slot(win, K + 3, K + 3, W)[rm] -= dA[p] * Sinv[rm] * dB[q];
            }
        __syncthreads();
        // slide the window: block row and column K + 4 enter (unless assembled above)
        if (N4 < H && !early) {
            for (int J = K + 1; J <= N4; ++J) assemble_block(slot(win, N4, J, W), N4, J, b, &sst, cring + (J & 7) * 72, uu, ox, oy,
                                                     st.inv_dt);
            for (int I = K + 1; I < N4; ++I) assemble_block(slot(win, I, N4, W), I, N4, b, &sst, cring + (N4 & 7) * 72, uu, ox, oy,
                                                     st.inv_dt);
        }
        if (N4 + 1 < H) load_c_row(cring, N4 + 1, b, cc, ox, oy);   // ring slot of row K-3, no longer read
        __syncthreads();
    }
}

// C (+)= sign * A B for W x W blocks with A streamed by rows from global memory and B in
// LDS.  Thread t owns row p = t / TPR and the columns q = (t % TPR) + TPR * i; it keeps
// chunks of 8 entries of its row of A in registers, so A is read once per output row.  Two
// chunk buffers alternate: the next chunk's loads are in flight while the current one is
// used, and they are unconditional (index clamped; entries past the row count as zero when
// used), so no select follows a load.
template <int QMAX>
__device__ void gemm_rows(double* C, const double* __restrict__ A, const double* B, int W, double sign,
                          bool accumulate) {
    const int tid = threadIdx.x, TPR = blockDim.x / W;
    const int p = tid / TPR, q0 = tid - p * TPR;
    if (p >= W) return;
    double acc[QMAX];
#pragma unroll
    for (int i = 0; i < QMAX; ++i) acc[i] = 0.0;
    auto load = [&](double (&a)[8], int m0) {
#pragma unroll
        for (int mm = 0; mm < 8; ++mm) a[mm] = A[p * W + min(m0 + mm, W - 1)];
    };
    auto use = [&](const double (&a)[8], int m0) {
#pragma unroll
        for (int i = 0; i < QMAX; ++i) {
            const int q = min(q0 + TPR * i, W - 1);     // clamped: tail lanes compute a discarded duplicate
#pragma unroll
            for (int mm = 0; mm < 8; ++mm) {
                const int m = min(m0 + mm, W - 1);
                acc[i] += (m0 + mm < W ? a[mm] : 0.0) * B[m * W + q];
            }
        }
    };
    double a0[8], a1[8];
    load(a0, 0);
    for (int m0 = 0; m0 < W; m0 += 16) {
        load(a1, m0 + 8);
        use(a0, m0);
        if (m0 + 8 >= W) break;
        load(a0, m0 + 16);
        use(a1, m0 + 8);
    }
#pragma unroll
    for (int i = 0; i < QMAX; ++i) {
        const int q = q0 + TPR * i;
        if (q < W) C[p * W + q] = (accumulate ? C[p * W + q] : 0.0) + sign * acc[i];
    }
}

// C = A B with A in LDS and B streamed by columns from global memory.
template <int PMAX>
__device__ void gemm_cols(double* C, const double* A, const double* __restrict__ B, int W) {
    const int tid = threadIdx.x, TPC = blockDim.x / W;
    const int q = tid / TPC, p0 = tid - q * TPC;
    if (q >= W) return;
    double acc[PMAX];
#pragma unroll
    for (int i = 0; i < PMAX; ++i) acc[i] = 0.0;
    // two alternating chunk buffers with unconditional loads, as in gemm_rows
    auto load = [&](double (&bc)[8], int m0) {
#pragma unroll
        for (int mm = 0; mm < 8; ++mm) bc[mm] = B[min(m0 + mm, W - 1) * W + q];
    };
    auto use = [&](const double (&bc)[8], int m0) {
#pragma unroll
        for (int i = 0; i < PMAX; ++i) {
            const int p = min(p0 + TPC * i, W - 1);
#pragma unroll
            for (int mm = 0; mm < 8; ++mm) {
                const int m = min(m0 + mm, W - 1);
                acc[i] += A[p * W + m] * (m0 + mm < W ? bc[mm] : 0.0);
            }
        }
    };
    double b0[8], b1[8];
    load(b0, 0);
    for (int m0 = 0; m0 < W; m0 += 16) {
        load(b1, m0 + 8);
        use(b0, m0);
        if (m0 + 8 >= W) break;
        load(b0, m0 + 16);
        use(b1, m0 + 8);
    }
#pragma unroll
    for (int i = 0; i < PMAX; ++i) {
        const int p = p0 + TPC * i;
        if (p < W) C[p * W + q] = acc[i];
    }
}

// Wider boxes (kSmallW < W <= 72): Gauss-Jordan in LDS, panels in the global workspace
// (blocks 16..21), the A(K, J) blocks staged into LDS for the Schur update (2 W^2 doubles).
// As in k_lu_factor_lds, the diagonal blocks at distance 3 make their panels and Schur terms
// scalings, formed elementwise.
template <typename T>
__global__ __launch_bounds__(256) void k_lu_factor_wide(const double* __restrict__ cc, double* __restrict__ work,
                                                        T* __restrict__ fac, int* __restrict__ flag, LuBox b,
                                                        StencilTable st, const double* __restrict__ uu) {
    extern __shared__ double lds[];
    const int W = b.W, H = b.H, WW = W * W;
    const int k = blockIdx.x;
    const int ox = (k % b.subx) * b.ownx - b.ov, oy = (k / b.subx) * b.owny - b.ov;
    double* win = work + (long)k * 22 * WW;
    T* out = fac + (long)k * H * 7 * WW;
    const int tid = threadIdx.x, nt = blockDim.x;
    // c is read from the field when a block is assembled (no LDS ring), which keeps a 70-wide
    // box within half the LDS of a CU: two workgroups per CU instead of one
    __shared__ LdsStencil sst;
    __shared__ double dA[72], dB[72];       // diagonals of A(K+3, K) and A(K, K+3)
    stage_stencil(&sst, b, st);
    __syncthreads();

    for (int I = 0; I < 4 && I < H; ++I)
        for (int J = 0; J < 4 && J < H; ++J)
            assemble_block_field(slot(win, I, J, W), I, J, b, &sst, cc, uu, ox, oy, st.inv_dt);
    __syncthreads();

    for (int K = 0; K < H; ++K) {
        const int nI = min(3, H - 1 - K);
        const int nd = min(nI, 2);
        T* rowK = out + (long)K * 7 * WW;
        for (int e = tid; e < WW; e += nt) lds[e] = slot(win, K, K, W)[e];
        if (nI == 3)
            for (int q = tid; q < W; q += nt) {
                dA[q] = slot(win, K + 3, K, W)[q * W + q];
                dB[q] = slot(win, K, K + 3, W)[q * W + q];
            }
        __syncthreads();
        const double* Sinv = gauss_jordan(lds, lds + WW, W, flag);
        // Lh(I,K) = A(I,K) S^-1 -> blocks 16+bi; Uh(K,J) = S^-1 A(K,J) -> blocks 19+bj (I, J = K+1, K+2)
        for (int bi = 0; bi < nd; ++bi)
            gemm_rows<24>(win + (long)(16 + bi) * WW, slot(win, K + 1 + bi, K, W), Sinv, W, 1.0, false);
        for (int bj = 0; bj < nd; ++bj)
            gemm_cols<24>(win + (long)(19 + bj) * WW, Sinv, slot(win, K, K + 1 + bj, W), W);
        // S^-1 of block row K and, while S^-1 is in LDS, the distance-3 scalings:
        // Lh(K+3,K) = diag(dA) S^-1, Uh(K,K+3) = S^-1 diag(dB), A(K+3,K+3) -= diag(dA) S^-1 diag(dB)
        for (int e = tid; e < WW; e += nt) {
            const int q = e / W, p = e - q * W, rm = p * W + q;
            const double sv = Sinv[rm];
            rowK[3 * WW + e] = (T)sv;
            if (nI == 3) {
                out[(long)(K + 3) * 7 * WW + e] = (T)(dA[p] * sv);
                rowK[6 * WW + e] = (T)(-(sv * dB[q]));
                slot(win, K + 3, K + 3, W)[rm] -= dA[p] * sv * dB[q];
            }
        }
        __syncthreads();
        double* As = lds;                // S^-1 is done: stage A(K, K+1..K+2) for the Schur update
        for (int e = tid; e < nd * WW; e += nt) {
            const int bj = e / WW, r = e - bj * WW;
            As[e] = slot(win, K, K + 1 + bj, W)[r];
        }
        __syncthreads();
        for (int bi = 0; bi < nd; ++bi)
            for (int bj = 0; bj < nd; ++bj)
                gemm_rows<24>(slot(win, K + 1 + bi, K + 1 + bj, W), win + (long)(16 + bi) * WW, As + (long)bj * WW,
                              W, -1.0, true);
        // A(I, K+3) -= Lh(I,K) diag(dB) and A(K+3, J) -= diag(dA) Uh(K,J), I, J = K+1, K+2
        if (nI == 3)
            for (int e = tid; e < 4 * WW; e += nt) {
                const int c4 = e / WW, rm = e - c4 * WW, p = rm / W, q = rm - p * W;
                if (c4 < 2)
                    slot(win, K + 1 + c4, K + 3, W)[rm] -= win[(long)(16 + c4) * WW + rm] * dB[q];
                else
                    slot(win, K + 3, K + c4 - 1, W)[rm] -= dA[p] * win[(long)(19 + c4 - 2) * WW + rm];
            }
        for (int e = tid; e < WW; e += nt) {
            const int q = e / W, p = e - q * W, rm = p * W + q;
            for (int bj = 0; bj < 3; ++bj) {
                if (bj < nd) rowK[4 * WW + bj * WW + e] = (T)(-win[(long)(19 + bj) * WW + rm]);
                else if (bj >= nI) rowK[4 * WW + bj * WW + e] = (T)0.0;
            }
            if (K < 3)
                for (int cb = 0; cb < 3 - K; ++cb) rowK[cb * WW + e] = (T)0.0;
            for (int bi = 0; bi < nd; ++bi)
                out[(long)(K + 1 + bi) * 7 * WW + (2 - bi) * WW + e] = (T)win[(long)(16 + bi) * WW + rm];
        }
        __syncthreads();
        const int N4 = K + 4;
        if (N4 < H) {
            for (int J = K + 1; J <= N4; ++J)
                assemble_block_field(slot(win, N4, J, W), N4, J, b, &sst, cc, uu, ox, oy, st.inv_dt);
            for (int I = K + 1; I < N4; ++I)
                assemble_block_field(slot(win, I, N4, W), I, N4, b, &sst, cc, uu, ox, oy, st.inv_dt);
        }
        __syncthreads();
    }
}

// Block solve.  Thread (p, g), g < G = blockDim / W, handles row p of a block row and the
// columns q = g + G*i of its dense product; it holds the factors of DEPTH block rows ahead
// in registers so that their loads overlap the barriers of the current row.  The factors are
// read once per apply and far exceed the caches; with three rows in flight they are loaded
// non-temporally, streaming past the caches instead of evicting the box vectors' gather
// lines (measured faster there; with one row in flight, on 70-wide boxes, it was slower).
//   forward  (half 0): z_I = y_I - [Lh(I,I-3..I-1)] y[(I-3)W : IW]        (3W columns)
//   backward (half 1): x_I = [S_II^-1 | -Uh(I,I+1..I+3)] y[IW : (I+4)W]    (4W columns)
template <typename T, int NPL, int DEPTH>
__global__ void k_lu_apply(const double* __restrict__ r, double* __restrict__ z, const T* __restrict__ fac,
                           LuBox b, double* __restrict__ sum_part, int mode, double* __restrict__ zbox) {
    extern __shared__ unsigned char smem_raw[];
    const int W = b.W, H = b.H, WW = W * W;
    T* y = reinterpret_cast<T*>(smem_raw);          // W*H box vector
    T* red = y + W * H;                              // G * W partial sums
    const int tid = threadIdx.x;
    const int G = blockDim.x / W;
    const int p = tid % W, g = tid / W;
    const bool act = g < G;
    const int k = blockIdx.x;
    const int ox = (k % b.subx) * b.ownx - b.ov, oy = (k / b.subx) * b.owny - b.ov;
    const T* F = fac + (long)k * H * 7 * WW;

    for (int e = tid; e < W * H; e += blockDim.x) {
        const int x = e % W, yy = e / W;
        // right-RAS restricts the owned cells only (Eq. (24)); the others restrict the whole box
        const bool own = x >= b.ov && x < b.ov + b.ownx && yy >= b.ov && yy < b.ov + b.owny;
        y[e] = (mode != 2 || own) ? (T)r[(long)wrapg(oy + yy, b.ny) * b.nx + wrapg(ox + x, b.nx)] : (T)0;
    }

    T pl[DEPTH + 1][NPL];
    constexpr bool kNonTemporal = DEPTH >= 3;
    auto load = [&](int I, int half, T* l) {
        const T* base = F + (long)I * 7 * WW + half * 3 * WW;
        const int ncol = half ? 4 * W : 3 * W;
#pragma unroll
        for (int i = 0; i < NPL; ++i) {
            const int q = g + G * i;
            if constexpr (kNonTemporal)
                l[i] = (act && q < ncol) ? __builtin_nontemporal_load(&base[q * W + p]) : (T)0;
            else
                l[i] = (act && q < ncol) ? base[q * W + p] : (T)0;
        }
    };
    auto rotate = [&]() {
#pragma unroll
        for (int d = 0; d < DEPTH; ++d)
#pragma unroll
            for (int i = 0; i < NPL; ++i) pl[d][i] = pl[d + 1][i];
    };

    // forward sweep
#pragma unroll
    for (int d = 0; d < DEPTH; ++d)
        if (d < H) load(d, 0, pl[d]);
    __syncthreads();
    for (int I = 0; I < H; ++I) {
        if (I + DEPTH < H) load(I + DEPTH, 0, pl[DEPTH]);
        if (act) {
            T acc = 0;
            const int base = (I - 3) * W;
#pragma unroll
            for (int i = 0; i < NPL; ++i) {
                const int q = g + G * i;
                if (q < 3 * W && base + q >= 0) acc += pl[0][i] * y[base + q];
            }
            red[g * W + p] = acc;
        }
        __syncthreads();
        if (tid < W) {
            T s = y[I * W + tid];
            for (int gg = 0; gg < G; ++gg) s -= red[gg * W + tid];
            y[I * W + tid] = s;
        }
        __syncthreads();
        rotate();
    }
    // backward sweep (S^-1 and -Uh in one product)
#pragma unroll
    for (int d = 0; d < DEPTH; ++d)
        if (H - 1 - d >= 0) load(H - 1 - d, 1, pl[d]);
    for (int I = H - 1; I >= 0; --I) {
        if (I - DEPTH >= 0) load(I - DEPTH, 1, pl[DEPTH]);
        if (act) {
            T acc = 0;
            const int base = I * W;
            const int qend = (1 + min(3, H - 1 - I)) * W;
#pragma unroll
            for (int i = 0; i < NPL; ++i) {
                const int q = g + G * i;
                if (q < qend) acc += pl[0][i] * y[base + q];
            }
            red[g * W + p] = acc;
        }
        __syncthreads();
        if (tid < W) {
            T s = 0;
            for (int gg = 0; gg < G; ++gg) s += red[gg * W + tid];
            y[I * W + tid] = s;
        }
        __syncthreads();
        rotate();
    }
    // extension, and the sum of what this box contributes (for the zero-mean projection)
    double acc = 0.0;
    if (mode == 0) {   // left-RAS: owned cells only (Eq. (23))
        for (int e = tid; e < b.ownx * b.owny; e += blockDim.x) {
            const int x = e % b.ownx + b.ov, yy = e / b.ownx + b.ov;
            const double v = (double)y[yy * W + x];
            z[(long)wrapg(oy + yy, b.ny) * b.nx + wrapg(ox + x, b.nx)] = v;
            acc += v;
        }
    } else {           // classical AS / right-RAS: the whole box, added per cell afterwards
        for (int e = tid; e < W * H; e += blockDim.x) {
            const double v = (double)y[e];
            zbox[(long)k * W * H + e] = v;
            acc += v;
        }
    }
    if (sum_part) {
        __shared__ double red[16];
        const double sum = block_sum_det(acc, red);
        if (tid == 0) sum_part[blockIdx.x] = sum;
    }
}

LuBox make_lubox(const pfc_ctx* c, const StencilTable& st) {
    LuBox b;
    b.W = c->dec.ext[0];
    b.H = c->dec.ext[1];
    b.subx = c->dec.sub[0];
    b.ownx = c->dec.own[0];
    b.owny = c->dec.own[1];
    b.ov = c->dec.ov;
    b.nx = c->g.nx;
    b.ny = c->g.ny;
    for (int i = 0; i < 49; ++i) b.idx7[i] = -1;
    for (int s = 0; s < st.S; ++s) b.idx7[(st.dy[s] + 3) * 7 + st.dx[s] + 3] = s;
    return b;
}

// Launch shape of the solve for box width W; NPL covers ceil(4W / G), G = threads / W:
//   W <= 24: 256 threads, G >= 10 -> NPL 10, prefetch 3 rows (FP32) / 1 row (FP64)  (measured best)
//   W <= 32: 256 threads, G >= 8  -> NPL 16, prefetch 2 rows (FP32) / 1 row (FP64)
//   W <= 72: 1024 threads, G >= 14 -> NPL 21, prefetch 1 row (FP32) / none (FP64)
template <typename T>
hipError_t launch_apply_t(pfc_ctx* c, const double* r, double* z, const LuBox& b, double* sum_part) {
    constexpr bool f32 = sizeof(T) == 4;
    const int threads = b.W <= 32 ? 256 : 1024;
    const int G = threads / b.W;
    const int npl = b.W <= 24 ? 10 : (b.W <= 32 ? 16 : 21);
    if (G * npl < 4 * b.W) return hipErrorInvalidValue;   // a block row's columns must be covered
    const size_t sh = sizeof(T) * ((size_t)b.W * b.H + (size_t)G * b.W);
    const T* f = (const T*)c->d_fac;
    const dim3 grid(c->dec.nsub), blk(threads);
    if (b.W <= 24)
        return launch_k(c, k_lu_apply<T, 10, f32 ? 3 : 1>, grid, blk, sh, r, z, f, b, sum_part, c->opts.ras_kind,
                        c->d_zbox);
    if (b.W <= 32)
        return launch_k(c, k_lu_apply<T, 16, f32 ? 2 : 1>, grid, blk, sh, r, z, f, b, sum_part, c->opts.ras_kind,
                        c->d_zbox);
    return launch_k(c, k_lu_apply<T, 21, f32 ? 1 : 0>, grid, blk, sh, r, z, f, b, sum_part, c->opts.ras_kind,
                    c->d_zbox);
}

}  // namespace

size_t lu_factor_lds_bytes(int W) { return sizeof(double) * (W <= kSmallW ? 7 : 2) * (size_t)W * W; }

size_t lu_work_blocks(int W) { return W <= kSmallW ? 16 : 22; }

size_t lu_factor_elems_per_block_row(int W) { return 7 * (size_t)W * W; }

hipError_t launch_lu_factor(pfc_ctx* c, const StencilTable& st) {
    const LuBox b = make_lubox(c, st);
    const size_t sh = lu_factor_lds_bytes(b.W);
    const dim3 grid(c->dec.nsub), blk(256);
    const bool f32 = c->opts.precond_fp32;
    float* ff = (float*)c->d_fac;
    double* fd = (double*)c->d_fac;
    if (b.W <= 24) {
        if (f32)
            hipLaunchKernelGGL((k_lu_factor_lds<float, 24>), grid, blk, sh, c->stream, c->d_c, c->d_work, ff,
                               c->d_flag, b, st, (const double*)c->d_u);
        else
            hipLaunchKernelGGL((k_lu_factor_lds<double, 24>), grid, blk, sh, c->stream, c->d_c, c->d_work, fd,
                               c->d_flag, b, st, (const double*)c->d_u);
    } else if (b.W <= kSmallW) {
        if (f32)
            hipLaunchKernelGGL((k_lu_factor_lds<float, kSmallW>), grid, blk, sh, c->stream, c->d_c, c->d_work, ff,
                               c->d_flag, b, st, (const double*)c->d_u);
        else
            hipLaunchKernelGGL((k_lu_factor_lds<double, kSmallW>), grid, blk, sh, c->stream, c->d_c, c->d_work, fd,
                               c->d_flag, b, st, (const double*)c->d_u);
    } else {
        if (f32)
            hipLaunchKernelGGL(k_lu_factor_wide<float>, grid, blk, sh, c->stream, c->d_c, c->d_work, ff, c->d_flag,
                               b, st, (const double*)c->d_u);
        else
            hipLaunchKernelGGL(k_lu_factor_wide<double>, grid, blk, sh, c->stream, c->d_c, c->d_work, fd, c->d_flag,
                               b, st, (const double*)c->d_u);
    }
    return hipGetLastError();
}

hipError_t launch_lu_apply(pfc_ctx* c, const double* r, double* z, double* sum_part) {
    const LuBox b = make_lubox(c, c->st);
    if (c->opts.precond_fp32) return launch_apply_t<float>(c, r, z, b, sum_part);
    return launch_apply_t<double>(c, r, z, b, sum_part);
}

hipError_t set_lu_lds_limits() {
    const void* fns[] = {(const void*)k_lu_factor_lds<double, 24>, (const void*)k_lu_factor_lds<float, 24>,
                         (const void*)k_lu_factor_lds<double, kSmallW>, (const void*)k_lu_factor_lds<float, kSmallW>,
                         (const void*)k_lu_factor_wide<double>, (const void*)k_lu_factor_wide<float>,
                         (const void*)k_lu_apply<double, 10, 1>, (const void*)k_lu_apply<float, 10, 3>,
                         (const void*)k_lu_apply<double, 16, 1>, (const void*)k_lu_apply<float, 16, 2>,
                         (const void*)k_lu_apply<double, 21, 0>, (const void*)k_lu_apply<float, 21, 1>};
    for (const void* f : fns) {
        hipError_t e = set_dynamic_lds_limit(f);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace pfc
