// Stencil kernels of the DVD scheme: residual (Sec. 3, Eq. (12)), Jacobian
// coefficient and exact Jacobian action (Sec. 4, Eq. (19)), discrete energy and
// mass (Sec. 3, Eqs. (7)-(8)).
//
// 2-D, M = 1, periodic: one kernel per operator.  On large grids a wave sweeps a strip of
// columns down a segment of rows; the composite radius-3 operator is three five-point
// Laplacians applied one row behind each other, row neighbours in registers and column
// neighbours from the adjacent lanes.  On small grids a block stages a tile with its halo in
// LDS and applies the three Laplacians there.  Either way each field is read from HBM once
// and the result written once.
// 3-D, and 2-D with a variable mobility or Neumann boundaries: seven-point passes through
// global memory (L2-resident neighbours).
#include "device_reduce.h"
#include "pfc_internal.h"
#include "tiling.h"

namespace pfc {
namespace {

#ifndef PFC_STENCIL_TILE_Y
#define PFC_STENCIL_TILE_Y 16
#endif
constexpr int TX = 64;
constexpr int TY = PFC_STENCIL_TILE_Y;   // 64 x 16 outputs measured fastest (occupancy beats halo reuse)
constexpr int NT = 256;

struct P {
    int nx, ny, nz;
    double ihx2, ihy2, ihz2;
    double gamma, inv_dt;
    int neu;   // Neumann-type boundaries: the ghost beyond a face mirrors the cell inside it
    int mob;   // variable mobility M(u) = 1 - u^2, u = (Phi + phi)/2
};

__device__ __forceinline__ int wrap(int i, int n) {
    i %= n;
    return i < 0 ? i + n : i;
}



// ---------------------------------------------------------------------------
// 2-D sliding-window stencils (M = 1, periodic): one wave sweeps a strip of SW_OUT = 58 columns
// down a segment of rows.  Each lane holds one column (the strip plus three halo columns on
// either side); a new input row enters every iteration and the three radius-1 stages of the
// composite operator follow it one row behind each other, their row neighbours in registers
// and their column neighbours from the adjacent lanes.  Each field value is read from HBM once
// per strip (plus the halo columns and the three rows above and below a segment), the result
// written once, and no LDS pass or barrier stands between the stages.  The input rows are
// loaded several rows ahead.  Work items (strip, segment) are dealt to the waves in a fixed
// order, so the per-block partial sums are reproducible.
// ---------------------------------------------------------------------------

constexpr int SW_OUT = 58;   // output columns per strip (64 lanes minus 3 halo lanes per side)
constexpr int SW_PF = 4;         // input rows in flight ahead of the sweep
// Grids of at least this many cells take the sliding sweeps; smaller ones the LDS tiles, whose
// blocks have every load of a tile in flight at once (a small grid gives the sweeps too few
// waves to hide their row-by-row latency).
constexpr long SW_MIN_CELLS = 1L << 21;
constexpr int SW_WAVES = 4096;   // waves of the largest grid (1024 blocks of NT = 256 threads)

struct SwGeom {
    int nstrip, seg, nseg, items;
};

__host__ __device__ inline SwGeom sw_geom(int nx, int ny) {
    SwGeom g;
    g.nstrip = (nx + SW_OUT - 1) / SW_OUT;
    // rows per segment: as short as lets every item have a wave of its own in one round of the
    // grid (SW_WAVES waves), but at least 16 rows to amortise the 6 warm-up rows
    const int nseg_max = max(1, SW_WAVES / g.nstrip);
    g.seg = max(16, (ny + nseg_max - 1) / nseg_max);
    g.nseg = (ny + g.seg - 1) / g.seg;
    g.items = g.nstrip * g.nseg;
    return g;
}

// Work items handed out so that the blocks on one XCD (block b runs on XCD b mod 8 when the
// grid is a multiple of 8 or one item per block) take one contiguous range of items, and
// neighbouring items share their halo reads in that XCD's L2.  A bijection on [0, items).
__device__ __forceinline__ int xcd_item(int it, int items) {
    const int q = items >> 3, rem = items & 7, x = it & 7, r = it >> 3;
    return x * q + min(x, rem) + r;
}

// The value of the next (dpp 0x130, wave_shl:1) or previous (0x138, wave_shr:1) lane of the
// wave, moved by the data-parallel primitives of the vector ALU (no LDS round trip); a lane
// with no such neighbour reads zero (bound_ctrl), so the move needs no copy of its old value.
template <int CTRL>
__device__ __forceinline__ double lane_move(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = (int)(b & 0xffffffffLL), hi = (int)(b >> 32);
    const int rl = __builtin_amdgcn_mov_dpp(lo, CTRL, 0xF, 0xF, true);
    const int rh = __builtin_amdgcn_mov_dpp(hi, CTRL, 0xF, 0xF, true);
    return __longlong_as_double(((long long)rh << 32) | (unsigned int)rl);
}

// lap along x of a value held one column per lane (lanes at the strip edges get garbage, unused)
__device__ __forceinline__ double lapx(double v, double ihx2) {
    return (lane_move<0x130>(v) + lane_move<0x138>(v) - 2.0 * v) * ihx2;
}

// F = (Phi - phi)/dt - Delta_d mu_d - src with per-block partial sums of F^2 (and Phi^2).
__global__ __launch_bounds__(NT) void k_residual2d(const double* __restrict__ Phi,
                                                   const double* __restrict__ phi,
                                                   const double* __restrict__ src,
                                                   double* __restrict__ F,
                                                   double* __restrict__ part, double* __restrict__ xpart, P p) {
    __shared__ double red[NT / 64];
    const SwGeom G = sw_geom(p.nx, p.ny);
    const int lane = threadIdx.x & 63;
    // the wave's index is the same in all its lanes: taken as a scalar, every row, segment and
    // loop bound below is scalar too, and the loop's branches are uniform
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ngroups = (G.items + NT / 64 - 1) / (NT / 64);   // items by groups of a block's waves
    double acc = 0.0, accx = 0.0;
    for (int gb = blockIdx.x; gb < ngroups; gb += gridDim.x) {
        const int it = xcd_item(gb, ngroups) * (NT / 64) + wave;
        if (it >= G.items) continue;
        const int strip = it % G.nstrip, sg = it / G.nstrip;
        const int xo = strip * SW_OUT + lane - 3;                 // this lane's column
        const int x = wrap(xo, p.nx);
        const bool out = lane >= 3 && lane < 3 + SW_OUT && xo < p.nx;
        const int y0 = sg * G.seg, y1 = min(y0 + G.seg, p.ny);
        // rows y0-3 .. y1+2 enter; F of row r-3 leaves when row r has entered
        const int nrow = y1 - y0 + 6;
        int yl = wrap(y0 - 3, p.ny);                               // row of the next load
        // Two sets of SW_PF prefetch slots: while one set's rows are consumed the other is
        // refilled, so a slot's old value is dead before its new load is issued and both
        // share one register; no copy (and so no wait) follows a load.  Past the segment's
        // last row that row is loaded again (in bounds, from the cache), so no branch stands
        // around a load either.
        // addresses: a scalar row base plus the lane's column offset, fixed for the sweep
        const unsigned ux = x, uxo = out ? xo : 0;
        auto load = [&](double& A, double& B, int k) {
            const long rb = (long)yl * p.nx;
            A = (Phi + rb)[ux];
            B = (phi + rb)[ux];
            if (k + 1 < nrow) yl = yl + 1 == p.ny ? 0 : yl + 1;
        };
        double pa[SW_PF], pb[SW_PF], qa[SW_PF], qb[SW_PF];
#pragma unroll
        for (int k = 0; k < SW_PF; ++k) load(pa[k], pb[k], k);
        // windows at the top of iteration k (row r = y0 - 3 + k entering):
        double u0 = 0, u1 = 0;                  // u at rows r-1, r-2
        double q1 = 0, q2 = 0;                  // q at rows r-1, r-2
        double l1 = 0, l2 = 0;                  // Lu at rows r-2, r-3
        double m2 = 0, m3 = 0;                  // mu at rows r-3, r-4
        double d1 = 0, d2 = 0, d3 = 0;          // Phi - phi at rows r-1, r-2, r-3
        double a1 = 0, a2 = 0, a3 = 0;          // Phi at rows r-1, r-2, r-3
        auto row = [&](double a, double bb, int k) {
            const double un = 0.5 * (a + bb);
            const double qn = 0.25 * (a * a * a + a * a * bb + a * bb * bb + bb * bb * bb);
            // Lu at row r-1, mu at row r-2, F at row r-3
            const double ln = lapx(u0, p.ihx2) + (un + u1 - 2.0 * u0) * p.ihy2;
            const double mn =
                (1.0 - p.gamma) * u1 + 2.0 * l1 + lapx(l1, p.ihx2) + (ln + l2 - 2.0 * l1) * p.ihy2 + q2;
            const double lm = lapx(m2, p.ihx2) + (mn + m3 - 2.0 * m2) * p.ihy2;
            if (k >= 6 && k < nrow && out) {
                double f = d3 * p.inv_dt - lm;
                const long rb = (long)(y0 - 6 + k) * p.nx;
                if (src) f -= (src + rb)[uxo];
                (F + rb)[uxo] = f;
                acc += f * f;
                accx += a3 * a3;
            }
            // shift the windows by one row
            m3 = m2; m2 = mn;
            l2 = l1; l1 = ln;
            q2 = q1; q1 = qn;
            u1 = u0; u0 = un;
            a3 = a2; a2 = a1; a1 = a;
            d3 = d2; d2 = d1; d1 = a - bb;
        };
        // iterations past the last row (up to 2 SW_PF - 1) store nothing
        for (int k0 = 0; k0 < nrow; k0 += 2 * SW_PF) {
#pragma unroll
            for (int j = 0; j < SW_PF; ++j) {
                const double a = pa[j], bb = pb[j];
                load(qa[j], qb[j], k0 + SW_PF + j);
                row(a, bb, k0 + j);
            }
#pragma unroll
            for (int j = 0; j < SW_PF; ++j) {
                const double a = qa[j], bb = qb[j];
                load(pa[j], pb[j], k0 + 2 * SW_PF + j);
                row(a, bb, k0 + SW_PF + j);
            }
        }
    }
    if (part) {
        const double s = block_sum_det(acc, red);
        if (threadIdx.x == 0) part[blockIdx.x] = s;
    }
    if (xpart) {
        const double s = block_sum_det(accx, red);
        if (threadIdx.x == 0) xpart[blockIdx.x] = s;
    }
}

// Jv = v/dt - Delta_d[(1-gamma)/2 v + Delta_d v + 1/2 Delta_d^2 v + c v] with v shifted by -s,
// s = shift_scale * sum(shift_part[0..shift_n)) when shift_part is given (zero-mean projection
// fused into the load; every block forms s in the same order and block 0 stores it in
// *shift_out).
__global__ __launch_bounds__(NT) void k_jv2d(const double* __restrict__ v,
                                             const double* __restrict__ cc,
                                             const double* __restrict__ shift_part, int shift_n,
                                             double shift_scale, double* __restrict__ shift_out,
                                             double* __restrict__ Jv, P p) {
    __shared__ double red[NT / 64];
    double sh = 0.0;
    if (shift_part) {
        sh = shift_scale * sum_partials_bcast(shift_part, shift_n, red);
        if (shift_out && threadIdx.x == 0 && blockIdx.x == 0) *shift_out = sh;
    }
    const SwGeom G = sw_geom(p.nx, p.ny);
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // scalar, as in k_residual2d
    const int ngroups = (G.items + NT / 64 - 1) / (NT / 64);
    for (int gb = blockIdx.x; gb < ngroups; gb += gridDim.x) {
        const int it = xcd_item(gb, ngroups) * (NT / 64) + wave;
        if (it >= G.items) continue;
        const int strip = it % G.nstrip, sg = it / G.nstrip;
        const int xo = strip * SW_OUT + lane - 3;
        const int x = wrap(xo, p.nx);
        const bool out = lane >= 3 && lane < 3 + SW_OUT && xo < p.nx;
        const int y0 = sg * G.seg, y1 = min(y0 + G.seg, p.ny);
        const int nrow = y1 - y0 + 6;
        int yl = wrap(y0 - 3, p.ny);                               // row of the next load
        // two sets of prefetch slots, refilled with no branch, as in k_residual2d
        const unsigned ux = x, uxo = out ? xo : 0;
        auto load = [&](double& A, double& B, int k) {
            const long rb = (long)yl * p.nx;
            A = (v + rb)[ux];
            B = (cc + rb)[ux];
            if (k + 1 < nrow) yl = yl + 1 == p.ny ? 0 : yl + 1;
        };
        double pv[SW_PF], pc[SW_PF], qv[SW_PF], qc[SW_PF];
#pragma unroll
        for (int k = 0; k < SW_PF; ++k) load(pv[k], pc[k], k);
        // windows at the top of iteration k (row r = y0 - 3 + k entering):
        double v0 = 0, v1 = 0, v2 = 0;          // v at rows r-1, r-2, r-3
        double c1 = 0, c2 = 0;                   // c at rows r-1, r-2
        double l1 = 0, l2 = 0;                   // Lv at rows r-2, r-3
        double w2 = 0, w3 = 0;                   // inner operator at rows r-3, r-4
        auto row = [&](double vr, double cn, int k) {
            const double vn = vr - sh;
            const double ln = lapx(v0, p.ihx2) + (vn + v1 - 2.0 * v0) * p.ihy2;
            const double wn = 0.5 * (1.0 - p.gamma) * v1 + l1 +
                              0.5 * (lapx(l1, p.ihx2) + (ln + l2 - 2.0 * l1) * p.ihy2) + c2 * v1;
            const double lw = lapx(w2, p.ihx2) + (wn + w3 - 2.0 * w2) * p.ihy2;
            if (k >= 6 && k < nrow && out) (Jv + (long)(y0 - 6 + k) * p.nx)[uxo] = v2 * p.inv_dt - lw;
            w3 = w2; w2 = wn;
            l2 = l1; l1 = ln;
            c2 = c1; c1 = cn;
            v2 = v1; v1 = v0; v0 = vn;
        };
        for (int k0 = 0; k0 < nrow; k0 += 2 * SW_PF) {
#pragma unroll
            for (int j = 0; j < SW_PF; ++j) {
                const double a = pv[j], b = pc[j];
                load(qv[j], qc[j], k0 + SW_PF + j);
                row(a, b, k0 + j);
            }
#pragma unroll
            for (int j = 0; j < SW_PF; ++j) {
                const double a = qv[j], b = qc[j];
                load(pv[j], pc[j], k0 + 2 * SW_PF + j);
                row(a, b, k0 + SW_PF + j);
            }
        }
    }
}

// Periodic index for i in [-n, 2n): one compare and add instead of a division.
__device__ __forceinline__ int wrap1(int i, int n) {
    return i < 0 ? i + n : (i >= n ? i - n : i);
}

// Halo staging in two phases: each thread first issues all of its global loads (a fixed,
// unrolled count), then writes them to LDS, so a block has every load in flight at once
// instead of one round trip per loop iteration.
constexpr int NE3 = (TY + 6) * (TX + 6);          // cells of the halo-3 tile
constexpr int NIT3 = (NE3 + NT - 1) / NT;
constexpr int NIT0 = (TY * TX + NT - 1) / NT;     // interior cells per thread

#define LAP2(A, y, x)                                                     \
    (((A)[y][(x) + 1] + (A)[y][(x)-1] - 2.0 * (A)[y][x]) * p.ihx2 +       \
     ((A)[(y) + 1][x] + (A)[(y)-1][x] - 2.0 * (A)[y][x]) * p.ihy2)

// ---------------------------------------------------------------------------
// 2-D tile stencils (M = 1, periodic), for grids too small to give the sliding sweeps enough
// waves: a 64x16 output tile is staged in LDS with a three-cell halo and the composite
// operator applied as three successive five-point Laplacians inside LDS (halo 3 -> 2 -> 1 -> 0).
// ---------------------------------------------------------------------------

// F = (Phi - phi)/dt - Delta_d mu_d - src, plus one partial sum of F^2 per block (and of
// Phi^2 in xpart when given).
// Persistent blocks walk their tiles; the halo of the next tile is loaded into registers
// while the current one is computed from LDS.
__global__ __launch_bounds__(NT) void k_residual2d_tile(const double* __restrict__ Phi,
                                                   const double* __restrict__ phi,
                                                   const double* __restrict__ src,
                                                   double* __restrict__ F,
                                                   double* __restrict__ part, double* __restrict__ xpart, P p) {
    __shared__ double su[TY + 6][TX + 6];     // u = (Phi + phi)/2, halo 3
    __shared__ double sl[TY + 4][TX + 4];     // Delta_d u, halo 2
    __shared__ double sm[TY + 2][TX + 2];     // cubic term q, then mu_d, halo 1
    __shared__ double red[NT / 64];
    const int ntx = (p.nx + TX - 1) / TX, nty = (p.ny + TY - 1) / TY;
    const TileRange tr = tile_range(ntx * nty);
    const int tid = threadIdx.x;
    const bool big = p.nx >= TX + 6 && p.ny >= TY + 6;   // one wrap step suffices
    double ra[NIT3], rb[NIT3];
    auto load = [&](int tile) {
        const int x0 = (tile % ntx) * TX, y0 = (tile / ntx) * TY;
#pragma unroll
        for (int k = 0; k < NIT3; ++k) {
            const int e = tid + k * NT;
            if (e < NE3) {
                const int ly = e / (TX + 6), lx = e - ly * (TX + 6);
                const int gy = big ? wrap1(y0 + ly - 3, p.ny) : wrap(y0 + ly - 3, p.ny);
                const int gx = big ? wrap1(x0 + lx - 3, p.nx) : wrap(x0 + lx - 3, p.nx);
                const long gi = (long)gy * p.nx + gx;
                ra[k] = Phi[gi];
                rb[k] = phi[gi];
            }
        }
    };
    double acc = 0.0, accx = 0.0;
    if (tr.first < tr.last) load(tr.first);
    for (int tile = tr.first; tile < tr.last; ++tile) {
        const int x0 = (tile % ntx) * TX, y0 = (tile / ntx) * TY;
        __syncthreads();                      // the previous tile is done with the LDS arrays
#pragma unroll
        for (int k = 0; k < NIT3; ++k) {
            const int e = tid + k * NT;
            if (e < NE3) {
                const int ly = e / (TX + 6), lx = e - ly * (TX + 6);
                const double a = ra[k], b = rb[k];
                su[ly][lx] = 0.5 * (a + b);
                const int qy = ly - 2, qx = lx - 2;
                if (qy >= 0 && qy < TY + 2 && qx >= 0 && qx < TX + 2)
                    sm[qy][qx] = 0.25 * (a * a * a + a * a * b + a * b * b + b * b * b);
            }
        }
        if (tile + 1 < tr.last) load(tile + 1);   // in flight during the passes below
        __syncthreads();
        for (int e = tid; e < (TY + 4) * (TX + 4); e += NT) {
            const int ly = e / (TX + 4), lx = e - ly * (TX + 4);
            sl[ly][lx] = LAP2(su, ly + 1, lx + 1);
        }
        __syncthreads();
        for (int e = tid; e < (TY + 2) * (TX + 2); e += NT) {
            const int ly = e / (TX + 2), lx = e - ly * (TX + 2);
            const double l = sl[ly + 1][lx + 1];
            sm[ly][lx] += (1.0 - p.gamma) * su[ly + 2][lx + 2] + 2.0 * l + LAP2(sl, ly + 1, lx + 1);
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < NIT0; ++k) {
            const int e = tid + k * NT;
            const int ly = e / TX, lx = e - ly * TX;
            const int gx = x0 + lx, gy = y0 + ly;
            if (e < TY * TX && gx < p.nx && gy < p.ny) {
                const long gi = (long)gy * p.nx + gx;
                const double a = Phi[gi];             // re-read: in L2
                double f = (a - phi[gi]) * p.inv_dt - LAP2(sm, ly + 1, lx + 1);
                if (src) f -= src[gi];
                F[gi] = f;
                acc += f * f;
                accx += a * a;
            }
        }
    }
    if (part) {
        const double s = block_sum_det(acc, red);
        if (tid == 0) part[blockIdx.x] = s;
    }
    if (xpart) {
        const double s = block_sum_det(accx, red);
        if (tid == 0) xpart[blockIdx.x] = s;
    }
}

// Jv = v/dt - Delta_d[(1-gamma)/2 v + Delta_d v + 1/2 Delta_d^2 v + c v] with v shifted by
// -s, s = shift_scale * sum(shift_part[0..shift_n)) when shift_part is given (zero-mean
// projection fused into the load; every block forms s in the same order and block 0
// stores it in *shift_out).
__global__ __launch_bounds__(NT) void k_jv2d_tile(const double* __restrict__ v,
                                             const double* __restrict__ cc,
                                             const double* __restrict__ shift_part, int shift_n,
                                             double shift_scale, double* __restrict__ shift_out,
                                             double* __restrict__ Jv, P p) {
    __shared__ double sv[TY + 6][TX + 6];
    __shared__ double sl[TY + 4][TX + 4];
    __shared__ double sn[TY + 2][TX + 2];     // c, then the inner operator, halo 1
    __shared__ double red[NT / 64];
    const int ntx = (p.nx + TX - 1) / TX;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int x0 = (tile % ntx) * TX, y0 = (tile / ntx) * TY, tid = threadIdx.x;
    double sh = 0.0;
    if (shift_part) {
        sh = shift_scale * sum_partials_bcast(shift_part, shift_n, red);
        if (shift_out && tid == 0 && blockIdx.x == 0) *shift_out = sh;
    }
    const bool big = p.nx >= TX + 6 && p.ny >= TY + 6;

    double rv[NIT3], rc[NIT3];
#pragma unroll
    for (int k = 0; k < NIT3; ++k) {
        const int e = tid + k * NT;
        if (e < NE3) {
            const int ly = e / (TX + 6), lx = e - ly * (TX + 6);
            const int gy = big ? wrap1(y0 + ly - 3, p.ny) : wrap(y0 + ly - 3, p.ny);
            const int gx = big ? wrap1(x0 + lx - 3, p.nx) : wrap(x0 + lx - 3, p.nx);
            const long gi = (long)gy * p.nx + gx;
            rv[k] = v[gi];
            const int qy = ly - 2, qx = lx - 2;
            rc[k] = (qy >= 0 && qy < TY + 2 && qx >= 0 && qx < TX + 2) ? cc[gi] : 0.0;
        }
    }
#pragma unroll
    for (int k = 0; k < NIT3; ++k) {
        const int e = tid + k * NT;
        if (e < NE3) {
            const int ly = e / (TX + 6), lx = e - ly * (TX + 6);
            sv[ly][lx] = rv[k] - sh;
            const int qy = ly - 2, qx = lx - 2;
            if (qy >= 0 && qy < TY + 2 && qx >= 0 && qx < TX + 2) sn[qy][qx] = rc[k];
        }
    }
    __syncthreads();
    for (int e = tid; e < (TY + 4) * (TX + 4); e += NT) {
        const int ly = e / (TX + 4), lx = e - ly * (TX + 4);
        sl[ly][lx] = LAP2(sv, ly + 1, lx + 1);
    }
    __syncthreads();
    for (int e = tid; e < (TY + 2) * (TX + 2); e += NT) {
        const int ly = e / (TX + 2), lx = e - ly * (TX + 2);
        const double vv = sv[ly + 2][lx + 2];
        sn[ly][lx] = 0.5 * (1.0 - p.gamma) * vv + sl[ly + 1][lx + 1] +
                     0.5 * LAP2(sl, ly + 1, lx + 1) + sn[ly][lx] * vv;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NIT0; ++k) {
        const int e = tid + k * NT;
        const int ly = e / TX, lx = e - ly * TX;
        const int gx = x0 + lx, gy = y0 + ly;
        if (e < TY * TX && gx < p.nx && gy < p.ny)
            Jv[(long)gy * p.nx + gx] = sv[ly + 3][lx + 3] * p.inv_dt - LAP2(sn, ly + 1, lx + 1);
    }
}

// Partial sums of G_d (Eq. (7)) and of phi per block: part[b] and part[nblk + b].
// With acc_phi (accepting a step): every cell also moves acc_phi -> acc_prev and phi -> acc_phi
// (phi^(n-1) <- phi^n, phi^n <- phi), the copies done in the same pass.
__global__ __launch_bounds__(NT) void k_energy2d(const double* __restrict__ phi,
                                                 double* __restrict__ part, P p, double* __restrict__ acc_phi,
                                                 double* __restrict__ acc_prev) {
    __shared__ double s[TY + 2][TX + 2];
    __shared__ double red[NT / 64];
    const int ntx = (p.nx + TX - 1) / TX;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int x0 = (tile % ntx) * TX, y0 = (tile / ntx) * TY, tid = threadIdx.x;
    for (int e = tid; e < (TY + 2) * (TX + 2); e += NT) {
        const int ly = e / (TX + 2), lx = e - ly * (TX + 2);
        s[ly][lx] = phi[(long)wrap(y0 + ly - 1, p.ny) * p.nx + wrap(x0 + lx - 1, p.nx)];
    }
    __syncthreads();
    double eg = 0.0, em = 0.0;
    for (int e = tid; e < TY * TX; e += NT) {
        const int ly = e / TX + 1, lx = e % TX + 1;
        if (x0 + lx - 1 < p.nx && y0 + ly - 1 < p.ny) {
            const double f = s[ly][lx];
            const double xp = s[ly][lx + 1] - f, xm = f - s[ly][lx - 1];
            const double yp = s[ly + 1][lx] - f, ym = f - s[ly - 1][lx];
            const double lap = (xp - xm) * p.ihx2 + (yp - ym) * p.ihy2;
            eg += 0.5 * (1.0 - p.gamma) * f * f + 0.25 * f * f * f * f + 0.5 * lap * lap -
                  0.5 * ((xp * xp + xm * xm) * p.ihx2 + (yp * yp + ym * ym) * p.ihy2);
            em += f;
            if (acc_phi) {
                const long q = (long)(y0 + ly - 1) * p.nx + (x0 + lx - 1);
                acc_prev[q] = acc_phi[q];
                acc_phi[q] = f;
            }
        }
    }
    const int nb = gridDim.x, b = blockIdx.x;
    const double sg = block_sum_det(eg, red);
    if (tid == 0) part[b] = sg;
    const double sm = block_sum_det(em, red);
    if (tid == 0) part[nb + b] = sm;
}

// ---------------------------------------------------------------------------
// Generic N-d multi-pass kernels (3-D; also valid for 2-D with nz = 1)
// ---------------------------------------------------------------------------

// Neighbour index i + 1 / i - 1 along an axis of n cells: periodic wrap, or the mirror ghost
// (the cell itself) of the Neumann-type boundaries.
__device__ __forceinline__ int nxt(int i, int n, int neu) { return i + 1 < n ? i + 1 : (neu ? i : 0); }
__device__ __forceinline__ int prv(int i, int n, int neu) { return i > 0 ? i - 1 : (neu ? i : n - 1); }

__device__ __forceinline__ double lap7(const double* __restrict__ a, int x, int y, int z, const P& p) {
    const long sxy = (long)p.nx * p.ny;
    const long c = z * sxy + (long)y * p.nx + x;
    const double ac = a[c];
    const int xp = nxt(x, p.nx, p.neu), xm = prv(x, p.nx, p.neu);
    const int yp = nxt(y, p.ny, p.neu), ym = prv(y, p.ny, p.neu);
    const long row = z * sxy + (long)y * p.nx;
    double r = (a[row + xp] + a[row + xm] - 2.0 * ac) * p.ihx2 +
               (a[z * sxy + (long)yp * p.nx + x] + a[z * sxy + (long)ym * p.nx + x] - 2.0 * ac) * p.ihy2;
    if (p.nz > 1) {
        const int zp = nxt(z, p.nz, p.neu), zm = prv(z, p.nz, p.neu);
        r += (a[zp * sxy + (long)y * p.nx + x] + a[zm * sxy + (long)y * p.nx + x] - 2.0 * ac) * p.ihz2;
    }
    return r;
}

// nabla_d . M nabla_d g at cell (x, y, z) with the face mobility the mean of the node values
// (Sec. 3); node mobilities from mfun(i).  A Neumann face has a zero difference, so no flux.
template <typename MF>
__device__ __forceinline__ double div_m_grad(const double* __restrict__ g, MF mfun, int x, int y, int z, const P& p) {
    const long sxy = (long)p.nx * p.ny;
    const long c = z * sxy + (long)y * p.nx + x;
    const double gc = g[c], mc = mfun(c);
    auto face = [&](long j) { return 0.5 * (mc + mfun(j)) * (g[j] - gc); };
    const long row = z * sxy + (long)y * p.nx;
    double r = (face(row + nxt(x, p.nx, p.neu)) + face(row + prv(x, p.nx, p.neu))) * p.ihx2 +
               (face(z * sxy + (long)nxt(y, p.ny, p.neu) * p.nx + x) + face(z * sxy + (long)prv(y, p.ny, p.neu) * p.nx + x)) *
                   p.ihy2;
    if (p.nz > 1)
        r += (face(nxt(z, p.nz, p.neu) * sxy + (long)y * p.nx + x) + face(prv(z, p.nz, p.neu) * sxy + (long)y * p.nx + x)) *
             p.ihz2;
    return r;
}

#define MP_INDEX                                                         \
    const int x = blockIdx.x * blockDim.x + threadIdx.x;                 \
    const int y = blockIdx.y * blockDim.y + threadIdx.y;                 \
    const int z = blockIdx.z;                                            \
    if (x >= p.nx || y >= p.ny) return;                                  \
    const long i = ((long)z * p.ny + y) * p.nx + x;

// out = (a + b)/2 (mode 0) or a - s (mode 1), s = shift_scale * sum(shift_part[0..shift_n))
// (s = 0 without shift_part; block 0 stores s in *shift_out).  Elementwise: out may be a.
__global__ __launch_bounds__(256) void k_mp_combine(const double* a, const double* __restrict__ b,
                                                    const double* __restrict__ shift_part, int shift_n,
                                                    double shift_scale, double* __restrict__ shift_out, int mode,
                                                    double* out, long n) {
    __shared__ double red[4];
    double sh = 0.0;
    if (shift_part) {
        sh = shift_scale * sum_partials_bcast(shift_part, shift_n, red);
        if (shift_out && threadIdx.x == 0 && blockIdx.x == 0) *shift_out = sh;
    }
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        out[i] = mode == 0 ? 0.5 * (a[i] + b[i]) : a[i] - sh;
}

__global__ void k_mp_lap(const double* __restrict__ u, double* __restrict__ out, P p) {
    MP_INDEX
    out[i] = lap7(u, x, y, z, p);
}

// mu = (1-gamma) u + 2 Lu + Delta Lu + q (residual) or inner Jacobian operator (jv).  u is read
// at the cell itself only, so out may be u (updated in place).
__global__ void k_mp_inner(const double* __restrict__ Phi, const double* __restrict__ phi,
                           const double* u, const double* __restrict__ Lu,
                           const double* __restrict__ cc, int jv, double* out, P p) {
    MP_INDEX
    const double l = Lu[i];
    const double ll = lap7(Lu, x, y, z, p);
    if (!jv) {
        const double a = Phi[i], b = phi[i];
        out[i] = (1.0 - p.gamma) * u[i] + 2.0 * l + ll + 0.25 * (a * a * a + a * a * b + a * b * b + b * b * b);
    } else {
        const double vv = u[i];
        out[i] = 0.5 * (1.0 - p.gamma) * vv + l + 0.5 * ll + cc[i] * vv;
    }
}

// residual (jv = 0): F = (Phi - phi)/dt - Delta mu - src ; jv: out = v/dt - Delta inner.  a is
// read at the cell itself only, so out may be a (updated in place).
__global__ void k_mp_final(const double* a, const double* __restrict__ b,
                           const double* __restrict__ m, const double* __restrict__ src, int jv,
                           double* out, P p) {
    MP_INDEX
    const double lm = lap7(m, x, y, z, p);
    double f = (jv ? a[i] : a[i] - b[i]) * p.inv_dt - lm;
    if (src) f -= src[i];
    out[i] = f;
}

// ---------------------------------------------------------------------------
// 3-D fused stencils (M = 1, periodic): a block owns a T3X x T3Y column of cells and marches
// it through a segment of z-planes.  Each plane entering (with a three-cell halo in x and y)
// is staged in LDS; the three radius-1 stages of the composite operator follow it one plane
// behind each other, each stage keeping the last three planes it produced in an LDS ring
// (the z-neighbours), so every field is read from HBM once per column (plus its x-y halo
// and the three planes above and below a segment) and the result written once, in one
// launch instead of four passes through memory.  Each plane's loads are issued into
// registers two planes ahead, so the stages of the two planes before it cover their latency.
// ---------------------------------------------------------------------------

constexpr int T3X = 32, T3Y = 8;
constexpr int H3N = (T3X + 6) * (T3Y + 6);   // halo-3 plane
constexpr int H2N = (T3X + 4) * (T3Y + 4);   // halo-2
constexpr int H1N = (T3X + 2) * (T3Y + 2);   // halo-1
constexpr int H0N = T3X * T3Y;               // the column's own cells
constexpr int DR3 = 5;                       // ring of own-cell planes (read 3 planes after its load)
constexpr int PF3 = (H3N + NT - 1) / NT;      // halo-3 cells per thread of a plane

struct Geom3 {
    int ntx, nty, zseg, nseg, items;
};

__host__ __device__ inline Geom3 geom3(int nx, int ny, int nz) {
    Geom3 g;
    g.ntx = (nx + T3X - 1) / T3X;
    g.nty = (ny + T3Y - 1) / T3Y;
    // segments as short as gives ~768 items (three resident blocks on each of 256 CUs, as
    // LDS allows), so that the items run in one round, but at least 8 planes (6 warm-up planes)
    const int cols = g.ntx * g.nty;
    const int want = max(1, 768 / cols);
    g.zseg = max(8, (nz + want - 1) / want);
    g.nseg = (nz + g.zseg - 1) / g.zseg;
    g.items = cols * g.nseg;
    return g;
}

// In-plane offsets of the halo-3 cells that this thread stages for the column at (x0, y0):
// cell tid + NT r of the (T3X + 6) x (T3Y + 6) plane, wrapped periodically; slots past the
// plane's last cell take that cell's offset (loaded, never stored).
__device__ __forceinline__ void halo3_offsets(int (&go)[PF3], int x0, int y0, const P& p) {
#pragma unroll
    for (int r = 0; r < PF3; ++r) {
        const int e = min((int)threadIdx.x + NT * r, H3N - 1);
        const int i = e % (T3X + 6), j = e / (T3X + 6);
        go[r] = wrap(y0 - 3 + j, p.ny) * p.nx + wrap(x0 - 3 + i, p.nx);
    }
}

// five-point x-y Laplacian of plane a (width w) at (i, j), plus the z term from planes zm, zp
__device__ __forceinline__ double lap3(const double* a, const double* zm, const double* zp, int w, int i, int j,
                                       const P& p) {
    const int c = j * w + i;
    const double ac = a[c];
    return (a[c + 1] + a[c - 1] - 2.0 * ac) * p.ihx2 + (a[c + w] + a[c - w] - 2.0 * ac) * p.ihy2 +
           (zm[c] + zp[c] - 2.0 * ac) * p.ihz2;
}

// F = (Phi - phi)/dt - Delta_d mu_d - src with per-block partial sums of F^2 (and Phi^2).
__global__ __launch_bounds__(NT) void k_residual3d(const double* __restrict__ Phi, const double* __restrict__ phi,
                                                   const double* __restrict__ src, double* __restrict__ F,
                                                   double* __restrict__ part, double* __restrict__ xpart, P p) {
    __shared__ double U[3][H3N];   // u = (Phi + phi)/2, halo 3
    __shared__ double Q[3][H1N];   // the cubic term, halo 1
    __shared__ double L[3][H2N];   // Delta_d u, halo 2
    __shared__ double M[3][H1N];   // mu_d, halo 1
    __shared__ double D[DR3][H0N]; // Phi - phi, own cells
    __shared__ double red[NT / 64];
    const Geom3 G = geom3(p.nx, p.ny, p.nz);
    const long sxy = (long)p.nx * p.ny;
    const int tid = threadIdx.x;
    double acc = 0.0, accx = 0.0;
    for (int ib = blockIdx.x; ib < G.items; ib += gridDim.x) {
        const int it = xcd_item(ib, G.items);
        const int col = it % (G.ntx * G.nty), sg = it / (G.ntx * G.nty);
        const int x0 = (col % G.ntx) * T3X, y0 = (col / G.ntx) * T3Y;
        const int z0 = sg * G.zseg, z1 = min(z0 + G.zseg, p.nz);
        const int nk = z1 - z0 + 6;
        int go[PF3];   // in-plane offsets of this thread's halo-3 cells
        halo3_offsets(go, x0, y0, p);
        // Three sets of slots, plane k in set k mod 3, loaded two planes ahead into the set whose
        // plane has just been consumed: no copy and no early wait follows a load, and two planes
        // of stage work cover its latency.  Past the segment's last plane that plane is loaded
        // again (in bounds, from the cache).
        auto fetch = [&](int k, double (&A)[PF3], double (&B)[PF3]) {
            const long zoff = (long)wrap(z0 - 3 + min(k, nk - 1), p.nz) * sxy;
#pragma unroll
            for (int r = 0; r < PF3; ++r) {
                A[r] = Phi[zoff + go[r]];
                B[r] = phi[zoff + go[r]];
            }
        };
        auto step = [&](int k, const double (&A)[PF3], const double (&B)[PF3], double (&NA)[PF3],
                        double (&NB)[PF3]) {
            const int zin = z0 - 3 + k;
            // A: plane zin enters (from the registers), and plane zin + 2's loads go out
#pragma unroll
            for (int r = 0; r < PF3; ++r) {
                const int e = tid + NT * r;
                if (e >= H3N) break;
                const int i = e % (T3X + 6), j = e / (T3X + 6);
                const double a = A[r], b = B[r];
                U[k % 3][e] = 0.5 * (a + b);
                if (i >= 2 && i < T3X + 4 && j >= 2 && j < T3Y + 4)
                    Q[k % 3][(j - 2) * (T3X + 2) + i - 2] = 0.25 * (a * a * a + a * a * b + a * b * b + b * b * b);
                if (i >= 3 && i < T3X + 3 && j >= 3 && j < T3Y + 3) {
                    D[k % DR3][(j - 3) * T3X + i - 3] = a - b;
                    if (xpart && zin >= z0 && zin < z1 && x0 + i - 3 < p.nx && y0 + j - 3 < p.ny) accx += a * a;
                }
            }
            fetch(k + 2, NA, NB);
            __syncthreads();
            // B: Lu at plane zin - 1 (halo 2)
            if (k >= 2)
                for (int e = tid; e < H2N; e += NT) {
                    const int i = e % (T3X + 4), j = e / (T3X + 4);
                    L[(k - 1) % 3][e] = lap3(U[(k - 1) % 3], U[(k - 2) % 3], U[k % 3], T3X + 6, i + 1, j + 1, p);
                }
            __syncthreads();
            // C: mu at plane zin - 2 (halo 1)
            if (k >= 4)
                for (int e = tid; e < H1N; e += NT) {
                    const int i = e % (T3X + 2), j = e / (T3X + 2);
                    const int c2 = (j + 1) * (T3X + 4) + i + 1;
                    const double l = L[(k - 2) % 3][c2];
                    const double ll = lap3(L[(k - 2) % 3], L[(k - 3) % 3], L[(k - 1) % 3], T3X + 4, i + 1, j + 1, p);
                    M[(k - 2) % 3][e] = (1.0 - p.gamma) * U[(k - 2) % 3][(j + 2) * (T3X + 6) + i + 2] + 2.0 * l + ll +
                                        Q[(k - 2) % 3][e];
                }
            __syncthreads();
            // D: F at plane zin - 3 (own cells)
            if (k >= 6)
                for (int e = tid; e < H0N; e += NT) {
                    const int i = e % T3X, j = e / T3X;
                    const int x = x0 + i, y = y0 + j;
                    if (x >= p.nx || y >= p.ny) continue;
                    const double lm = lap3(M[(k - 3) % 3], M[(k - 4) % 3], M[(k - 2) % 3], T3X + 2, i + 1, j + 1, p);
                    const long gi = (long)(zin - 3) * sxy + (long)y * p.nx + x;
                    double f = D[(k - 3) % DR3][e] * p.inv_dt - lm;
                    if (src) f -= src[gi];
                    F[gi] = f;
                    acc += f * f;
                }
        };
        double s0a[PF3], s0b[PF3], s1a[PF3], s1b[PF3], s2a[PF3], s2b[PF3];
        fetch(0, s0a, s0b);
        fetch(1, s1a, s1b);
        __syncthreads();   // the previous item's last reads of the rings
        for (int k0 = 0; k0 < nk; k0 += 3) {
            step(k0, s0a, s0b, s2a, s2b);
            if (k0 + 1 >= nk) break;
            step(k0 + 1, s1a, s1b, s0a, s0b);
            if (k0 + 2 >= nk) break;
            step(k0 + 2, s2a, s2b, s1a, s1b);
        }
    }
    if (part) {
        const double t = block_sum_det(acc, red);
        if (threadIdx.x == 0) part[blockIdx.x] = t;
    }
    if (xpart) {
        const double t = block_sum_det(accx, red);
        if (threadIdx.x == 0) xpart[blockIdx.x] = t;
    }
}

// Jv = v/dt - Delta_d[(1-gamma)/2 v + Delta_d v + 1/2 Delta_d^2 v + c v] with v shifted by -s
// (s as in k_jv2d: from shift_part, every block in the same order, block 0 stores it).
__global__ __launch_bounds__(NT) void k_jv3d(const double* __restrict__ v, const double* __restrict__ cc,
                                             const double* __restrict__ shift_part, int shift_n, double shift_scale,
                                             double* __restrict__ shift_out, double* __restrict__ Jv, P p) {
    __shared__ double V[3][H3N];   // v - s, halo 3
    __shared__ double C[3][H1N];   // c, halo 1
    __shared__ double L[3][H2N];   // Delta_d v, halo 2
    __shared__ double Wr[3][H1N];  // the inner operator, halo 1
    __shared__ double D[DR3][H0N]; // v - s, own cells
    __shared__ double red[NT / 64];
    double sh = 0.0;
    if (shift_part) {
        sh = shift_scale * sum_partials_bcast(shift_part, shift_n, red);
        if (shift_out && threadIdx.x == 0 && blockIdx.x == 0) *shift_out = sh;
    }
    const Geom3 G = geom3(p.nx, p.ny, p.nz);
    const long sxy = (long)p.nx * p.ny;
    const int tid = threadIdx.x;
    for (int ib = blockIdx.x; ib < G.items; ib += gridDim.x) {
        const int it = xcd_item(ib, G.items);
        const int col = it % (G.ntx * G.nty), sg = it / (G.ntx * G.nty);
        const int x0 = (col % G.ntx) * T3X, y0 = (col / G.ntx) * T3Y;
        const int z0 = sg * G.zseg, z1 = min(z0 + G.zseg, p.nz);
        const int nk = z1 - z0 + 6;
        int go[PF3];
        halo3_offsets(go, x0, y0, p);
        // three sets of slots loaded two planes ahead, as in k_residual3d
        auto fetch = [&](int k, double (&A)[PF3], double (&B)[PF3]) {
            const long zoff = (long)wrap(z0 - 3 + min(k, nk - 1), p.nz) * sxy;
#pragma unroll
            for (int r = 0; r < PF3; ++r) {
                A[r] = v[zoff + go[r]];
                B[r] = cc[zoff + go[r]];
            }
        };
        auto step = [&](int k, const double (&A)[PF3], const double (&B)[PF3], double (&NA)[PF3],
                        double (&NB)[PF3]) {
            const int zin = z0 - 3 + k;
#pragma unroll
            for (int r = 0; r < PF3; ++r) {
                const int e = tid + NT * r;
                if (e >= H3N) break;
                const int i = e % (T3X + 6), j = e / (T3X + 6);
                const double a = A[r] - sh;
                V[k % 3][e] = a;
                if (i >= 2 && i < T3X + 4 && j >= 2 && j < T3Y + 4) C[k % 3][(j - 2) * (T3X + 2) + i - 2] = B[r];
                if (i >= 3 && i < T3X + 3 && j >= 3 && j < T3Y + 3) D[k % DR3][(j - 3) * T3X + i - 3] = a;
            }
            fetch(k + 2, NA, NB);
            __syncthreads();
            if (k >= 2)
                for (int e = tid; e < H2N; e += NT) {
                    const int i = e % (T3X + 4), j = e / (T3X + 4);
                    L[(k - 1) % 3][e] = lap3(V[(k - 1) % 3], V[(k - 2) % 3], V[k % 3], T3X + 6, i + 1, j + 1, p);
                }
            __syncthreads();
            if (k >= 4)
                for (int e = tid; e < H1N; e += NT) {
                    const int i = e % (T3X + 2), j = e / (T3X + 2);
                    const double l = L[(k - 2) % 3][(j + 1) * (T3X + 4) + i + 1];
                    const double ll = lap3(L[(k - 2) % 3], L[(k - 3) % 3], L[(k - 1) % 3], T3X + 4, i + 1, j + 1, p);
                    const double vv = V[(k - 2) % 3][(j + 2) * (T3X + 6) + i + 2];
                    Wr[(k - 2) % 3][e] = 0.5 * (1.0 - p.gamma) * vv + l + 0.5 * ll + C[(k - 2) % 3][e] * vv;
                }
            __syncthreads();
            if (k >= 6)
                for (int e = tid; e < H0N; e += NT) {
                    const int i = e % T3X, j = e / T3X;
                    const int x = x0 + i, y = y0 + j;
                    if (x >= p.nx || y >= p.ny) continue;
                    const double lw = lap3(Wr[(k - 3) % 3], Wr[(k - 4) % 3], Wr[(k - 2) % 3], T3X + 2, i + 1, j + 1, p);
                    Jv[(long)(zin - 3) * sxy + (long)y * p.nx + x] = D[(k - 3) % DR3][e] * p.inv_dt - lw;
                }
        };
        double s0a[PF3], s0b[PF3], s1a[PF3], s1b[PF3], s2a[PF3], s2b[PF3];
        fetch(0, s0a, s0b);
        fetch(1, s1a, s1b);
        __syncthreads();
        for (int k0 = 0; k0 < nk; k0 += 3) {
            step(k0, s0a, s0b, s2a, s2b);
            if (k0 + 1 >= nk) break;
            step(k0 + 1, s1a, s1b, s0a, s0b);
            if (k0 + 2 >= nk) break;
            step(k0 + 2, s2a, s2b, s1a, s1b);
        }
    }
}

// The last pass with the variable mobility M(u) = 1 - u^2.  Residual (jv = 0, a = Phi, b = phi,
// m = mu): F = (Phi - phi)/dt - nabla . M nabla mu - src, u = (Phi + phi)/2 at each node.
// Jacobian action (jv = 1, a = v, m = the inner operator w, u and mu of the iterate given):
// out = v/dt - nabla . M nabla w - nabla . (M'(u) v / 2) nabla mu, M'(u) v / 2 = -u v.
// a is read at the cell itself only, so out may be a.
__global__ void k_mp_final_mob(const double* a, const double* __restrict__ b, const double* __restrict__ m,
                               const double* __restrict__ src, int jv, const double* __restrict__ u,
                               const double* __restrict__ mu, double* out, P p) {
    MP_INDEX
    if (!jv) {
        auto mob = [&](long j) {
            const double uj = 0.5 * (a[j] + b[j]);
            return 1.0 - uj * uj;
        };
        double f = (a[i] - b[i]) * p.inv_dt - div_m_grad(m, mob, x, y, z, p);
        if (src) f -= src[i];
        out[i] = f;
    } else {
        auto mob = [&](long j) { return 1.0 - u[j] * u[j]; };
        auto dmob = [&](long j) { return -u[j] * a[j]; };
        const double t1 = div_m_grad(m, mob, x, y, z, p);
        const double t2 = div_m_grad(mu, dmob, x, y, z, p);
        out[i] = a[i] * p.inv_dt - t1 - t2;
    }
}

__global__ __launch_bounds__(NT) void k_mp_energy(const double* __restrict__ phi,
                                                  double* __restrict__ part, P p) {
    __shared__ double red[NT / 64];
    const long n = (long)p.nx * p.ny * p.nz;
    const long sxy = (long)p.nx * p.ny;
    double eg = 0.0, em = 0.0;
    for (long i = blockIdx.x * (long)NT + threadIdx.x; i < n; i += (long)gridDim.x * NT) {
        const int x = (int)(i % p.nx), y = (int)((i / p.nx) % p.ny), z = (int)(i / sxy);
        const double f = phi[i];
        const int xp = nxt(x, p.nx, p.neu), xm = prv(x, p.nx, p.neu);
        const int yp = nxt(y, p.ny, p.neu), ym = prv(y, p.ny, p.neu);
        const double dxp = phi[z * sxy + (long)y * p.nx + xp] - f, dxm = f - phi[z * sxy + (long)y * p.nx + xm];
        const double dyp = phi[z * sxy + (long)yp * p.nx + x] - f, dym = f - phi[z * sxy + (long)ym * p.nx + x];
        double lap = (dxp - dxm) * p.ihx2 + (dyp - dym) * p.ihy2;
        double grad = (dxp * dxp + dxm * dxm) * p.ihx2 + (dyp * dyp + dym * dym) * p.ihy2;
        if (p.nz > 1) {
            const int zp = nxt(z, p.nz, p.neu), zm = prv(z, p.nz, p.neu);
            const double dzp = phi[zp * sxy + (long)y * p.nx + x] - f, dzm = f - phi[zm * sxy + (long)y * p.nx + x];
            lap += (dzp - dzm) * p.ihz2;
            grad += (dzp * dzp + dzm * dzm) * p.ihz2;
        }
        eg += 0.5 * (1.0 - p.gamma) * f * f + 0.25 * f * f * f * f + 0.5 * lap * lap - 0.5 * grad;
        em += f;
    }
    const double sg = block_sum_det(eg, red);
    if (threadIdx.x == 0) part[blockIdx.x] = sg;
    const double sm = block_sum_det(em, red);
    if (threadIdx.x == 0) part[gridDim.x + blockIdx.x] = sm;
}

__global__ __launch_bounds__(NT) void k_sumsq(const double* __restrict__ x, long n,
                                              double* __restrict__ part) {
    __shared__ double red[NT / 64];
    double acc = 0.0;
    for (long i = blockIdx.x * (long)NT + threadIdx.x; i < n; i += (long)gridDim.x * NT) acc += x[i] * x[i];
    const double s = block_sum_det(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void k_coef(const double* __restrict__ Phi, const double* __restrict__ phi,
                       double* __restrict__ c, long n) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const double a = Phi[i], b = phi[i];
        c[i] = 0.25 * (3.0 * a * a + 2.0 * a * b + b * b);
    }
}

P make_params(const pfc_ctx* c, double dt) {
    P p;
    p.nx = c->g.nx;
    p.ny = c->g.ny;
    p.nz = c->g.nz;
    p.ihx2 = c->g.ihx2;
    p.ihy2 = c->g.ihy2;
    p.ihz2 = c->g.ihz2;
    p.gamma = c->model.gamma;
    p.inv_dt = dt > 0 ? 1.0 / dt : 0.0;
    p.neu = c->model.boundary == PFC_BC_NEUMANN;
    p.mob = c->model.mobility == PFC_MOBILITY_1_MINUS_SQ;
    return p;
}

dim3 tiles2d(const pfc_ctx* c) { return dim3(((c->g.nx + TX - 1) / TX) * ((c->g.ny + TY - 1) / TY)); }
inline bool sliding(int nx, int ny) { return (long)nx * ny >= SW_MIN_CELLS; }
// grid of the 2-D residual and Jacobian action, at most 1024 blocks: one wave per (strip,
// segment) item of the sliding sweeps, or persistent blocks over the tiles (four resident
// blocks per CU, LDS-limited, on 256 CUs)
inline unsigned grid2d(int nx, int ny) {
    const long b = sliding(nx, ny) ? ((long)sw_geom(nx, ny).items + NT / 64 - 1) / (NT / 64)
                                   : (long)((nx + TX - 1) / TX) * ((ny + TY - 1) / TY);
    return (unsigned)(b < 1024 ? b : 1024);
}
inline unsigned grid3d(int nx, int ny, int nz) {
    const int b = geom3(nx, ny, nz).items;
    return (unsigned)(b < 1024 ? b : 1024);
}
dim3 residual_grid(const pfc_ctx* c) {
    return dim3(c->g.dim == 3 ? grid3d(c->g.nx, c->g.ny, c->g.nz) : grid2d(c->g.nx, c->g.ny));
}
dim3 mp_grid(const pfc_ctx* c) { return dim3((c->g.nx + 63) / 64, (c->g.ny + 3) / 4, c->g.nz); }

}  // namespace

bool fused2d(const pfc_ctx* c) {
    return c->g.dim == 2 && c->model.mobility == PFC_MOBILITY_1 && c->model.boundary == PFC_BC_PERIODIC;
}

bool fused3d(const pfc_ctx* c) {
    return c->g.dim == 3 && c->model.mobility == PFC_MOBILITY_1 && c->model.boundary == PFC_BC_PERIODIC;
}

int residual_partial_count(const pfc_ctx* c) {
    return fused2d(c) || fused3d(c) ? (int)residual_grid(c).x : kRedBlocks;
}

int energy_partial_count(const pfc_ctx* c) { return fused2d(c) ? (int)tiles2d(c).x : kRedBlocks; }

hipError_t launch_residual(const pfc_ctx* c, const double* Phi, const double* phi, double dt,
                           const double* src, double* F, double* norm_part, double* xnorm_part) {
    const P p = make_params(c, dt);
    if (fused2d(c)) {
        return sliding(c->g.nx, c->g.ny)
                   ? launch_k(c, k_residual2d, residual_grid(c), dim3(NT), 0, Phi, phi, src, F, norm_part, xnorm_part, p)
                   : launch_k(c, k_residual2d_tile, residual_grid(c), dim3(NT), 0, Phi, phi, src, F, norm_part,
                              xnorm_part, p);
    }
    if (fused3d(c))
        return launch_k(c, k_residual3d, residual_grid(c), dim3(NT), 0, Phi, phi, src, F, norm_part, xnorm_part, p);
    if (xnorm_part) hipLaunchKernelGGL(k_sumsq, dim3(kRedBlocks), dim3(NT), 0, c->stream, Phi, c->g.N, xnorm_part);
    double* u = c->d_tmp3;
    double* Lu = c->d_tmp3 + c->g.N;
    hipLaunchKernelGGL(k_mp_combine, dim3(2048), dim3(256), 0, c->stream, Phi, phi, nullptr, 0, 0.0, nullptr, 0, u,
                       c->g.N);
    hipLaunchKernelGGL(k_mp_lap, mp_grid(c), dim3(64, 4), 0, c->stream, u, Lu, p);
    // mu replaces u in place (u is read at the cell only); F is then written directly
    hipLaunchKernelGGL(k_mp_inner, mp_grid(c), dim3(64, 4), 0, c->stream, Phi, phi, u, Lu, nullptr, 0, u, p);
    if (p.mob)
        hipLaunchKernelGGL(k_mp_final_mob, mp_grid(c), dim3(64, 4), 0, c->stream, Phi, phi, u, src, 0, nullptr,
                           nullptr, F, p);
    else
        hipLaunchKernelGGL(k_mp_final, mp_grid(c), dim3(64, 4), 0, c->stream, Phi, phi, u, src, 0, F, p);
    if (norm_part) hipLaunchKernelGGL(k_sumsq, dim3(kRedBlocks), dim3(NT), 0, c->stream, F, c->g.N, norm_part);
    return hipGetLastError();
}

hipError_t launch_coef(const pfc_ctx* c, const double* Phi, const double* phi, double* cbuf) {
    hipLaunchKernelGGL(k_coef, dim3(2048), dim3(256), 0, c->stream, Phi, phi, cbuf, c->g.N);
    if (c->model.mobility == PFC_MOBILITY_1_MINUS_SQ && cbuf == c->d_c) {
        // the mobility term of the Jacobian action needs u = (Phi + phi)/2 and mu_d of the iterate
        const P p = make_params(c, 1.0);
        double* Lu = c->d_tmp3;
        hipLaunchKernelGGL(k_mp_combine, dim3(2048), dim3(256), 0, c->stream, Phi, phi, nullptr, 0, 0.0, nullptr, 0,
                           c->d_u, c->g.N);
        hipLaunchKernelGGL(k_mp_lap, mp_grid(c), dim3(64, 4), 0, c->stream, c->d_u, Lu, p);
        hipLaunchKernelGGL(k_mp_inner, mp_grid(c), dim3(64, 4), 0, c->stream, Phi, phi, c->d_u, Lu, nullptr, 0,
                           c->d_mu, p);
    }
    return hipGetLastError();
}

hipError_t launch_jv(const pfc_ctx* c, const double* v, const double* cbuf, double dt, const double* shift_part,
                     int shift_n, double shift_scale, double* shift_out, double* Jv) {
    const P p = make_params(c, dt);
    if (fused2d(c)) {
        return sliding(c->g.nx, c->g.ny)
                   ? launch_k(c, k_jv2d, residual_grid(c), dim3(NT), 0, v, cbuf, shift_part, shift_n, shift_scale,
                              shift_out, Jv, p)
                   : launch_k(c, k_jv2d_tile, residual_grid(c), dim3(NT), 0, v, cbuf, shift_part, shift_n,
                              shift_scale, shift_out, Jv, p);
    }
    if (fused3d(c))
        return launch_k(c, k_jv3d, residual_grid(c), dim3(NT), 0, v, cbuf, shift_part, shift_n, shift_scale, shift_out,
                        Jv, p);
    // the shifted v lives in the output buffer, the inner operator in the scratch vector, and the
    // last pass updates the output in place (it reads the shifted v at the cell only)
    double* w = c->d_tmp3;
    double* Lu = c->d_tmp3 + c->g.N;
    hipLaunchKernelGGL(k_mp_combine, dim3(2048), dim3(256), 0, c->stream, v, nullptr, shift_part, shift_n,
                       shift_scale, shift_out, 1, Jv, c->g.N);
    hipLaunchKernelGGL(k_mp_lap, mp_grid(c), dim3(64, 4), 0, c->stream, Jv, Lu, p);
    hipLaunchKernelGGL(k_mp_inner, mp_grid(c), dim3(64, 4), 0, c->stream, nullptr, nullptr, Jv, Lu, cbuf, 1, w, p);
    if (p.mob)
        hipLaunchKernelGGL(k_mp_final_mob, mp_grid(c), dim3(64, 4), 0, c->stream, Jv, nullptr, w, nullptr, 1, c->d_u,
                           c->d_mu, Jv, p);
    else
        hipLaunchKernelGGL(k_mp_final, mp_grid(c), dim3(64, 4), 0, c->stream, Jv, nullptr, w, nullptr, 1, Jv, p);
    return hipGetLastError();
}

int residual2d_blocks(int nx, int ny) { return (int)grid2d(nx, ny); }

hipError_t launch_residual2d_plain(hipStream_t s, int nx, int ny, double ihx2, double ihy2, double gamma,
                                   double dt, const double* Phi, const double* phi, const double* src, double* F,
                                   double* norm_part) {
    P p;
    p.nx = nx;
    p.ny = ny;
    p.nz = 1;
    p.ihx2 = ihx2;
    p.ihy2 = ihy2;
    p.ihz2 = 0.0;
    p.gamma = gamma;
    p.inv_dt = dt > 0 ? 1.0 / dt : 0.0;
    p.neu = 0;
    p.mob = 0;
    if (sliding(nx, ny))
        hipLaunchKernelGGL(k_residual2d, dim3(grid2d(nx, ny)), dim3(NT), 0, s, Phi, phi, src, F, norm_part,
                           (double*)nullptr, p);
    else
        hipLaunchKernelGGL(k_residual2d_tile, dim3(grid2d(nx, ny)), dim3(NT), 0, s, Phi, phi, src, F, norm_part,
                           (double*)nullptr, p);
    return hipGetLastError();
}

hipError_t launch_energy(const pfc_ctx* c, const double* phi, double* part2, double* acc_phi, double* acc_prev) {
    const P p = make_params(c, 0.0);
    if (fused2d(c)) {
        hipLaunchKernelGGL(k_energy2d, tiles2d(c), dim3(NT), 0, c->stream, phi, part2, p, acc_phi, acc_prev);
    } else {
        if (acc_phi) {
            const size_t bytes = sizeof(double) * c->g.N;
            hipError_t e = hipMemcpyAsync(acc_prev, acc_phi, bytes, hipMemcpyDeviceToDevice, c->stream);
            if (e == hipSuccess) e = hipMemcpyAsync(acc_phi, phi, bytes, hipMemcpyDeviceToDevice, c->stream);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL(k_mp_energy, dim3(kRedBlocks), dim3(NT), 0, c->stream, phi, part2, p);
    }
    return hipGetLastError();
}

}  // namespace pfc
