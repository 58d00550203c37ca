// Restricted additive Schwarz with ILU(0) subdomain solves (Sec. 4, Eqs. (23), (25), (26)).
//
// Subdomain matrix: A_k = R_k J R_k^T, which is the Jacobian of the subdomain problem
// with phi = 0 on the three-layer ring around the extended box.  Row i of A_k has one
// entry per composite-stencil offset o with i + o inside the box:
//     A(i, i+o) = kconst(o) - d1(o) * c(i+o)
// (kconst: I/dt - (1-gamma)/2 Delta - Delta^2 - 1/2 Delta^3, d1: Delta; c from Eq. (19)).
//
// ILU(0) keeps exactly that pattern, natural (z, y, x) order, IKJ elimination.  Rows
// are scheduled by the wavefront level x + 3y (2-D) / x + 3y + 7z (3-D): every
// lower-triangular neighbour of a cell has a strictly smaller level, so all cells of
// one level factor and solve independently.  One workgroup per subdomain; the solve (one
// wave) keeps the box vector in LDS and streams the factors, packed level by level in
// groups of four so that a lane's loads are 16 or 32 bytes wide and the lanes of a level
// read consecutive addresses.  Classical AS and right-RAS (Eqs. (22), (24)) keep each box's
// extended solution and add them per cell in a second kernel.
#include <algorithm>
#include <vector>

#include "device_reduce.h"
#include "pfc_internal.h"

namespace pfc {

void build_stencil_table(const Geom& g, double gamma, double dt, StencilTable* t) {
    // D1 = Delta_d, D2 = D1 * D1, D3 = D2 * D1 as 7x7x7 offset maps (index (dz+3, dy+3, dx+3)).
    static thread_local double d1[7][7][7], d2[7][7][7], d3[7][7][7];
    for (int a = 0; a < 7; ++a)
        for (int b = 0; b < 7; ++b)
            for (int c = 0; c < 7; ++c) d1[a][b][c] = d2[a][b][c] = d3[a][b][c] = 0.0;
    d1[3][3][3] = -2.0 * (g.ihx2 + g.ihy2 + (g.dim == 3 ? g.ihz2 : 0.0));
    d1[3][3][4] += g.ihx2;
    d1[3][3][2] += g.ihx2;
    d1[3][4][3] += g.ihy2;
    d1[3][2][3] += g.ihy2;
    if (g.dim == 3) {
        d1[4][3][3] += g.ihz2;
        d1[2][3][3] += g.ihz2;
    }
    auto conv = [](double (*a)[7][7], double (*b)[7][7], double (*out)[7][7]) {
        for (int z = 0; z < 7; ++z)
            for (int y = 0; y < 7; ++y)
                for (int x = 0; x < 7; ++x) {
                    if (a[z][y][x] == 0.0) continue;
                    for (int dz = -1; dz <= 1; ++dz)
                        for (int dy = -1; dy <= 1; ++dy)
                            for (int dx = -1; dx <= 1; ++dx) {
                                const double bv = b[3 + dz][3 + dy][3 + dx];
                                if (bv == 0.0) continue;
                                const int zz = z + dz, yy = y + dy, xx = x + dx;
                                if (zz < 0 || zz > 6 || yy < 0 || yy > 6 || xx < 0 || xx > 6) continue;
                                out[zz][yy][xx] += a[z][y][x] * bv;
                            }
                }
    };
    conv(d1, d1, d2);
    conv(d2, d1, d3);
    int s = 0;
    const int zr = g.dim == 3 ? 3 : 0;
    for (int dz = -zr; dz <= zr; ++dz)
        for (int dy = -3; dy <= 3; ++dy)
            for (int dx = -3; dx <= 3; ++dx) {
                if (std::abs(dx) + std::abs(dy) + std::abs(dz) > 3) continue;
                t->dx[s] = (int8_t)dx;
                t->dy[s] = (int8_t)dy;
                t->dz[s] = (int8_t)dz;
                const double k1 = d1[3 + dz][3 + dy][3 + dx];
                const double k2 = d2[3 + dz][3 + dy][3 + dx];
                const double k3 = d3[3 + dz][3 + dy][3 + dx];
                double kc = -0.5 * (1.0 - gamma) * k1 - k2 - 0.5 * k3;
                if (dx == 0 && dy == 0 && dz == 0) {
                    kc += 1.0 / dt;
                    t->diag = s;
                }
                t->inv_dt = 1.0 / dt;
                t->kconst[s] = kc;
                t->d1[s] = k1;
                ++s;
            }
    t->S = s;
}

namespace {

struct Box {
    int ex, ey, ez, next;
    int subx, suby, ownx, owny, ownz, ov;
    int nx, ny, nz;
};

__device__ __forceinline__ int wrapg(int i, int n) {
    i %= n;
    return i < 0 ? i + n : i;
}

__device__ __forceinline__ void box_origin(const Box& b, int k, int* ox, int* oy, int* oz) {
    const int kx = k % b.subx, ky = (k / b.subx) % b.suby, kz = k / (b.subx * b.suby);
    *ox = kx * b.ownx - b.ov;
    *oy = ky * b.owny - b.ov;
    *oz = b.nz > 1 ? kz * b.ownz - b.ov : 0;
}

__device__ __forceinline__ long gidx(const Box& b, int ox, int oy, int oz, int x, int y, int z) {
    const int gx = wrapg(ox + x, b.nx), gy = wrapg(oy + y, b.ny), gz = b.nz > 1 ? wrapg(oz + z, b.nz) : 0;
    return ((long)gz * b.ny + gy) * b.nx + gx;
}

__device__ __forceinline__ bool inbox(const Box& b, int x, int y, int z) {
    return x >= 0 && x < b.ex && y >= 0 && y < b.ey && z >= 0 && z < b.ez;
}

// Packed ILU(0) factors of one box, level-major.  For the n_l cells of a level the D lower
// factors come as QL groups of four ([group][cell][4]), then the reciprocal pivot and the D
// upper factors as QU groups of four; unused slots are zero.  A lane reads its cell's factors
// with 16-byte (FP32) or 32-byte (FP64) loads that are contiguous across the lanes.
template <int S>
struct IluPack {
    static constexpr int D = S / 2;
    static constexpr int QL = (D + 3) / 4;
    static constexpr int QU = (D + 4) / 4;
    static constexpr int kPerCell = 4 * (QL + QU);
    template <typename T>
    using Vec = T __attribute__((ext_vector_type(4)));
};

// The composite stencil's offsets in natural order (z, then y, then x; |dx| + |dy| + |dz| <= 3,
// the order build_stencil_table uses), and for each pair (s, t) the index of offset(t) -
// offset(s), or -1.  Known at compile time, so the elimination reads each pivot row at fixed
// offsets and skips the pairs outside the pattern without a test.
template <int S>
struct IluPairs {
    int8_t dx[S], dy[S], dz[S];
    int8_t u[S][S];
    constexpr IluPairs() : dx(), dy(), dz(), u() {
        int idx[7][7][7] = {};
        for (int z = 0; z < 7; ++z)
            for (int y = 0; y < 7; ++y)
                for (int x = 0; x < 7; ++x) idx[z][y][x] = -1;
        const int zr = S == 63 ? 3 : 0;
        int n = 0;
        for (int z = -zr; z <= zr; ++z)
            for (int y = -3; y <= 3; ++y)
                for (int x = -3; x <= 3; ++x) {
                    if ((x < 0 ? -x : x) + (y < 0 ? -y : y) + (z < 0 ? -z : z) > 3) continue;
                    dx[n] = (int8_t)x;
                    dy[n] = (int8_t)y;
                    dz[n] = (int8_t)z;
                    idx[z + 3][y + 3][x + 3] = n++;
                }
        for (int s = 0; s < S; ++s)
            for (int t = 0; t < S; ++t) {
                const int x = dx[t] - dx[s] + 3, y = dy[t] - dy[s] + 3, z = dz[t] - dz[s] + 3;
                const bool inside = x >= 0 && x < 7 && y >= 0 && y < 7 && z >= 0 && z < 7;
                u[s][t] = (int8_t)(inside ? idx[z][y][x] : -1);
            }
    }
};
template <int S>
inline constexpr IluPairs<S> kIluPairs{};

template <typename T, int S>
__global__ __launch_bounds__(256) void k_ilu_factor(const double* __restrict__ cc,
                                                    const int* __restrict__ lptr,
                                                    const int* __restrict__ lpts, double* __restrict__ work,
                                                    T* __restrict__ fac, int* __restrict__ flag, Box b,
                                                    StencilTable st, int nlev, const double* __restrict__ uu) {
    constexpr int D = S / 2;                  // the zero offset sits in the middle (natural order)
    const int k = blockIdx.x;
    int ox, oy, oz;
    box_origin(b, k, &ox, &oy, &oz);
    double* W = work + (long)k * b.next * S;
    // assemble A_k row by row
    for (int i = threadIdx.x; i < b.next; i += blockDim.x) {
        const int x = i % b.ex, y = (i / b.ex) % b.ey, z = i / (b.ex * b.ey);
        const long gi = gidx(b, ox, oy, oz, x, y, z);
        for (int s = 0; s < S; ++s) {
            const int xx = x + kIluPairs<S>.dx[s], yy = y + kIluPairs<S>.dy[s], zz = z + kIluPairs<S>.dz[s];
            double v = 0.0;
            if (inbox(b, xx, yy, zz)) v = subdomain_entry(st, s, cc[gidx(b, ox, oy, oz, xx, yy, zz)], uu, gi);
            W[(long)i * S + s] = v;
        }
    }
    __syncthreads();
    for (int lev = 0; lev < nlev; ++lev) {
        for (int p = lptr[lev] + threadIdx.x; p < lptr[lev + 1]; p += blockDim.x) {
            const int pk = lpts[p];
            const int x = pk & 255, y = (pk >> 8) & 255, z = pk >> 16;
            const long i = ((long)z * b.ey + y) * b.ex + x;
            double* row = W + i * S;
            // the row being eliminated lives in registers; the unrolled loops let every load
            // of the earlier (pivot) rows it needs be in flight together
            double r[S];
            bool in[S];
#pragma unroll
            for (int t = 0; t < S; ++t) {
                r[t] = row[t];
                in[t] = inbox(b, x + kIluPairs<S>.dx[t], y + kIluPairs<S>.dy[t], z + kIluPairs<S>.dz[t]);
            }
#pragma unroll
            for (int s = 0; s < D; ++s) {
                if (!in[s]) continue;
                const long kk = i + ((long)kIluPairs<S>.dz[s] * b.ey + kIluPairs<S>.dy[s]) * b.ex + kIluPairs<S>.dx[s];
                const double* rk = W + kk * S;
                const double aik = r[s] / rk[D];
                r[s] = aik;
#pragma unroll
                for (int t = s + 1; t < S; ++t) {
                    const int u = kIluPairs<S>.u[s][t];   // resolved at compile time
                    if (u >= 0 && in[t]) r[t] -= aik * rk[u];
                }
            }
#pragma unroll
            for (int t = 0; t < S; ++t) row[t] = r[t];
            const double piv = r[D];
            if (!(piv != 0.0) || !isfinite(piv)) *flag = 1;
        }
        __syncthreads();
    }
    // pack level-major in groups of four factors (see IluPack): lower factors first, then the
    // reciprocal pivot followed by the upper factors; the padding slots hold zero
    using P = IluPack<S>;
    T* out = fac + (long)k * b.next * P::kPerCell;
    for (int lev = 0; lev < nlev; ++lev) {
        const int p0 = lptr[lev], nl = lptr[lev + 1] - p0;
        const long lb = (long)p0 * P::kPerCell, ub = lb + (long)P::QL * 4 * nl;
        for (int p = threadIdx.x; p < nl; p += blockDim.x) {
            const int pk = lpts[p0 + p];
            const int x = pk & 255, y = (pk >> 8) & 255, z = pk >> 16;
            const double* row = W + (((long)z * b.ey + y) * b.ex + x) * S;
            for (int q = 0; q < P::QL; ++q)
                for (int e = 0; e < 4; ++e) {
                    const int t = 4 * q + e;
                    out[lb + ((long)q * nl + p) * 4 + e] = (T)(t < D ? row[t] : 0.0);
                }
            for (int q = 0; q < P::QU; ++q)
                for (int e = 0; e < 4; ++e) {
                    const int u = 4 * q + e;
                    out[ub + ((long)q * nl + p) * 4 + e] = (T)(u == 0 ? 1.0 / row[D] : (u <= D ? row[D + u] : 0.0));
                }
        }
    }
}

// One wave per box: forward then backward substitution over the wavefront levels with the
// box vector in LDS.  Each lane takes C cells of a level (the host picks C from the widest
// level).  The factors of the next PF levels are in flight in registers while a level is
// computed: the loads are unconditional (clamped to the last cell and level), so the number of
// loads issued after any level's factors is fixed and the wait before a level covers that
// level only.  Neighbour indices are the cell index plus a per-box constant offset, clamped
// into the box: a neighbour outside the box has a zero factor (the pattern of A_k stops at
// the box), so whatever the clamped read returns adds nothing.
// The apply runs one wave per box, and a wave's LDS operations take effect in program order,
// so a level only has to keep the compiler from moving LDS accesses across the level boundary.
// The scheduling barrier keeps each level's work (and the fetch that follows it) in its place,
// so that the wait before a level is for that level's loads.
__device__ __forceinline__ void wave_lds_order() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_sched_barrier(0);
}

template <typename T, int S, int C>
struct IluApplyShape {
    using P = IluPack<S>;
    static constexpr int kLoadsPerLevel = C * (1 + P::QL * (int)(sizeof(T) / 4));   // vector memory ops
    static constexpr int PF = 60 / kLoadsPerLevel < 1 ? 1 : (60 / kLoadsPerLevel > 4 ? 4 : 60 / kLoadsPerLevel);
};

template <typename V, int PF, int C, int Q>
__device__ __forceinline__ void zero_slots(V (&f)[PF][C][Q], int (&pk)[PF][C], int (&nl)[PF]) {
#pragma unroll
    for (int j = 0; j < PF; ++j) {
        nl[j] = 0;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            pk[j][c] = 0;
#pragma unroll
            for (int q = 0; q < Q; ++q) f[j][c][q] = V{};
        }
    }
}

template <typename T, int S, int C>
__global__ __launch_bounds__(64) void k_ilu_apply(const double* __restrict__ r, double* __restrict__ z,
                                                  const T* __restrict__ fac, const int* __restrict__ lptr,
                                                  const int* __restrict__ lpts, Box b, StencilTable st,
                                                  int nlev, double* __restrict__ sum_part, int mode,
                                                  double* __restrict__ zbox) {
    using P = IluPack<S>;
    using V = typename P::template Vec<T>;
    constexpr int D = S / 2;                  // centre of the natural-order stencil
    constexpr int QL = P::QL, QU = P::QU, PF = IluApplyShape<T, S, C>::PF;
    extern __shared__ unsigned char smem_raw[];
    T* yv = reinterpret_cast<T*>(smem_raw);
    const int tid = threadIdx.x;
    const int k = blockIdx.x;
    int ox, oy, oz;
    box_origin(b, k, &ox, &oy, &oz);
    const int zoff = b.nz > 1 ? b.ov : 0, owz = b.nz > 1 ? b.ownz : 1;
    for (int i = tid; i < b.next; i += blockDim.x) {
        const int x = i % b.ex, y = (i / b.ex) % b.ey, zz = i / (b.ex * b.ey);
        // right-RAS restricts the owned cells only (Eq. (24)); the others restrict the whole box
        const bool own = x >= b.ov && x < b.ov + b.ownx && y >= b.ov && y < b.ov + b.owny && zz >= zoff &&
                         zz < zoff + owz;
        yv[i] = (mode != 2 || own) ? (T)r[gidx(b, ox, oy, oz, x, y, zz)] : (T)0;
    }
    if (tid == 0) yv[b.next] = (T)0;   // spare slot for lanes without a cell
    const T* F = fac + (long)k * b.next * P::kPerCell;
    const int last = b.next - 1;
    auto cell = [&](int pk) { return ((pk >> 16) * b.ey + ((pk >> 8) & 255)) * b.ex + (pk & 255); };
    auto noff = [&](int s) { return ((int)st.dz[s] * b.ey + st.dy[s]) * b.ex + st.dx[s]; };
    wave_lds_order();
    // forward sweep (unit lower factor)
    {
        V f[PF][C][QL];
        int pk[PF][C], nl[PF];
        auto fetch = [&](int lev, V (&dst)[C][QL], int (&pkd)[C], int& nld) {
            const int l = min(max(lev, 0), nlev - 1);
            const int p0 = lptr[l];
            nld = lptr[l + 1] - p0;
            const V* base = reinterpret_cast<const V*>(F + (long)p0 * P::kPerCell);
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const int p = min(tid + 64 * c, nld - 1);
                pkd[c] = lpts[p0 + p];
#pragma unroll
                for (int q = 0; q < QL; ++q) dst[c][q] = __builtin_nontemporal_load(&base[(long)q * nld + p]);
            }
        };
        zero_slots(f, pk, nl);
        // the first pass computes nothing (levels -PF..-1) and only fetches; entering the loop
        // with no loads in flight lets the wait before each level count just that level's loads
        for (int l0 = -PF; l0 < nlev; l0 += PF) {
#pragma unroll
            for (int j = 0; j < PF; ++j) {
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    // a lane with no cell (or a level outside 0..nlev-1) works on the spare slot
                    const bool ok = l0 + j >= 0 && l0 + j < nlev && tid + 64 * c < nl[j];
                    const int i = ok ? cell(pk[j][c]) : b.next;
                    T acc = yv[i];
#pragma unroll
                    for (int q = 0; q < D; ++q) acc -= f[j][c][q / 4][q % 4] * yv[min(max(i + noff(q), 0), last)];
                    // adding the zero padding keeps every loaded register live until here, so
                    // none is reused (and waited for) while its load is still in flight
#pragma unroll
                    for (int t = D; t < 4 * QL; ++t) acc += f[j][c][t / 4][t % 4];
                    yv[i] = acc;
                }
                wave_lds_order();
                fetch(l0 + j + PF, f[j], pk[j], nl[j]);
            }
        }
    }
    // backward sweep (upper factors, then the stored reciprocal pivot)
    {
        V f[PF][C][QU];
        int pk[PF][C], nl[PF];
        auto fetch = [&](int lev, V (&dst)[C][QU], int (&pkd)[C], int& nld) {
            const int l = min(max(lev, 0), nlev - 1);
            const int p0 = lptr[l];
            nld = lptr[l + 1] - p0;
            const V* base = reinterpret_cast<const V*>(F + (long)p0 * P::kPerCell) + (long)QL * nld;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const int p = min(tid + 64 * c, nld - 1);
                pkd[c] = lpts[p0 + p];
#pragma unroll
                for (int q = 0; q < QU; ++q) dst[c][q] = __builtin_nontemporal_load(&base[(long)q * nld + p]);
            }
        };
        zero_slots(f, pk, nl);
        for (int l0 = nlev - 1 + PF; l0 >= 0; l0 -= PF) {
#pragma unroll
            for (int j = 0; j < PF; ++j) {
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const bool ok = l0 - j >= 0 && l0 - j < nlev && tid + 64 * c < nl[j];
                    const int i = ok ? cell(pk[j][c]) : b.next;
                    T acc = yv[i];
#pragma unroll
                    for (int q = 1; q <= D; ++q)
                        acc -= f[j][c][q / 4][q % 4] * yv[min(max(i + noff(D + q), 0), last)];
#pragma unroll
                    for (int t = D + 1; t < 4 * QU; ++t) acc += f[j][c][t / 4][t % 4];
                    yv[i] = acc * f[j][c][0][0];
                }
                wave_lds_order();
                fetch(l0 - j - PF, f[j], pk[j], nl[j]);
            }
        }
    }
    double acc = 0.0;
    if (mode == 0) {   // left-RAS: restricted extension, the owned cells only (Eq. (23))
        const int owx = b.ownx, owy = b.owny;
        for (int e = threadIdx.x; e < owx * owy * owz; e += blockDim.x) {
            const int x = e % owx + b.ov, y = (e / owx) % owy + b.ov, zz = e / (owx * owy) + zoff;
            const double v = (double)yv[(zz * b.ey + y) * b.ex + x];
            z[gidx(b, ox, oy, oz, x, y, zz)] = v;
            acc += v;
        }
    } else {           // classical AS / right-RAS: the whole extended solution, added per cell later
        for (int i = threadIdx.x; i < b.next; i += blockDim.x) {
            const double v = (double)yv[i];
            zbox[(long)k * b.next + i] = v;
            acc += v;
        }
    }
    if (sum_part) {
        __shared__ double red[16];
        const double sum = block_sum_det(acc, red);
        if (threadIdx.x == 0) sum_part[blockIdx.x] = sum;
    }
}

// z(p) = sum of zbox over the boxes whose extended region covers cell p (classical AS and
// right-RAS extension, Eqs. (22), (24)).  Along each axis the candidates are the owner box and
// ceil(ov / own) boxes on either side (all boxes, in order, when that reaches round the
// periodic axis), so each covering box is visited once, in the same order for every run.
struct SumGeom {
    int n[3], sub[3], own[3], ext[3], ovl[3], R[3];
};

// Candidate t (0 <= t < count) of one axis: its box index and the cell's position in that box's
// extension (>= ext when the box does not cover the cell).
struct AxisCover {
    int k0, R, sub, own, ovl, n, all, count;
    __device__ AxisCover(int pos, int R_, int sub_, int own_, int ovl_, int n_)
        : k0(pos / own_), R(R_), sub(sub_), own(own_), ovl(ovl_), n(n_),
          all(2 * R_ + 1 >= sub_), count(2 * R_ + 1 >= sub_ ? sub_ : 2 * R_ + 1) {}
    __device__ int box(int t) const { return all ? t : wrapg(k0 - R + t, sub); }
    __device__ int local(int pos, int kk) const { return wrapg(pos - (kk * own - ovl), n); }
};

__global__ __launch_bounds__(256) void k_schwarz_sum(const double* __restrict__ zbox, double* __restrict__ z,
                                                     SumGeom g, long N, int next) {
    for (long p = blockIdx.x * (long)blockDim.x + threadIdx.x; p < N; p += (long)gridDim.x * blockDim.x) {
        const int px = (int)(p % g.n[0]), py = (int)((p / g.n[0]) % g.n[1]), pz = (int)(p / ((long)g.n[0] * g.n[1]));
        const AxisCover ax(px, g.R[0], g.sub[0], g.own[0], g.ovl[0], g.n[0]);
        const AxisCover ay(py, g.R[1], g.sub[1], g.own[1], g.ovl[1], g.n[1]);
        const AxisCover az(pz, g.R[2], g.sub[2], g.own[2], g.ovl[2], g.n[2]);
        double acc = 0.0;
        for (int tz = 0; tz < az.count; ++tz) {
            const int kz = az.box(tz), lz = az.local(pz, kz);
            if (lz >= g.ext[2]) continue;
            for (int ty = 0; ty < ay.count; ++ty) {
                const int ky = ay.box(ty), ly = ay.local(py, ky);
                if (ly >= g.ext[1]) continue;
                for (int tx = 0; tx < ax.count; ++tx) {
                    const int kx = ax.box(tx), lx = ax.local(px, kx);
                    if (lx >= g.ext[0]) continue;
                    const long k = ((long)kz * g.sub[1] + ky) * g.sub[0] + kx;
                    acc += zbox[k * next + ((long)lz * g.ext[1] + ly) * g.ext[0] + lx];
                }
            }
        }
        z[p] = acc;
    }
}

Box make_box(const pfc_ctx* c) {
    Box b;
    b.ex = c->dec.ext[0];
    b.ey = c->dec.ext[1];
    b.ez = c->g.dim == 3 ? c->dec.ext[2] : 1;
    b.next = c->dec.next;
    b.subx = c->dec.sub[0];
    b.suby = c->dec.sub[1];
    b.ownx = c->dec.own[0];
    b.owny = c->dec.own[1];
    b.ownz = c->dec.own[2];
    b.ov = c->dec.ov;
    b.nx = c->g.nx;
    b.ny = c->g.ny;
    b.nz = c->g.nz;
    return b;
}

}  // namespace

// Host-side level schedule for the box shape of the context.
void build_ilu_schedule(const pfc_ctx* c, std::vector<int>* lptr, std::vector<int>* lpts) {
    const int ex = c->dec.ext[0], ey = c->dec.ext[1], ez = c->g.dim == 3 ? c->dec.ext[2] : 1;
    const int maxlev = (ex - 1) + 3 * (ey - 1) + 7 * (ez - 1) + 1;
    std::vector<std::vector<int>> by(maxlev);
    for (int z = 0; z < ez; ++z)
        for (int y = 0; y < ey; ++y)
            for (int x = 0; x < ex; ++x) by[x + 3 * y + 7 * z].push_back(x | (y << 8) | (z << 16));
    lptr->assign(1, 0);
    lpts->clear();
    for (auto& v : by) {
        if (v.empty()) continue;   // a level value no cell of a thin box takes
        for (int p : v) lpts->push_back(p);
        lptr->push_back((int)lpts->size());
    }
}

template <int S>
hipError_t launch_ilu_factor_s(pfc_ctx* c, const StencilTable& st, const Box& b) {
    for (int s = 0; s < S; ++s)   // the kernel's pair table assumes this offset order
        if (st.dx[s] != kIluPairs<S>.dx[s] || st.dy[s] != kIluPairs<S>.dy[s] || st.dz[s] != kIluPairs<S>.dz[s])
            return hipErrorInvalidValue;
    if (c->opts.precond_fp32)
        hipLaunchKernelGGL((k_ilu_factor<float, S>), dim3(c->dec.nsub), dim3(256), 0, c->stream, c->d_c,
                           c->d_level_ptr, c->d_level_pts, c->d_work, (float*)c->d_fac, c->d_flag, b, st, c->nlev,
                           (const double*)c->d_u);
    else
        hipLaunchKernelGGL((k_ilu_factor<double, S>), dim3(c->dec.nsub), dim3(256), 0, c->stream, c->d_c,
                           c->d_level_ptr, c->d_level_pts, c->d_work, (double*)c->d_fac, c->d_flag, b, st, c->nlev,
                           (const double*)c->d_u);
    return hipGetLastError();
}

hipError_t launch_ilu_factor(pfc_ctx* c, const StencilTable& st) {
    const Box b = make_box(c);
    if (st.diag != st.S / 2) return hipErrorInvalidValue;   // natural order puts the centre in the middle
    if (st.S == 25) return launch_ilu_factor_s<25>(c, st, b);
    if (st.S == 63) return launch_ilu_factor_s<63>(c, st, b);
    return hipErrorInvalidValue;
}

hipError_t launch_schwarz_sum(const pfc_ctx* c, const double* zbox, double* z) {
    SumGeom g;
    const int gn[3] = {c->g.nx, c->g.ny, c->g.nz};
    for (int a = 0; a < 3; ++a) {
        const bool on = a < c->g.dim;
        g.n[a] = on ? gn[a] : 1;
        g.sub[a] = on ? c->dec.sub[a] : 1;
        g.own[a] = on ? c->dec.own[a] : 1;
        g.ext[a] = on ? c->dec.ext[a] : 1;
        g.ovl[a] = on ? c->dec.ov : 0;
        g.R[a] = (g.ovl[a] + g.own[a] - 1) / g.own[a];
        if (std::min(2 * g.R[a] + 1, g.sub[a]) > 16) return hipErrorInvalidValue;   // checked by pfc_create
    }
    const long N = c->g.N;
    const unsigned grid = (unsigned)std::min<long>((N + 255) / 256, 8192);
    hipLaunchKernelGGL(k_schwarz_sum, dim3(grid), dim3(256), 0, c->stream, zbox, z, g, N, c->dec.next);
    return hipGetLastError();
}

template <typename T, int S, int C>
hipError_t launch_ilu_apply_c(pfc_ctx* c, const double* r, double* z, double* sum_part, const Box& b) {
    return launch_k(c, k_ilu_apply<T, S, C>, dim3(c->dec.nsub), dim3(64), sizeof(T) * (b.next + 1), r, z,
                    (const T*)c->d_fac, c->d_level_ptr, c->d_level_pts, b, c->st, c->nlev, sum_part,
                    c->opts.ras_kind, c->d_zbox);
}

template <typename T, int S>
hipError_t launch_ilu_apply_t(pfc_ctx* c, const double* r, double* z, double* sum_part, const Box& b) {
    switch (c->ilu_cells_per_lane) {
        case 1: return launch_ilu_apply_c<T, S, 1>(c, r, z, sum_part, b);
        case 2: return launch_ilu_apply_c<T, S, 2>(c, r, z, sum_part, b);
        case 3: return launch_ilu_apply_c<T, S, 3>(c, r, z, sum_part, b);
        default: return hipErrorInvalidValue;
    }
}

template <int S>
hipError_t launch_ilu_apply_s(pfc_ctx* c, const double* r, double* z, double* sum_part, const Box& b) {
    return c->opts.precond_fp32 ? launch_ilu_apply_t<float, S>(c, r, z, sum_part, b)
                                : launch_ilu_apply_t<double, S>(c, r, z, sum_part, b);
}

hipError_t launch_ilu_apply(pfc_ctx* c, const double* r, double* z, double* sum_part) {
    const Box b = make_box(c);
    if (c->st.diag != c->st.S / 2) return hipErrorInvalidValue;
    if (c->st.S == 25) return launch_ilu_apply_s<25>(c, r, z, sum_part, b);
    if (c->st.S == 63) return launch_ilu_apply_s<63>(c, r, z, sum_part, b);
    return hipErrorInvalidValue;
}

int ilu_fac_elems_per_cell(int S) {
    if (S == 25) return IluPack<25>::kPerCell;
    if (S == 63) return IluPack<63>::kPerCell;
    return 0;
}

hipError_t set_ilu_lds_limits() {
    const void* fs[] = {
        (const void*)k_ilu_apply<double, 25, 1>, (const void*)k_ilu_apply<float, 25, 1>,
        (const void*)k_ilu_apply<double, 63, 1>, (const void*)k_ilu_apply<float, 63, 1>,
        (const void*)k_ilu_apply<double, 25, 2>, (const void*)k_ilu_apply<float, 25, 2>,
        (const void*)k_ilu_apply<double, 63, 2>, (const void*)k_ilu_apply<float, 63, 2>,
        (const void*)k_ilu_apply<double, 25, 3>, (const void*)k_ilu_apply<float, 25, 3>,
        (const void*)k_ilu_apply<double, 63, 3>, (const void*)k_ilu_apply<float, 63, 3>};
    for (const void* f : fs) {
        const hipError_t e = set_dynamic_lds_limit(f);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace pfc
