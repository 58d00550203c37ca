// Restricted additive Schwarz with ILU(k) subdomain solves, k >= 0 levels of fill (Sec. 4
// subdomain solvers; the ILU(1) and ILU(2) columns of Table 1).
//
// Pattern.  The level-k pattern of the box matrix A_k (the zero-ring subdomain matrix of
// Eqs. (25)-(26), natural z, y, x order) follows the level-of-fill rule: entries of A_k have
// level 0; eliminating row i, each kept lower entry (i, m) gives every later column j of row m
// the level lev(i, m) + lev(m, j) + 1, and entries above level k are dropped (Saad, Iterative
// Methods for Sparse Linear Systems, Sec. 10.3.3).  The pattern depends only on the box shape,
// so the host builds it once for all boxes, with the schedules below.
//
// Factorisation (one wave per box).  A_k is assembled in FP64 in the pattern's row-major
// layout, then rows are eliminated in the IKJ order on that pattern: for each kept lower
// entry m of row i in increasing order, a_im /= a_mm and a_ij -= a_im a_mj for every j > m
// of row m that is in row i's pattern.  Rows whose lower entries lie in earlier dependency
// levels are independent; a level's rows are worked by groups of 16 lanes, each row held in
// LDS with a column -> position map of the box, so a pivot row's update needs no precomputed
// intersection table.
//
// Apply (one wave per box).  Forward and backward substitution by dependency levels with the
// box vector in LDS.  The rows of a level are packed into passes of at most 64 lanes; each
// row gets ceil(len / 4) consecutive lanes, a lane holds four consecutive entries of one row
// (16-byte FP32 loads, contiguous across the lanes), lane products go to LDS and the row's
// first lane adds its lanes' products in order.  Backward rows carry the reciprocal pivot in
// their first slot, against the spare zero slot of the vector.  The factors of the next passes
// are in flight while a pass is computed.
#include <algorithm>
#include <queue>
#include <string>
#include <vector>

#include "device_reduce.h"
#include "pfc_internal.h"

namespace pfc {

struct IlukPlan {
    int n = 0;                   // cells per box
    long nnz = 0;                // entries of the level-k pattern per box
    int maxrow = 0;              // longest row of the pattern
    int nfl = 0;                 // dependency levels of the factorisation (= forward levels)
    int npass_f = 0, npass_b = 0;
    long nlanes = 0;             // lane slots of all passes (epl values each)
    int maxseg = 1;              // most lanes one row takes in a pass
    int epl = 4;                 // entries per lane slot, 4 or 8
    int* d_rowptr = nullptr;     // [n + 1]
    uint16_t* d_col = nullptr;   // [nnz] local column
    int8_t* d_sten = nullptr;    // [nnz] stencil offset index, or -1 for a fill entry
    uint16_t* d_diag = nullptr;  // [n] position of the diagonal in its row
    int* d_flev = nullptr;       // [nfl + 1] factorisation levels ...
    uint16_t* d_frow = nullptr;  // [n] ... and their rows
    int2* d_pass = nullptr;      // [npass_f + npass_b]: first lane slot, used lanes
    uint32_t* d_meta = nullptr;  // [nlanes]: row | lanes of the row << 16 on a row's first lane
    uint16_t* d_acol = nullptr;  // [4 nlanes] column of each value slot (n = the spare zero slot)
    int* d_src = nullptr;        // [4 nlanes] source of each slot: >= 0 entry, -1 zero, <= -2 1/entry(-2 - code)
    double* d_W = nullptr;       // [nsub][nnz] FP64 working factors
};

namespace {

constexpr int kGroup = 16;                 // lanes per row in the factorisation
constexpr int kRowsPerWave = 64 / kGroup;

struct KBox {
    int ex, ey, ez, n;
    int subx, suby, ownx, owny, ownz, ov;
    int nx, ny, nz;
};

__device__ __forceinline__ int kwrap(int i, int m) {
    i %= m;
    return i < 0 ? i + m : i;
}

__device__ __forceinline__ void korigin(const KBox& b, int k, int* ox, int* oy, int* oz) {
    const int kx = k % b.subx, ky = (k / b.subx) % b.suby, kz = k / (b.subx * b.suby);
    *ox = kx * b.ownx - b.ov;
    *oy = ky * b.owny - b.ov;
    *oz = b.nz > 1 ? kz * b.ownz - b.ov : 0;
}

__device__ __forceinline__ long kgidx(const KBox& b, int ox, int oy, int oz, int i) {
    const int x = i % b.ex, y = (i / b.ex) % b.ey, z = i / (b.ex * b.ey);
    const int gx = kwrap(ox + x, b.nx), gy = kwrap(oy + y, b.ny), gz = b.nz > 1 ? kwrap(oz + z, b.nz) : 0;
    return ((long)gz * b.ny + gy) * b.nx + gx;
}

__device__ __forceinline__ void wave_order() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_sched_barrier(0);
}

// LDS of the factorisation: per row group a row buffer (maxrow doubles) and a column ->
// position map of the box (n shorts, -1 where the row has no entry).
inline size_t factor_lds_bytes(int n, int maxrow) {
    return (size_t)kRowsPerWave * (sizeof(double) * maxrow + sizeof(short) * ((n + 3) & ~3));
}

template <typename T>
__global__ __launch_bounds__(64) void k_iluk_factor(const double* __restrict__ cc, const int* __restrict__ rowptr,
                                                    const uint16_t* __restrict__ col,
                                                    const int8_t* __restrict__ sten,
                                                    const uint16_t* __restrict__ diag,
                                                    const int* __restrict__ flev,
                                                    const uint16_t* __restrict__ frow, int nfl,
                                                    const int* __restrict__ src, long nvals, double* __restrict__ W,
                                                    T* __restrict__ fac, int* __restrict__ flag, KBox b,
                                                    StencilTable st, long nnz, int maxrow,
                                                    const double* __restrict__ uu) {
    extern __shared__ unsigned char smem_raw[];
    double* rbuf = reinterpret_cast<double*>(smem_raw);
    short* pmap = reinterpret_cast<short*>(rbuf + kRowsPerWave * maxrow);
    const int tid = threadIdx.x, grp = tid / kGroup, g = tid % kGroup;
    const int mstride = (b.n + 3) & ~3;
    double* row = rbuf + grp * maxrow;
    short* map = pmap + grp * mstride;
    const int k = blockIdx.x;
    int ox, oy, oz;
    korigin(b, k, &ox, &oy, &oz);
    double* Wk = W + (long)k * nnz;
    // assemble A_k on the pattern: A(i, j) = kconst(s) - d1(s) c(j) on stencil entries, 0 on fill
    for (int i = tid; i < b.n; i += 64) {
        const long gi = kgidx(b, ox, oy, oz, i);
        for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            const int s = sten[e];
            Wk[e] = s >= 0 ? subdomain_entry(st, s, cc[kgidx(b, ox, oy, oz, col[e])], uu, gi) : 0.0;
        }
    }
    for (int j = g; j < mstride; j += kGroup) map[j] = -1;
    __syncthreads();
    for (int lev = 0; lev < nfl; ++lev) {
        const int l0 = flev[lev], cnt = flev[lev + 1] - l0;
        for (int base = 0; base < cnt; base += kRowsPerWave) {
            const bool act = base + grp < cnt;
            const int i = act ? frow[l0 + base + grp] : 0;
            const int r0 = rowptr[i], len = act ? rowptr[i + 1] - r0 : 0, di = diag[i];
            for (int p = g; p < len; p += kGroup) {
                row[p] = Wk[r0 + p];
                map[col[r0 + p]] = (short)p;
            }
            wave_order();
            const int nlow = act ? di : 0;
            for (int p = 0; p < nlow; ++p) {        // kept lower entries of row i, increasing column
                const int m = col[r0 + p];
                const int m0 = rowptr[m], mlen = rowptr[m + 1] - m0, dm = diag[m];
                const double aim = row[p] / Wk[m0 + dm];
                wave_order();
                if (g == 0) row[p] = aim;
                for (int q = dm + 1 + g; q < mlen; q += kGroup) {
                    const int pi = map[col[m0 + q]];
                    if (pi >= 0) row[pi] -= aim * Wk[m0 + q];
                }
                wave_order();
            }
            for (int p = g; p < len; p += kGroup) {
                Wk[r0 + p] = row[p];
                map[col[r0 + p]] = -1;
            }
            if (act && g == 0) {
                const double piv = row[di];
                if (!(piv != 0.0) || !isfinite(piv)) *flag = 1;
            }
            wave_order();
        }
        __syncthreads();   // the level's rows are in W before the next level reads them
    }
    // the apply layout: one value per slot, from its source entry
    T* out = fac + (long)k * nvals;
    for (long v = tid; v < nvals; v += 64) {
        const int code = src[v];
        out[v] = (T)(code >= 0 ? Wk[code] : (code == -1 ? 0.0 : 1.0 / Wk[-2 - code]));
    }
}

template <typename T>
struct Vec4Of {
    using type = T __attribute__((ext_vector_type(4)));
};

// PF passes in flight; forward passes first, then backward, in execution order.  A lane slot
// holds EPL (4 or 8) consecutive entries of one row.  MAXSEG bounds the lanes of one row (a
// power of two >= the widest row's), so a row's first lane issues all of its partial-sum reads
// at once and adds them in lane order.  The pass table entry of the next fetch is read one
// fetch ahead, so the factor loads of a pass never wait for it.
template <typename T, int PF, int MAXSEG, int EPL>
__global__ __launch_bounds__(64) void k_iluk_apply(const double* __restrict__ r, double* __restrict__ z,
                                                   const T* __restrict__ fac, const int2* __restrict__ pass,
                                                   const uint32_t* __restrict__ meta,
                                                   const uint16_t* __restrict__ acol, int npass_f, int npass,
                                                   long nvals, KBox b, double* __restrict__ sum_part, int mode,
                                                   double* __restrict__ zbox) {
    using V = typename Vec4Of<T>::type;
    using C4 = unsigned short __attribute__((ext_vector_type(4)));
    constexpr int NV = EPL / 4;
    extern __shared__ unsigned char smem_raw[];
    T* x = reinterpret_cast<T*>(smem_raw);
    __shared__ T part[64];
    const int tid = threadIdx.x, k = blockIdx.x;
    int ox, oy, oz;
    korigin(b, k, &ox, &oy, &oz);
    const int zoff = b.nz > 1 ? b.ov : 0, owz = b.nz > 1 ? b.ownz : 1;
    for (int i = tid; i < b.n; i += 64) {
        const int xx = i % b.ex, yy = (i / b.ex) % b.ey, zz = i / (b.ex * b.ey);
        const bool own = xx >= b.ov && xx < b.ov + b.ownx && yy >= b.ov && yy < b.ov + b.owny && zz >= zoff &&
                         zz < zoff + owz;
        x[i] = (mode != 2 || own) ? (T)r[kgidx(b, ox, oy, oz, i)] : (T)0;
    }
    if (tid == 0) x[b.n] = (T)0;   // spare slot: the column of every padding value
    const V* F = reinterpret_cast<const V*>(fac + (long)k * nvals);
    const C4* AC = reinterpret_cast<const C4*>(acol);
    int2 ps_next = pass[0];
    V f[PF][NV];
    C4 cl[PF][NV];
    uint32_t mt[PF];
    int used[PF];
    auto fetch = [&](int p, int j) {
        const int2 ps = ps_next;                      // entry of pass min(p, npass - 1)
        ps_next = pass[min(p + 1, npass - 1)];
        const long slot = ps.x + min(tid, ps.y - 1);
        used[j] = p < npass ? ps.y : 0;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            f[j][v] = __builtin_nontemporal_load(&F[slot * NV + v]);
            cl[j][v] = AC[slot * NV + v];
        }
        mt[j] = meta[slot];
    };
#pragma unroll
    for (int j = 0; j < PF; ++j) {   // the first round computes on zeros against slot 0
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            f[j][v] = V{};
            cl[j][v] = C4{0, 0, 0, 0};
        }
        mt[j] = 0u;
        used[j] = 0;
    }
    wave_order();
    // the first round only fetches (passes -PF..-1 compute nothing), so the loop is entered with
    // no factor loads in flight
    for (int p0 = -PF; p0 < npass; p0 += PF) {
#pragma unroll
        for (int j = 0; j < PF; ++j) {
            const int p = p0 + j;
            T prod = (T)0;
#pragma unroll
            for (int v = 0; v < NV; ++v)
                prod += f[j][v][0] * x[cl[j][v][0]] + f[j][v][1] * x[cl[j][v][1]] + f[j][v][2] * x[cl[j][v][2]] +
                        f[j][v][3] * x[cl[j][v][3]];
            part[tid] = prod;
            wave_order();
            const int lanes = (int)(mt[j] >> 16);
            if (tid < used[j] && lanes > 0) {
                T pv[MAXSEG];
#pragma unroll
                for (int u = 0; u < MAXSEG; ++u) pv[u] = part[min(tid + u, 63)];
                T s = (T)0;
#pragma unroll
                for (int u = 0; u < MAXSEG; ++u) s += u < lanes ? pv[u] : (T)0;
                const int i = (int)(mt[j] & 0xFFFFu);
                // forward: x_i = r_i - sum_j l_ij x_j (unit lower factor); backward: slot 0 holds
                // 1/u_ii against the zero slot, x_i = (x_i - sum_j u_ij x_j) / u_ii
                x[i] = p < npass_f ? x[i] - s : (x[i] - s) * f[j][0][0];
            }
            wave_order();
            fetch(p + PF, j);
        }
    }
    double acc = 0.0;
    if (mode == 0) {   // left-RAS: restricted extension, the owned cells only (Eq. (23))
        const int owx = b.ownx, owy = b.owny;
        for (int e = tid; e < owx * owy * owz; e += 64) {
            const int xx = e % owx + b.ov, yy = (e / owx) % owy + b.ov, zz = e / (owx * owy) + zoff;
            const int i = (zz * b.ey + yy) * b.ex + xx;
            const double v = (double)x[i];
            z[kgidx(b, ox, oy, oz, i)] = v;
            acc += v;
        }
    } else {           // classical AS / right-RAS: the whole extended solution, added per cell later
        for (int i = tid; i < b.n; i += 64) {
            const double v = (double)x[i];
            zbox[(long)k * b.n + i] = v;
            acc += v;
        }
    }
    if (sum_part) {
        __shared__ double red[16];
        const double sum = block_sum_det(acc, red);
        if (tid == 0) sum_part[blockIdx.x] = sum;
    }
}

// ---- host: the level-k pattern and the schedules --------------------------------------------

struct HostPlan {
    int n = 0, maxrow = 0;
    std::vector<int> rowptr;
    std::vector<uint16_t> col, diag, frow;
    std::vector<int8_t> sten;
    std::vector<int> flev;
    std::vector<int2> pass;
    std::vector<uint32_t> meta;
    std::vector<uint16_t> acol;
    std::vector<int> src;
    int npass_f = 0, npass_b = 0;
    int maxseg = 1;
    int epl = 4;                 // entries per lane slot
};

// Rows of one triangle packed into passes by dependency level.  entries(i) lists the source
// codes and columns of row i's slots; rows with no slot are skipped.
template <typename Entries>
void pack_passes(const std::vector<std::vector<int>>& levels, Entries entries, HostPlan* hp, int* npass,
                 bool* ok) {
    std::vector<int> codes, cols;
    for (const auto& lev : levels) {
        int lanes_used = 0;
        int2 cur{(int)hp->meta.size(), 0};
        auto flush = [&]() {
            if (cur.y > 0) {
                hp->pass.push_back(cur);
                ++*npass;
            }
            cur = int2{(int)hp->meta.size(), 0};
            lanes_used = 0;
        };
        for (int i : lev) {
            codes.clear();
            cols.clear();
            entries(i, &codes, &cols);
            if (codes.empty()) continue;
            const int E = hp->epl;
            const int lanes = ((int)codes.size() + E - 1) / E;
            if (lanes > 64) {
                *ok = false;
                return;
            }
            if (lanes_used + lanes > 64) flush();
            hp->maxseg = std::max(hp->maxseg, lanes);
            for (int l = 0; l < lanes; ++l) {
                hp->meta.push_back(l == 0 ? ((uint32_t)i | ((uint32_t)lanes << 16)) : 0u);
                for (int e = 0; e < E; ++e) {
                    const int q = E * l + e;
                    hp->src.push_back(q < (int)codes.size() ? codes[q] : -1);
                    hp->acol.push_back((uint16_t)(q < (int)codes.size() ? cols[q] : hp->n));
                }
            }
            lanes_used += lanes;
            cur.y += lanes;
        }
        flush();
    }
}

bool build_host_plan(int ex, int ey, int ez, const StencilTable& st, int level, HostPlan* hp, std::string* err) {
    const int n = ex * ey * ez;
    if (n >= 65535) {
        *err = "ILU(k) box too large (at most 65534 cells)";
        return false;
    }
    hp->n = n;
    // pattern of A_k with the stencil index of each entry
    std::vector<std::vector<std::pair<int, int>>> A(n);
    for (int z = 0; z < ez; ++z)
        for (int y = 0; y < ey; ++y)
            for (int x = 0; x < ex; ++x) {
                const int i = (z * ey + y) * ex + x;
                for (int s = 0; s < st.S; ++s) {
                    const int xx = x + st.dx[s], yy = y + st.dy[s], zz = z + st.dz[s];
                    if (xx < 0 || xx >= ex || yy < 0 || yy >= ey || zz < 0 || zz >= ez) continue;
                    A[i].push_back({(zz * ey + yy) * ex + xx, s});
                }
                std::sort(A[i].begin(), A[i].end());
            }
    // level of fill, row by row in IKJ order
    const int INF = 1 << 30;
    std::vector<std::vector<std::pair<int, int>>> R(n);   // (column, level), sorted by column
    std::vector<int> lev(n, INF), touched;
    for (int i = 0; i < n; ++i) {
        std::priority_queue<int, std::vector<int>, std::greater<int>> low;
        touched.clear();
        for (const auto& e : A[i]) {
            lev[e.first] = 0;
            touched.push_back(e.first);
            if (e.first < i) low.push(e.first);
        }
        while (!low.empty()) {
            const int m = low.top();
            low.pop();
            const int lim = lev[m];
            for (const auto& e : R[m]) {
                const int j = e.first;
                if (j <= m) continue;
                const int nl = lim + e.second + 1;
                if (nl > level || nl >= lev[j]) continue;
                if (lev[j] == INF) {
                    touched.push_back(j);
                    if (j < i) low.push(j);
                }
                lev[j] = nl;
            }
        }
        std::sort(touched.begin(), touched.end());
        R[i].reserve(touched.size());
        for (int j : touched) {
            R[i].push_back({j, lev[j]});
            lev[j] = INF;
        }
    }
    // row-major tables
    hp->rowptr.assign(1, 0);
    for (int i = 0; i < n; ++i) {
        size_t a = 0;
        int d = -1;
        for (size_t p = 0; p < R[i].size(); ++p) {
            const int j = R[i][p].first;
            while (a < A[i].size() && A[i][a].first < j) ++a;
            const bool in_a = a < A[i].size() && A[i][a].first == j;
            hp->col.push_back((uint16_t)j);
            hp->sten.push_back((int8_t)(in_a ? A[i][a].second : -1));
            if (j == i) d = (int)p;
        }
        if (d < 0) {
            *err = "ILU(k) pattern without a diagonal";
            return false;
        }
        hp->diag.push_back((uint16_t)d);
        hp->rowptr.push_back((int)hp->col.size());
        hp->maxrow = std::max(hp->maxrow, (int)R[i].size());
    }
    // dependency levels: forward (= factorisation) and backward
    std::vector<int> lf(n, 0), lb(n, 0);
    int nf = 0, nb = 0;
    for (int i = 0; i < n; ++i) {
        int l = 0;
        for (int p = hp->rowptr[i]; p < hp->rowptr[i] + hp->diag[i]; ++p) l = std::max(l, lf[hp->col[p]] + 1);
        lf[i] = l;
        nf = std::max(nf, l + 1);
    }
    for (int i = n - 1; i >= 0; --i) {
        int l = 0;
        for (int p = hp->rowptr[i] + hp->diag[i] + 1; p < hp->rowptr[i + 1]; ++p) l = std::max(l, lb[hp->col[p]] + 1);
        lb[i] = l;
        nb = std::max(nb, l + 1);
    }
    std::vector<std::vector<int>> F(nf), B(nb);
    for (int i = 0; i < n; ++i) {
        F[lf[i]].push_back(i);
        B[lb[i]].push_back(i);
    }
    hp->flev.assign(1, 0);
    for (const auto& v : F) {
        for (int i : v) hp->frow.push_back((uint16_t)i);
        hp->flev.push_back((int)hp->frow.size());
    }
    // entries per lane: four, or eight when a row would need more than 64 lanes of four
    int longest = 0;
    for (int i = 0; i < n; ++i)
        longest = std::max({longest, (int)hp->diag[i], hp->rowptr[i + 1] - hp->rowptr[i] - hp->diag[i]});
    hp->epl = longest > 256 ? 8 : 4;
    bool ok = true;
    pack_passes(F, [&](int i, std::vector<int>* codes, std::vector<int>* cols) {
        for (int p = hp->rowptr[i]; p < hp->rowptr[i] + hp->diag[i]; ++p) {
            codes->push_back(p);
            cols->push_back(hp->col[p]);
        }
    }, hp, &hp->npass_f, &ok);
    if (ok)
        pack_passes(B, [&](int i, std::vector<int>* codes, std::vector<int>* cols) {
            const int d = hp->rowptr[i] + hp->diag[i];
            codes->push_back(-2 - d);    // reciprocal pivot, against the zero slot
            cols->push_back(n);
            for (int p = d + 1; p < hp->rowptr[i + 1]; ++p) {
                codes->push_back(p);
                cols->push_back(hp->col[p]);
            }
        }, hp, &hp->npass_b, &ok);
    if (!ok) {
        *err = "ILU(k) row longer than 512 entries";
        return false;
    }
    return true;
}

template <typename T>
hipError_t upload(T** d, const std::vector<T>& h) {
    hipError_t e = hipMalloc((void**)d, sizeof(T) * std::max<size_t>(h.size(), 1));
    if (e != hipSuccess) {
        *d = nullptr;
        return e;
    }
    return h.empty() ? hipSuccess : hipMemcpy(*d, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice);
}

KBox make_kbox(const pfc_ctx* c) {
    KBox b;
    b.ex = c->dec.ext[0];
    b.ey = c->dec.ext[1];
    b.ez = c->g.dim == 3 ? c->dec.ext[2] : 1;
    b.n = c->dec.next;
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

constexpr int kApplyPF = 3;

}  // namespace

void iluk_plan_free(IlukPlan* p) {
    if (!p) return;
    void* ptrs[] = {p->d_rowptr, p->d_col, p->d_sten, p->d_diag, p->d_flev, p->d_frow,
                    p->d_pass, p->d_meta, p->d_acol, p->d_src, p->d_W};
    for (void* q : ptrs)
        if (q) hipFree(q);
    delete p;
}

pfc_status iluk_plan_create(pfc_ctx* c, int level, std::string* err) {
    HostPlan hp;
    const int ex = c->dec.ext[0], ey = c->dec.ext[1], ez = c->g.dim == 3 ? c->dec.ext[2] : 1;
    if (!build_host_plan(ex, ey, ez, c->st, level, &hp, err)) return PFC_EINVAL;
    const size_t esz = c->opts.precond_fp32 ? 4 : 8;
    if (esz * ((size_t)hp.n + 1) + 64 * esz > 150 * 1024) {
        *err = "ILU(k) box vector too large for LDS";
        return PFC_EINVAL;
    }
    if (factor_lds_bytes(hp.n, hp.maxrow) > 150 * 1024) {
        *err = "ILU(k) rows too long for the factorisation's LDS";
        return PFC_EINVAL;
    }
    IlukPlan* p = new IlukPlan();
    p->n = hp.n;
    p->nnz = (long)hp.col.size();
    p->maxrow = hp.maxrow;
    p->nfl = (int)hp.flev.size() - 1;
    p->npass_f = hp.npass_f;
    p->npass_b = hp.npass_b;
    p->nlanes = (long)hp.meta.size();
    p->maxseg = hp.maxseg;
    p->epl = hp.epl;
    bool ok = upload(&p->d_rowptr, hp.rowptr) == hipSuccess && upload(&p->d_col, hp.col) == hipSuccess &&
              upload(&p->d_sten, hp.sten) == hipSuccess && upload(&p->d_diag, hp.diag) == hipSuccess &&
              upload(&p->d_flev, hp.flev) == hipSuccess && upload(&p->d_frow, hp.frow) == hipSuccess &&
              upload(&p->d_pass, hp.pass) == hipSuccess && upload(&p->d_meta, hp.meta) == hipSuccess &&
              upload(&p->d_acol, hp.acol) == hipSuccess && upload(&p->d_src, hp.src) == hipSuccess &&
              hipMalloc((void**)&p->d_W, sizeof(double) * (size_t)c->dec.nsub * p->nnz) == hipSuccess;
    if (!ok) {
        iluk_plan_free(p);
        *err = "out of device memory for the ILU(k) tables";
        return PFC_ENOMEM;
    }
    c->iluk = p;
    c->fac_elems = (size_t)c->dec.nsub * p->epl * p->nlanes;
    return PFC_OK;
}

void iluk_plan_stats(const IlukPlan* p, long* nnz, int* fac_levels, int* passes_f, int* passes_b, long* slots) {
    *nnz = p->nnz;
    *fac_levels = p->nfl;
    *passes_f = p->npass_f;
    *passes_b = p->npass_b;
    *slots = (long)p->epl * p->nlanes;
}

hipError_t launch_iluk_factor(pfc_ctx* c, const StencilTable& st) {
    const IlukPlan* p = c->iluk;
    const KBox b = make_kbox(c);
    const size_t sh = factor_lds_bytes(p->n, p->maxrow);
    const long nvals = (long)p->epl * p->nlanes;
    if (c->opts.precond_fp32)
        hipLaunchKernelGGL(k_iluk_factor<float>, dim3(c->dec.nsub), dim3(64), sh, c->stream, c->d_c, p->d_rowptr,
                           p->d_col, p->d_sten, p->d_diag, p->d_flev, p->d_frow, p->nfl, p->d_src, nvals, p->d_W,
                           (float*)c->d_fac, c->d_flag, b, st, p->nnz, p->maxrow, (const double*)c->d_u);
    else
        hipLaunchKernelGGL(k_iluk_factor<double>, dim3(c->dec.nsub), dim3(64), sh, c->stream, c->d_c, p->d_rowptr,
                           p->d_col, p->d_sten, p->d_diag, p->d_flev, p->d_frow, p->nfl, p->d_src, nvals, p->d_W,
                           (double*)c->d_fac, c->d_flag, b, st, p->nnz, p->maxrow, (const double*)c->d_u);
    return hipGetLastError();
}

template <typename T, int MAXSEG, int EPL>
hipError_t launch_iluk_apply_t(pfc_ctx* c, const double* r, double* z, double* sum_part) {
    const IlukPlan* p = c->iluk;
    const KBox b = make_kbox(c);
    return launch_k(c, k_iluk_apply<T, kApplyPF, MAXSEG, EPL>, dim3(c->dec.nsub), dim3(64), sizeof(T) * (p->n + 1),
                    r, z, (const T*)c->d_fac, (const int2*)p->d_pass, (const uint32_t*)p->d_meta,
                    (const uint16_t*)p->d_acol, p->npass_f, p->npass_f + p->npass_b, (long)EPL * p->nlanes, b,
                    sum_part, c->opts.ras_kind, c->d_zbox);
}

template <typename T, int EPL>
hipError_t launch_iluk_apply_e(pfc_ctx* c, const double* r, double* z, double* sum_part) {
    const int m = c->iluk->maxseg;
    if (m <= 4) return launch_iluk_apply_t<T, 4, EPL>(c, r, z, sum_part);
    if (m <= 8) return launch_iluk_apply_t<T, 8, EPL>(c, r, z, sum_part);
    if (m <= 16) return launch_iluk_apply_t<T, 16, EPL>(c, r, z, sum_part);
    if (m <= 32) return launch_iluk_apply_t<T, 32, EPL>(c, r, z, sum_part);
    return launch_iluk_apply_t<T, 64, EPL>(c, r, z, sum_part);
}

template <typename T>
hipError_t launch_iluk_apply_s(pfc_ctx* c, const double* r, double* z, double* sum_part) {
    return c->iluk->epl == 8 ? launch_iluk_apply_e<T, 8>(c, r, z, sum_part) : launch_iluk_apply_e<T, 4>(c, r, z, sum_part);
}

hipError_t launch_iluk_apply(pfc_ctx* c, const double* r, double* z, double* sum_part) {
    return c->opts.precond_fp32 ? launch_iluk_apply_s<float>(c, r, z, sum_part)
                                : launch_iluk_apply_s<double>(c, r, z, sum_part);
}

template <typename T, int EPL>
hipError_t set_apply_limits() {
    const void* fs[] = {(const void*)k_iluk_apply<T, kApplyPF, 4, EPL>, (const void*)k_iluk_apply<T, kApplyPF, 8, EPL>,
                        (const void*)k_iluk_apply<T, kApplyPF, 16, EPL>, (const void*)k_iluk_apply<T, kApplyPF, 32, EPL>,
                        (const void*)k_iluk_apply<T, kApplyPF, 64, EPL>};
    for (const void* f : fs) {
        const hipError_t e = set_dynamic_lds_limit(f);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t set_iluk_lds_limits() {
    hipError_t e = set_dynamic_lds_limit((const void*)k_iluk_factor<float>);
    if (e == hipSuccess) e = set_dynamic_lds_limit((const void*)k_iluk_factor<double>);
    if (e == hipSuccess) e = set_apply_limits<float, 4>();
    if (e == hipSuccess) e = set_apply_limits<float, 8>();
    if (e == hipSuccess) e = set_apply_limits<double, 4>();
    if (e == hipSuccess) e = set_apply_limits<double, 8>();
    return e;
}

}  // namespace pfc
