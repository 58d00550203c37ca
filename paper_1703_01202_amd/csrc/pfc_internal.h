// Internal declarations of libpfc (not part of the C ABI).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "../../include/pfc.h"
#include "../../include/pfc_net.h"

namespace pfc {

constexpr int kMaxStencil = 63;        // composite stencil |dx|+|dy|+|dz| <= 3 in 3-D
constexpr int kRedBlocks = 512;        // fixed reduction grid: deterministic partial sums
constexpr int kRedThreads = 256;

// Mesh: n[0] = nx (fastest), spacing h[a] = L[a]/n[a].
struct Geom {
    int dim;
    int nx, ny, nz;
    long N;
    double ihx2, ihy2, ihz2;           // 1/h^2 per axis (ihz2 = 0 in 2-D)
    double cell_volume;
};

// Constant-coefficient stencil of the Jacobian in one subdomain row, in natural
// (z, y, x lexicographic) order of the offsets.  J_ij = kconst[s] - d1[s] * c_j with
// j = i + offset s (Sec. 4, Eq. (19) written entry by entry).
struct StencilTable {
    int S;                             // 25 (2-D) or 63 (3-D)
    int diag;                          // index of the zero offset
    int8_t dx[kMaxStencil], dy[kMaxStencil], dz[kMaxStencil];
    double kconst[kMaxStencil];
    double d1[kMaxStencil];
    double inv_dt;                     // the 1/dt that kconst holds at the zero offset
};

// Entry (i, j) of a subdomain matrix, offset s: kconst(s) - d1(s) c_j; with a variable mobility
// (u = (Phi + phi)/2 given) the spatial part of row i is scaled by the node mobility
// M_i = 1 - u_i^2 at its cell gi: the subdomain operator freezes M at the row's cell, a
// preconditioner for nabla . M nabla.
__host__ __device__ inline double subdomain_entry(const StencilTable& t, int s, double cj, const double* u, long gi) {
    const double a = t.kconst[s] - t.d1[s] * cj;
    if (!u) return a;
    const double m = 1.0 - u[gi] * u[gi];
    const double d = s == t.diag ? t.inv_dt : 0.0;
    return d + m * (a - d);
}

// Overlapping decomposition: equal boxes of own[a] cells, extended by `ov` layers.
struct Decomp {
    int sub[3];
    int own[3];
    int ext[3];
    int ov;
    int nsub;
    int next;                          // cells per extended box
};

// Event-pair timer for per-kernel durations on the context stream.  A region of one kernel
// hands its event pair to that kernel's launch (launch_k), whose dispatch records both, so
// timing adds no packets to the queue; regions of several kernels record the events around
// them.
// Elapsed times are read one synchronisation late: the pairs completed at the previous
// synchronisation are read just before the next one waits, while the GPU still runs the work
// enqueued in between, so the queries stay off the critical path.
struct KernelTimer {
    std::vector<hipEvent_t> pool;
    std::vector<int> free;                       // unused pairs (index of the start event)
    std::vector<std::pair<int, int>> pending;   // (start idx, kind) recorded since the last synchronisation
    std::vector<std::pair<int, int>> done;      // complete at the last synchronisation, not yet read
    long count[4] = {0, 0, 0, 0};
    double total_ms[4] = {0, 0, 0, 0};
    bool ext = false;                            // the open region is timed by its launch
    mutable hipEvent_t launch_ev[2] = {nullptr, nullptr};   // pair for the next launch_k
};

// Inference buffers of one solver context for the learned guess (the network's parameters
// are shared read-only, so contexts on different streams and threads can use one network).
struct NetWork {
    float* x = nullptr;    // input planes [2][N]
    float* a = nullptr;    // second-layer activations, 32 channels x N (16 bytes per 4 channels),
                           // then the output layer's 9 per-tap sum planes of N
    float* b1c = nullptr;  // layer-1 bias with the step-size term (32 floats)
};
constexpr int kNetWorkFloats = 32 + 9;   // floats of NetWork::a per cell

struct IlukPlan;   // ILU(k) pattern, schedules and working factors (ras_iluk.hip)

}  // namespace pfc

struct pfc_ctx {
    pfc_grid grid;
    pfc_model model;
    pfc_opts opts;
    hipStream_t stream = nullptr;
    pfc::Geom g;
    pfc::Decomp dec;
    pfc::StencilTable st;              // Jacobian stencil at the last factorisation (offsets fixed)
    std::string err;

    // ILU(0) level schedule, shared by all boxes (same shape): points sorted by level
    int nlev = 0;
    int ilu_cells_per_lane = 1;        // C of the ILU apply: cells of the widest level / 64, rounded up
    int* d_level_ptr = nullptr;        // [nlev + 1]
    int* d_level_pts = nullptr;        // [next], packed coords x | y << 8 | z << 16

    // factors
    double* d_work = nullptr;          // ILU natural-layout workspace / LU window (FP64)
    void* d_fac = nullptr;             // packed factors (double or float)
    size_t fac_elems = 0;
    int* d_flag = nullptr;             // pivot failure flag
    double* d_zbox = nullptr;          // per-box extended solutions (classical AS, right-RAS)
    int lu_W = 0, lu_H = 0;            // exact LU: block size (box x-extent) and block rows
    pfc::IlukPlan* iluk = nullptr;     // ILU(k): pattern and schedules shared by the boxes

    // vectors (N doubles each)
    double* d_c = nullptr;             // Jacobian coefficient at the current iterate
    double* d_F = nullptr;
    double* d_X = nullptr;             // Newton iterate
    double* d_T = nullptr;             // line-search trial
    double* d_S = nullptr;             // Newton direction
    double* d_w = nullptr;
    double* d_r = nullptr;
    double* d_V = nullptr;             // (restart+1) * N
    double* d_Z = nullptr;             // restart * N
    double* d_prev = nullptr;          // phi^(n-1) for extrapolation
    double* d_tmp3 = nullptr;          // multi-pass temporaries (2 * N): 3-D, variable mobility, Neumann
    double* d_u = nullptr;             // variable mobility: u = (Phi + phi)/2 of the iterate ...
    double* d_mu = nullptr;            // ... and its mu_d, for the Jacobian action

    // reductions
    double* d_part = nullptr;          // partials summed on the device (Gram-Schmidt, apply sums)
    double* d_scal = nullptr;          // device scalars, then partials summed on the host
    double* h_pin = nullptr;           // pinned host mirror of d_scal (mapped, coherent)
    double* d_hpin = nullptr;          // h_pin as seen by kernels: values only the host reads
                                       // (norm partials, Hessenberg column, apply means) are
                                       // written here directly, with no copy
    double* h_y = nullptr;             // pinned staging of the FGMRES update coefficients
    int n_scal = 0;                    // doubles in d_scal / h_pin

    // time history
    long step = 0;
    double F_n = 0, F_nm1 = 0, dt_nm1 = 0, t = 0;
    bool have_prev = false, have_energy = false;

    // factorisation reuse across time steps (opts.precond_lag)
    bool fac_valid = false;
    double fac_dt = 0.0;               // dt the factors were built with
    long fac_step = -1;                // time step that built them
    double fac_gpn = 0.0;              // GMRES iterations per Newton step of that time step
    double last_gpn = 0.0;             // ... of the last time step

    // learned initial guess (pfc_attach_net); the network is not owned
    pfc_net* net = nullptr;
    double net_scale[6] = {1.0, 1.0, 1.0, 1.0, 0.0, 0.0};   // s_a, s_b, s_o, s_c, beta, gamma
    double net_dt[3] = {0.0, 0.0, 0.0};      // dt_ref, and the range [dt_lo, dt_hi] it is used in
    pfc::NetWork netw;                       // inference buffers

    // HIP graphs of the Arnoldi steps (opts.use_graph): one per Krylov index, valid for arn_dt
    std::vector<hipGraphExec_t> arn_graph;
    double arn_dt = -1.0;
    long graph_launches = 0;

    pfc::KernelTimer timer;
};

namespace pfc {

template <typename Tup, size_t... I>
inline void arg_ptrs(Tup& t, void** p, std::index_sequence<I...>) {
    ((p[I] = (void*)&std::get<I>(t)), ...);
}

// Launch kern on c's stream.  If a timed region left an event pair for it, the launch goes
// through hipExtLaunchKernel, whose dispatch records the start and stop events itself.
template <typename... K, typename... A>
inline hipError_t launch_k(const pfc_ctx* c, void (*kern)(K...), dim3 grid, dim3 block, size_t sh, A... args) {
    hipEvent_t* ev = c->timer.launch_ev;
    if (!ev[0]) {
        hipLaunchKernelGGL(kern, grid, block, sh, c->stream, args...);
        return hipGetLastError();
    }
    const hipEvent_t e0 = ev[0], e1 = ev[1];
    ev[0] = ev[1] = nullptr;
    std::tuple<K...> t{static_cast<K>(args)...};
    void* p[sizeof...(K) > 0 ? sizeof...(K) : 1];
    arg_ptrs(t, p, std::index_sequence_for<K...>{});
    return hipExtLaunchKernel(reinterpret_cast<const void*>(kern), grid, block, p, sh, c->stream, e0, e1, 0);
}

// Allow a kernel the whole 160 KB LDS of a gfx950 CU minus its static LDS.
inline hipError_t set_dynamic_lds_limit(const void* f) {
    hipFuncAttributes a;
    hipError_t e = hipFuncGetAttributes(&a, f);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - (int)a.sharedSizeBytes);
}

// ---- stencil kernels (stencil.hip) ----
// Reductions leave per-block partials (device_reduce.h); partial_count gives their number.
bool fused2d(const pfc_ctx* c);                 // 2-D, M = 1, periodic: the single-kernel stencils
bool fused3d(const pfc_ctx* c);                 // 3-D, M = 1, periodic: the single-kernel stencils
int residual_partial_count(const pfc_ctx* c);   // blocks of the residual kernel
// The 2-D residual kernel outside a context: grid nx x ny with 1/h^2 per axis, on stream s;
// writes residual2d_blocks(nx, ny) (at most 1024) partial sums of F^2 to norm_part.
int residual2d_blocks(int nx, int ny);
hipError_t launch_residual2d_plain(hipStream_t s, int nx, int ny, double ihx2, double ihy2, double gamma,
                                   double dt, const double* Phi, const double* phi, const double* src, double* F,
                                   double* norm_part);
int energy_partial_count(const pfc_ctx* c);     // blocks of the energy kernel (two partials each)
// F and per-block partials of ||F||^2 (norm_part) and of ||Phi||^2 (xnorm_part); both nullable
hipError_t launch_residual(const pfc_ctx* c, const double* Phi, const double* phi, double dt,
                           const double* src, double* F, double* norm_part, double* xnorm_part);
hipError_t launch_coef(const pfc_ctx* c, const double* Phi, const double* phi, double* cbuf);
// Jv of (v - s), s = shift_scale * sum(shift_part[0..shift_n)) (no shift if shift_part is null);
// s is stored in *shift_out when given.
hipError_t launch_jv(const pfc_ctx* c, const double* v, const double* cbuf, double dt, const double* shift_part,
                     int shift_n, double shift_scale, double* shift_out, double* Jv);
// energy and mass partials of phi; with acc_phi also acc_prev <- acc_phi, acc_phi <- phi
hipError_t launch_energy(const pfc_ctx* c, const double* phi, double* part2, double* acc_phi = nullptr,
                         double* acc_prev = nullptr);

// ---- BLAS-1 (blas.hip) ----
hipError_t launch_dot(hipStream_t s, const double* x, const double* y, long n, double* partials);
hipError_t launch_reduce_rows_n(hipStream_t s, const double* partials, int rows, int count, double* out,
                                double scale);
hipError_t launch_multidot(hipStream_t s, const double* V, long ld, int k, const double* w, long n,
                           double* partials);
hipError_t launch_maxpy(hipStream_t s, const double* V, long ld, int k, const double* coef_part, int coef_n,
                        double sign, double* w, long n, double* norm_part, double* coef_out, bool assign = false,
                        const double* shift_part = nullptr, int shift_n = 0, double shift_scale = 0.0);
hipError_t launch_maxpy_dot(hipStream_t s, const double* V, long ld, int k, const double* coef_part, int coef_n,
                            double sign, double* w, long n, double* dot_part, double* coef_out);
hipError_t launch_normalize(hipStream_t s, double* w, const double* part, int np, long n, double* h_out);
hipError_t launch_axpby(hipStream_t s, double a, const double* x, double b, const double* y,
                        double* out, long n);
hipError_t launch_scale(hipStream_t s, const double* x, double a, double* out, long n);
hipError_t launch_shift(hipStream_t s, double* x, const double* part, int np, double scale, long n);
hipError_t launch_extrap(hipStream_t s, const double* phi, const double* prev, double ratio,
                         double* out, long n);

// ---- Schwarz preconditioner (ras_ilu.hip, ras_lu.hip) ----
// sum_part (nullable): one partial per subdomain of the sum of the output z.
void build_stencil_table(const Geom& g, double gamma, double dt, StencilTable* t);
hipError_t launch_ilu_factor(pfc_ctx* c, const StencilTable& t);
hipError_t launch_ilu_apply(pfc_ctx* c, const double* r, double* z, double* sum_part);
// packed ILU(0) factor elements per cell for a stencil of S offsets
int ilu_fac_elems_per_cell(int S);
// ---- ILU(k) (ras_iluk.hip) ----
pfc_status iluk_plan_create(pfc_ctx* c, int level, std::string* err);   // sets c->iluk, c->fac_elems
void iluk_plan_free(IlukPlan* p);
void iluk_plan_stats(const IlukPlan* p, long* nnz, int* fac_levels, int* passes_f, int* passes_b, long* slots);
hipError_t launch_iluk_factor(pfc_ctx* c, const StencilTable& st);
hipError_t launch_iluk_apply(pfc_ctx* c, const double* r, double* z, double* sum_part);
hipError_t set_iluk_lds_limits();
constexpr int kIluMaxCellsPerLane = 3;   // widest wavefront level an ILU(0) box may have: 64 * this
hipError_t launch_lu_factor(pfc_ctx* c, const StencilTable& t);
hipError_t launch_lu_apply(pfc_ctx* c, const double* r, double* z, double* sum_part);
// z = sum over the boxes covering each cell of their extended solutions in zbox (classical AS
// and right-RAS), in a fixed order per cell
hipError_t launch_schwarz_sum(const pfc_ctx* c, const double* zbox, double* z);

// ---- learned initial guess (net.hip) ----
// X = phi + out_scale net(x; c), x[0] = (phi - mean) inv_sa (mean from sum_part[0..np)),
// x[1] = ratio (phi - prev) inv_x1, c = cond, using the buffers w; before the mass shift.  diff_part (nullable) receives kRedBlocks partial sums of phi - X for
// that shift.  The network must be prepared (net_prepare) and not trained meanwhile.
pfc_status net_guess(pfc_net* net, hipStream_t s, const double* phi, const double* prev, int ny, int nx,
                     double ratio, double cond, double inv_sa, double inv_x1, double out_scale,
                     const double* sum_part, int np, const NetWork& w, double* X, double* diff_part);
// Round and pack the current parameters for inference (synchronises the network's stream).
pfc_status net_prepare(pfc_net* net);
const char* net_error(const pfc_net* net);

}  // namespace pfc
