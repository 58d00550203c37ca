// Host driver of the Newton-Krylov-Schwarz solve (Sec. 4) and the time loop with
// adaptive steps (Sec. 3, Eq. (16)), behind the C ABI of include/pfc.h.
//
// Device work is enqueued on the context stream; the host reads back one small
// vector per Arnoldi step (Hessenberg column and norm) and one norm per Newton or
// line-search evaluation, and keeps the Hessenberg matrix and Givens rotations.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "pfc_internal.h"

namespace pfc {
int residual_partial_count(const pfc_ctx* c);
int energy_partial_count(const pfc_ctx* c);
void build_ilu_schedule(const pfc_ctx* c, std::vector<int>* lptr, std::vector<int>* lpts);
hipError_t set_ilu_lds_limits();
hipError_t set_lu_lds_limits();
size_t lu_factor_lds_bytes(int W);
size_t lu_work_blocks(int W);
size_t lu_factor_elems_per_block_row(int W);
}  // namespace pfc

using namespace pfc;

namespace {

// d_scal: scalar slots, then (from SC_P) partials that the host sums after one copy
// Layout of d_scal / h_pin in doubles.  The Gram-Schmidt coefficients of Arnoldi step j go to
// half j % 2 of their region, so two steps can be in flight before the host reads them.
constexpr int kScal = 464;
constexpr int SC_H = 8;         // first Gram-Schmidt coefficients (2 x 64)
constexpr int SC_H2 = 136;      // second pass coefficients (2 x 64)
constexpr int SC_Y = 264;       // update coefficients (64)
constexpr int SC_SHIFT = 328;   // shift of the update
constexpr int SC_M = 336;       // means of the preconditioned vectors z_j (64)
constexpr int SC_HN = 400;      // norms of the new basis vectors, h_(j+1,j) (64)
constexpr int SC_P = kScal;     // partials: host-summed ones in h_pin, device-summed norms in d_scal
inline int sc_half(int j) { return 64 * (j & 1); }

// d_part: partials summed by the next kernel on the device
//   [0, 64 R)        first Gram-Schmidt pass, row j = partials of v_j . w  (R = kRedBlocks)
//   [64 R, 128 R)    second pass
//   [128 R, ...)     row j (nsub partials) = per-subdomain sums of z_j, j < 64
inline double* part_md1(pfc_ctx* c) { return c->d_part; }
inline double* part_md2(pfc_ctx* c) { return c->d_part + 64L * kRedBlocks; }
inline double* part_apply(pfc_ctx* c, int j) { return c->d_part + 128L * kRedBlocks + (long)j * c->dec.nsub; }

// Sum of np partials copied back to h_pin[SC_P ...], in index order.
double host_sum(const pfc_ctx* c, int off, int np) {
    double s = 0.0;
    for (int i = 0; i < np; ++i) s += c->h_pin[SC_P + off + i];
    return s;
}

#define HIPCHK(expr)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess) {                                                          \
            c->err = std::string(#expr) + ": " + hipGetErrorString(e_);                  \
            return PFC_EHIP;                                                             \
        }                                                                                \
    } while (0)

#define CHK(expr)                          \
    do {                                   \
        pfc_status s_ = (expr);            \
        if (s_ != PFC_OK) return s_;       \
    } while (0)

pfc_status fail(pfc_ctx* c, pfc_status s, const std::string& msg) {
    if (c) c->err = msg;
    return s;
}

// ---- per-kernel timing ----
// one_kernel: the region is a single launch_k launch, which records the events itself
void timer_begin(pfc_ctx* c, int kind, int* slot, bool one_kernel = false) {
    *slot = -1;
    if (!(c->opts.timing & (1 << kind))) return;
    auto& T = c->timer;
    if (T.free.empty()) {
        // timing-only events: no system-scope fence (cache writeback and invalidation) when
        // they complete; the host reads results after stream synchronisations, not events
        hipEvent_t e0, e1;
        if (hipEventCreateWithFlags(&e0, hipEventDisableSystemFence) != hipSuccess) return;
        if (hipEventCreateWithFlags(&e1, hipEventDisableSystemFence) != hipSuccess) {
            (void)hipEventDestroy(e0);
            return;
        }
        T.free.push_back((int)T.pool.size());
        T.pool.push_back(e0);
        T.pool.push_back(e1);
    }
    *slot = T.free.back();
    T.free.pop_back();
    T.ext = one_kernel;
    if (one_kernel) {
        T.launch_ev[0] = T.pool[*slot];
        T.launch_ev[1] = T.pool[*slot + 1];
    } else {
        hipEventRecord(T.pool[*slot], c->stream);
    }
    T.pending.push_back({*slot, kind});
}

void timer_end(pfc_ctx* c, int slot) {
    if (slot < 0) return;
    auto& T = c->timer;
    if (!T.ext) {
        hipEventRecord(T.pool[slot + 1], c->stream);
    } else if (T.launch_ev[0]) {   // no launch took the pair: the region is not counted
        T.launch_ev[0] = T.launch_ev[1] = nullptr;
        T.pending.pop_back();
        T.free.push_back(slot);
    }
    T.ext = false;
}

// add the elapsed times of completed pairs to the totals and free the pairs
void timer_read(pfc_ctx* c, std::vector<std::pair<int, int>>& list) {
    auto& T = c->timer;
    for (auto& pr : list) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, T.pool[pr.first], T.pool[pr.first + 1]) == hipSuccess) {
            T.total_ms[pr.second] += ms;
            T.count[pr.second] += 1;
        }
        T.free.push_back(pr.first);
    }
    list.clear();
}

pfc_status sync(pfc_ctx* c) {
    timer_read(c, c->timer.done);   // complete since the last synchronisation
    HIPCHK(hipStreamSynchronize(c->stream));
    c->timer.done.swap(c->timer.pending);
    return PFC_OK;
}

// every recorded pair read (synchronises)
pfc_status timer_drain(pfc_ctx* c) {
    HIPCHK(hipStreamSynchronize(c->stream));
    timer_read(c, c->timer.done);
    timer_read(c, c->timer.pending);
    return PFC_OK;
}

// Euclidean norm of a device vector (synchronises).
pfc_status norm2(pfc_ctx* c, const double* x, double* out) {
    HIPCHK(launch_dot(c->stream, x, x, c->g.N, c->d_hpin + SC_P));   // partials straight to the host
    CHK(sync(c));
    *out = std::sqrt(host_sum(c, 0, kRedBlocks));
    if (!std::isfinite(*out)) return fail(c, PFC_ENAN, "non-finite norm");
    return PFC_OK;
}

// x += scale * sum(y) with the sum formed on the device (no synchronisation)
pfc_status shift_by_sum(pfc_ctx* c, double* x, const double* y, double scale) {
    double* part = part_md1(c);
    HIPCHK(launch_dot(c->stream, y, nullptr, c->g.N, part));
    HIPCHK(launch_shift(c->stream, x, part, kRedBlocks, scale, c->g.N));
    return PFC_OK;
}

pfc_status residual_impl(pfc_ctx* c, const double* Phi, const double* phi, double dt, const double* src,
                         double* F, double* nrm) {
    int ts;
    timer_begin(c, 1, &ts, fused2d(c) || fused3d(c));
    HIPCHK(launch_residual(c, Phi, phi, dt, src, F, nrm ? c->d_hpin + SC_P : nullptr, nullptr));
    timer_end(c, ts);
    if (!nrm) return PFC_OK;
    const int np = residual_partial_count(c);
    CHK(sync(c));
    *nrm = std::sqrt(host_sum(c, 0, np));
    if (!std::isfinite(*nrm)) return fail(c, PFC_ENAN, "non-finite residual norm");
    return PFC_OK;
}

// out = J (v - s) with s = mean of v formed from the apply's per-subdomain sums in
// shift_part (nullable), stored in *shift_out.
pfc_status jv_impl(pfc_ctx* c, const double* v, double dt, const double* shift_part, double* shift_out,
                   double* out) {
    int ts;
    timer_begin(c, 2, &ts, fused2d(c) || fused3d(c));
    HIPCHK(launch_jv(c, v, c->d_c, dt, shift_part, c->dec.nsub, 1.0 / (double)c->g.N, shift_out, out));
    timer_end(c, ts);
    return PFC_OK;
}

pfc_status setup_impl(pfc_ctx* c, const double* Phi, const double* phi, double dt) {
    HIPCHK(launch_coef(c, Phi, phi, c->d_c));
    StencilTable st;
    build_stencil_table(c->g, c->model.gamma, dt, &st);
    c->st = st;
    HIPCHK(hipMemsetAsync(c->d_flag, 0, sizeof(int), c->stream));
    int ts;
    timer_begin(c, 3, &ts);
    if (c->opts.sub_solver == PFC_SUB_LU)
        HIPCHK(launch_lu_factor(c, st));
    else if (c->opts.sub_solver == PFC_SUB_ILUK)
        HIPCHK(launch_iluk_factor(c, st));
    else
        HIPCHK(launch_ilu_factor(c, st));
    timer_end(c, ts);
    int flag = 0;
    HIPCHK(hipMemcpyAsync(c->h_pin, c->d_flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    CHK(sync(c));
    std::memcpy(&flag, c->h_pin, sizeof(int));
    if (flag) {
        c->fac_valid = false;
        return fail(c, PFC_EPIVOT, "zero or non-finite pivot in a subdomain factorisation");
    }
    c->fac_valid = true;
    c->fac_dt = dt;
    c->fac_step = c->step;
    return PFC_OK;
}

// May the factors of an earlier time step precondition this one (opts.precond_lag)?
bool may_reuse_factors(const pfc_ctx* c, double dt) {
    const int lag = c->opts.precond_lag;
    if (lag <= 0 || !c->fac_valid || c->fac_step < 0) return false;
    if (c->step - c->fac_step >= lag) return false;
    if (std::fabs(dt - c->fac_dt) > 0.2 * c->fac_dt) return false;
    return c->last_gpn <= 2.0 * c->fac_gpn + 1.0;
}

// z = H^-1 r; with sum_part the apply kernel also leaves one partial sum of z per subdomain.
// Classical AS and right-RAS leave each box's extended solution in d_zbox, added per cell by
// a second kernel.
pfc_status apply_raw(pfc_ctx* c, const double* r, double* z, double* sum_part) {
    const bool left = c->opts.ras_kind == PFC_RAS_LEFT;
    int ts;
    timer_begin(c, 0, &ts, left);
    if (c->opts.sub_solver == PFC_SUB_LU)
        HIPCHK(launch_lu_apply(c, r, z, sum_part));
    else if (c->opts.sub_solver == PFC_SUB_ILUK)
        HIPCHK(launch_iluk_apply(c, r, z, sum_part));
    else
        HIPCHK(launch_ilu_apply(c, r, z, sum_part));
    if (!left) HIPCHK(launch_schwarz_sum(c, c->d_zbox, z));
    timer_end(c, ts);
    return PFC_OK;
}

pfc_status apply_impl(pfc_ctx* c, const double* r, double* z) {
    const bool proj = c->opts.mass_project;
    CHK(apply_raw(c, r, z, proj ? part_apply(c, 0) : nullptr));
    if (proj) HIPCHK(launch_shift(c->stream, z, part_apply(c, 0), c->dec.nsub, -1.0 / (double)c->g.N, c->g.N));
    return PFC_OK;
}

// One Arnoldi step j of FGMRES, enqueued: z_j = H^-1 v_j, w = J z_j, two classical
// Gram-Schmidt passes against v_0..v_j (norm partials fused), and v_(j+1) = w / ||w|| with
// the norm summed on the device.  The values the host needs (mean of z_j, both coefficient
// columns, h_(j+1,j)) are written by the kernels straight into the mapped host buffer, so the
// step has no copy and needs no host value: the next step can be enqueued before the host
// has read this one.
pfc_status enqueue_arnoldi_step(pfc_ctx* c, int j, double dt) {
    const long N = c->g.N;
    const bool proj = c->opts.mass_project;
    double* V = c->d_V;
    double* zj = c->d_Z + (long)j * N;
    double* w = V + (long)(j + 1) * N;
    // z_j = H^-1 v_j, kept unprojected; its mean m_j is removed on the fly (Jv load
    // shift, and once from the update), which is the zero-mean projection of R12
    double* pj = proj ? part_apply(c, j) : nullptr;
    CHK(apply_raw(c, V + (long)j * N, zj, pj));
    CHK(jv_impl(c, zj, dt, pj, c->d_hpin + SC_M + j, w));
    // CGS2: h = V^T w ; w -= V h and h2 = V^T w in one pass ; w -= V h2 (norm partials fused)
    HIPCHK(launch_multidot(c->stream, V, N, j + 1, w, N, part_md1(c)));
    HIPCHK(launch_maxpy_dot(c->stream, V, N, j + 1, part_md1(c), kRedBlocks, -1.0, w, N, part_md2(c),
                            c->d_hpin + SC_H + sc_half(j)));
    HIPCHK(launch_maxpy(c->stream, V, N, j + 1, part_md2(c), kRedBlocks, -1.0, w, N, c->d_scal + SC_P,
                        c->d_hpin + SC_H2 + sc_half(j)));
    // v_(j+1) = w / ||w|| on the device; ||w|| = h_(j+1,j) goes to the host
    HIPCHK(launch_normalize(c->stream, w, c->d_scal + SC_P, kRedBlocks, N, c->d_hpin + SC_HN + j));
    return PFC_OK;
}

void drop_graphs(pfc_ctx* c) {
    for (hipGraphExec_t& e : c->arn_graph)
        if (e) {
            (void)hipGraphExecDestroy(e);
            e = nullptr;
        }
    c->arn_dt = -1.0;
}

// The Arnoldi step, launched eagerly or (opts.use_graph) as a graph captured on first use for
// this j and dt.  Every kernel argument of the step is fixed for a given j except the 1/dt of
// J v, so the cache is dropped when dt changes.  If capture fails the context goes on eagerly.
pfc_status arnoldi_step(pfc_ctx* c, int j, double dt) {
    if (!c->opts.use_graph || c->opts.timing) return enqueue_arnoldi_step(c, j, dt);
    if (c->arn_dt != dt) {
        drop_graphs(c);
        c->arn_graph.assign(c->opts.gmres_restart, nullptr);
        c->arn_dt = dt;
    }
    if (!c->arn_graph[j]) {
        hipGraph_t g = nullptr;
        HIPCHK(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
        const pfc_status s = enqueue_arnoldi_step(c, j, dt);
        const hipError_t e = hipStreamEndCapture(c->stream, &g);
        if (s != PFC_OK || e != hipSuccess || !g) {
            if (g) (void)hipGraphDestroy(g);
            c->opts.use_graph = 0;
            c->err.clear();
            return enqueue_arnoldi_step(c, j, dt);
        }
        hipGraphExec_t exec = nullptr;
        const hipError_t ei = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ei != hipSuccess) {
            c->opts.use_graph = 0;
            return enqueue_arnoldi_step(c, j, dt);
        }
        c->arn_graph[j] = exec;
    }
    HIPCHK(hipGraphLaunch(c->arn_graph[j], c->stream));
    c->graph_launches++;
    return PFC_OK;
}

// Right-preconditioned flexible GMRES(m) from x = 0 on J x = b (Sec. 4, Eq. (21)).
// Classical Gram-Schmidt with one re-orthogonalisation pass; Givens rotations on the host.
// bnorm_in >= 0 is ||b|| when the caller knows it (saves one synchronisation).  The right-hand
// side is bsign * b (bsign = +-1), so a caller holding F solves J x = -F without forming -F.
// x is only written (the first cycle's update assigns it).  Returns with work still
// enqueued: the caller synchronises before reading x on the host.
pfc_status fgmres(pfc_ctx* c, const double* b, double* x, double dt, double rtol, double atol, int* its,
                  double* res_out, double bnorm_in = -1.0, double bsign = 1.0) {
    const long N = c->g.N;
    const int m = c->opts.gmres_restart;
    const int maxit = c->opts.gmres_maxit;
    const bool proj = c->opts.mass_project;
    const bool lookahead = c->last_gpn >= 1.5;
    double bnorm = bnorm_in;
    if (bnorm < 0.0) CHK(norm2(c, b, &bnorm));
    const double target = std::max(rtol * bnorm, atol);
    *its = 0;
    *res_out = bnorm;
    if (bnorm <= target) {
        HIPCHK(hipMemsetAsync(x, 0, sizeof(double) * N, c->stream));
        return PFC_OK;
    }
    std::vector<double> H((m + 1) * m), cs(m), sn(m), g(m + 1), y(SC_SHIFT - SC_Y + 1, 0.0);
    double* V = c->d_V;
    double* Z = c->d_Z;
    double beta = bnorm;
    bool first = true, x_zero = true;
    int total = 0;
    while (true) {
        // r = bsign b - J x  (x = 0 on the first cycle)
        if (first) {
            HIPCHK(launch_scale(c->stream, b, bsign / beta, V, N));
        } else {
            CHK(jv_impl(c, x, dt, nullptr, nullptr, c->d_r));
            HIPCHK(launch_axpby(c->stream, bsign, b, -1.0, c->d_r, c->d_r, N));
            CHK(norm2(c, c->d_r, &beta));
            if (beta <= target) {
                *res_out = beta;
                break;
            }
            HIPCHK(launch_scale(c->stream, c->d_r, 1.0 / beta, V, N));
        }
        first = false;
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int jdone = 0;
        bool conv = false;
        // Arnoldi steps are enqueued one or two at a time (lookahead: the next step goes in
        // before the host reads this one, one synchronisation for both; used when the last
        // time step needed two or more iterations per linear solve, and wasted only when a
        // solve converges at its first step of a pair)
        for (int j = 0; j < m && !conv && total < maxit;) {
            const bool ahead = lookahead && j + 1 < m && total + 1 < maxit;
            CHK(arnoldi_step(c, j, dt));
            if (ahead) CHK(arnoldi_step(c, j + 1, dt));
            CHK(sync(c));
            const int jend = ahead ? j + 2 : j + 1;
            for (; j < jend; ++j) {
                const double hn = c->h_pin[SC_HN + j];
                if (!std::isfinite(hn)) return fail(c, PFC_ENAN, "non-finite Arnoldi norm");
                for (int i = 0; i <= j; ++i)
                    H[i * m + j] = c->h_pin[SC_H + sc_half(j) + i] + c->h_pin[SC_H2 + sc_half(j) + i];
                H[(j + 1) * m + j] = hn;
                for (int i = 0; i < j; ++i) {
                    const double t = cs[i] * H[i * m + j] + sn[i] * H[(i + 1) * m + j];
                    H[(i + 1) * m + j] = -sn[i] * H[i * m + j] + cs[i] * H[(i + 1) * m + j];
                    H[i * m + j] = t;
                }
                const double den = std::hypot(H[j * m + j], H[(j + 1) * m + j]);
                cs[j] = den > 0 ? H[j * m + j] / den : 1.0;
                sn[j] = den > 0 ? H[(j + 1) * m + j] / den : 0.0;
                H[j * m + j] = den;
                H[(j + 1) * m + j] = 0.0;
                g[j + 1] = -sn[j] * g[j];
                g[j] = cs[j] * g[j];
                ++total;
                jdone = j + 1;
                *res_out = std::fabs(g[j + 1]);
                if (*res_out <= target || hn == 0.0) {
                    conv = true;
                    break;
                }
                if (total >= maxit) break;
            }
        }
        // y = R^{-1} g ; x += Z y
        for (int i = jdone - 1; i >= 0; --i) {
            double s = g[i];
            for (int k = i + 1; k < jdone; ++k) s -= H[i * m + k] * y[k];
            y[i] = s / H[i * m + i];
        }
        // x += sum_j y_j (z_j - m_j); the m_j came back with the last Hessenberg column
        double shift = 0.0;
        if (proj)
            for (int i = 0; i < jdone; ++i) shift += y[i] * c->h_pin[SC_M + i];
        y[SC_SHIFT - SC_Y] = shift;
        // staged through pinned memory: the copy runs asynchronously, and h_y is not written
        // again before a later synchronisation (the next cycle's or the caller's norm)
        std::copy(y.begin(), y.end(), c->h_y);
        HIPCHK(hipMemcpyAsync(c->d_scal + SC_Y, c->h_y, sizeof(double) * (SC_SHIFT - SC_Y + 1), hipMemcpyHostToDevice,
                              c->stream));
        // x (+)= Z y, minus the shift when projecting, in one pass
        HIPCHK(launch_maxpy(c->stream, Z, N, jdone, c->d_scal + SC_Y, 1, 1.0, x, N, nullptr, nullptr, x_zero,
                            proj ? c->d_scal + SC_SHIFT : nullptr, 1, -1.0));
        x_zero = false;
        if (conv || total >= maxit) break;
    }
    *its = total;
    if (*res_out > target) return fail(c, PFC_EKRYLOV, "GMRES did not reach its tolerance");
    return PFC_OK;
}

// Rounding floor of ||F||: eps times a bound of the operator norm of F applied to Phi.
// With kappa = sum_a 4/h_a^2 the spectral radius of -Delta_d, each term of Eq. (12) is
// bounded by (1/dt + (1-gamma)/2 kappa + kappa^2 + kappa^3/2 + 3 kappa) ||Phi||.
double residual_floor(const pfc_ctx* c, double dt, double xnorm) {
    const double k = 4.0 * (c->g.ihx2 + c->g.ihy2 + c->g.ihz2);
    const double op = 1.0 / dt + 0.5 * std::fabs(1.0 - c->model.gamma) * k + k * k + 0.5 * k * k * k + 3.0 * k;
    return 2.220446049250313e-16 * op * xnorm;
}

// First evaluation of a solve, one synchronisation: F = F(X) into d_F with ||F|| and ||X||
// (for the rounding floor) and, with want_ref, the reference ||F(phi^n)|| of the relative
// test (the residual of the paper's initial guess Phi_0 = phi^n; d_r is its scratch).
pfc_status first_residual(pfc_ctx* c, const double* phi, double dt, bool want_ref, double* fn, double* xnorm,
                          double* fref) {
    const int np = residual_partial_count(c);
    double* part = c->d_hpin + SC_P;   // partials straight to the host
    int ts;
    timer_begin(c, 1, &ts);
    if (want_ref) HIPCHK(launch_residual(c, phi, phi, dt, nullptr, c->d_r, part + 2 * np, nullptr));
    HIPCHK(launch_residual(c, c->d_X, phi, dt, nullptr, c->d_F, part, part + np));
    timer_end(c, ts);
    CHK(sync(c));
    *fn = std::sqrt(host_sum(c, 0, np));
    *xnorm = std::sqrt(host_sum(c, np, np));
    *fref = want_ref ? std::sqrt(host_sum(c, 2 * np, np)) : *fn;
    if (!std::isfinite(*fn) || !std::isfinite(*fref)) return fail(c, PFC_ENAN, "non-finite residual norm");
    return PFC_OK;
}

// Newton from the iterate in d_X.  The stop test of Eq. (20) is
// ||F|| <= max(eps_r * fref, eps_a, rounding floor) with fref = ||F(Phi_0)||, or with
// want_ref the reference ||F(phi^n)|| (returned in *fref_out when given).
pfc_status newton_impl(pfc_ctx* c, const double* phi, double dt, pfc_step_stats* st, bool reuse = false,
                       bool want_ref = false, double* fref_out = nullptr) {
    const long N = c->g.N;
    double fn, xnorm, fref;
    CHK(first_residual(c, phi, dt, want_ref, &fn, &xnorm, &fref));
    if (fref_out) *fref_out = fref;
    const double target = std::max({c->opts.newton_rtol * fref, c->opts.newton_atol, residual_floor(c, dt, xnorm)});
    st->res0 = fn;
    st->newton_its = 0;
    st->gmres_its = 0;
    st->ls_cuts = 0;
    bool factored = reuse;                          // lagged factors of an earlier step
    for (int it = 0; it < c->opts.newton_maxit && fn > target; ++it) {
        if (!factored || c->opts.precond_lag < 0) {
            CHK(setup_impl(c, c->d_X, phi, dt));    // factor once per solve (or at every iteration), reuse afterwards
            factored = true;
        } else {
            HIPCHK(launch_coef(c, c->d_X, phi, c->d_c));
        }
        // J S = -F
        int its = 0;
        double lres = 0;
        pfc_status s = fgmres(c, c->d_F, c->d_S, dt, c->opts.lin_rtol, c->opts.lin_atol, &its, &lres, fn, -1.0);
        st->gmres_its += its;
        if (s != PFC_OK && s != PFC_EKRYLOV) return s;
        // backtracking line search on ||F||
        double lam = 1.0, ftn = 0.0;
        bool ok = false;
        while (true) {
            HIPCHK(launch_axpby(c->stream, 1.0, c->d_X, lam, c->d_S, c->d_T, N));
            CHK(residual_impl(c, c->d_T, phi, dt, nullptr, c->d_r, &ftn));
            if (ftn <= (1.0 - 1e-4 * lam) * fn) {
                ok = true;
                break;
            }
            if (lam <= 1.0 / 1024.0) break;
            lam *= 0.5;
            st->ls_cuts++;
        }
        st->newton_its++;
        if (!ok) return fail(c, PFC_ENOTCONV, "line search failed");
        std::swap(c->d_X, c->d_T);
        std::swap(c->d_F, c->d_r);
        fn = ftn;
    }
    st->res_final = fn;
    if (fn > target) return fail(c, PFC_ENOTCONV, "Newton did not reach its tolerance");
    return PFC_OK;
}

// energy and mass of phi; with acc_phi the step is accepted in the same pass
// (acc_prev <- acc_phi, acc_phi <- phi)
pfc_status energy_impl(pfc_ctx* c, const double* phi, double* e, double* m, double* acc_phi = nullptr,
                       double* acc_prev = nullptr) {
    const int np = energy_partial_count(c);
    HIPCHK(launch_energy(c, phi, c->d_hpin + SC_P, acc_phi, acc_prev));
    CHK(sync(c));
    *e = host_sum(c, 0, np) * c->g.cell_volume;
    *m = host_sum(c, np, np) * c->g.cell_volume;
    if (!std::isfinite(*e)) return fail(c, PFC_ENAN, "non-finite energy");
    return PFC_OK;
}

template <typename T>
pfc_status dalloc(pfc_ctx* c, T** p, size_t count) {
    if (hipMalloc((void**)p, sizeof(T) * std::max<size_t>(count, 1)) != hipSuccess) {
        *p = nullptr;
        return fail(c, PFC_ENOMEM, "device allocation failed");
    }
    return PFC_OK;
}

void free_all(pfc_ctx* c) {
    void* ptrs[] = {c->d_level_ptr, c->d_level_pts, c->d_work, c->d_fac, c->d_flag, c->d_c, c->d_u, c->d_mu,
                    c->d_F, c->d_X, c->d_T, c->d_S, c->d_w, c->d_r, c->d_V, c->d_Z, c->d_prev,
                    c->d_tmp3, c->d_part, c->d_scal, c->netw.x, c->netw.a, c->netw.b1c, c->d_zbox};
    for (void* p : ptrs)
        if (p) hipFree(p);
    drop_graphs(c);
    iluk_plan_free(c->iluk);
    c->iluk = nullptr;
    if (c->h_pin) hipHostFree(c->h_pin);
    if (c->h_y) hipHostFree(c->h_y);
    for (auto e : c->timer.pool) hipEventDestroy(e);
}

// Which initial guess this step uses: the learned one when a network is attached, the
// history exists and dt is within the range of step sizes the network was trained on;
// otherwise linear extrapolation when asked for (or as the learned guess's fallback) and the
// history exists; otherwise the previous solution (the paper's choice, Sec. 4).
int guess_kind(const pfc_ctx* c, double dt) {
    const int g = c->opts.guess;
    if (!c->have_prev) return PFC_GUESS_PREVIOUS;
    if (g == PFC_GUESS_LEARNED && c->net && dt >= c->net_dt[1] && dt <= c->net_dt[2]) return PFC_GUESS_LEARNED;
    if (g == PFC_GUESS_EXTRAP || g == PFC_GUESS_LEARNED) return PFC_GUESS_EXTRAP;
    return PFC_GUESS_PREVIOUS;
}

// X = initial guess of kind `used` for the step phi^n -> phi^(n+1) of size dt, from
// phi = phi^n, prev = phi^(n-1) and ratio = dt_n / dt_(n-1); the extrapolated and learned
// guesses are shifted to the mass of phi^n when mass_project is set.
pfc_status guess_into(pfc_ctx* c, const double* phi, const double* prev, double dt, double ratio, int used,
                      double* X) {
    const long N = c->g.N;
    if (used == PFC_GUESS_PREVIOUS) {
        HIPCHK(hipMemcpyAsync(X, phi, sizeof(double) * N, hipMemcpyDeviceToDevice, c->stream));
        return PFC_OK;
    }
    if (used == PFC_GUESS_EXTRAP) {
        HIPCHK(launch_extrap(c->stream, phi, prev, ratio, X, N));
    } else {
        double* part = part_md1(c);
        HIPCHK(launch_dot(c->stream, phi, nullptr, N, part));
        double* diff = c->opts.mass_project ? part_md2(c) : nullptr;   // partials of phi - X
        // l = ln(dt/dt_ref), step scale g = exp(beta l + gamma l^2), condition c = l/s_c
        const double* sc = c->net_scale;
        const double l = std::log(dt / c->net_dt[0]), g = std::exp(sc[4] * l + sc[5] * l * l);
        pfc_status s = net_guess(c->net, c->stream, phi, prev, c->g.ny, c->g.nx, ratio, l / sc[3], 1.0 / sc[0],
                                 1.0 / (sc[1] * g), sc[2] * g, part, kRedBlocks, c->netw, X, diff);
        if (s != PFC_OK) return fail(c, s, std::string("learned guess: ") + net_error(c->net));
        if (diff) HIPCHK(launch_shift(c->stream, X, diff, kRedBlocks, 1.0 / (double)N, N));
        return PFC_OK;
    }
    if (c->opts.mass_project) {   // restore the mass of phi^n exactly: X += mean(phi - X)
        HIPCHK(launch_axpby(c->stream, 1.0, phi, -1.0, X, c->d_w, N));
        CHK(shift_by_sum(c, X, c->d_w, 1.0 / (double)N));
    }
    return PFC_OK;
}

// d_X = the guess of kind `used` for the step of size dt from the stored history.
pfc_status make_guess(pfc_ctx* c, const double* phi, double dt, int used) {
    return guess_into(c, phi, c->d_prev, dt, used == PFC_GUESS_PREVIOUS ? 1.0 : dt / c->dt_nm1, used, c->d_X);
}

}  // namespace

extern "C" {


void pfc_default_opts(pfc_opts* o) {
    std::memset(o, 0, sizeof(*o));
    o->newton_rtol = 1e-8;
    o->newton_atol = 1e-10;
    o->lin_rtol = 1e-3;
    o->lin_atol = 1e-11;
    o->newton_maxit = 50;
    o->gmres_restart = 30;
    o->gmres_maxit = 300;
    o->sub[0] = o->sub[1] = o->sub[2] = 2;
    o->overlap = 2;
    o->ras_kind = PFC_RAS_LEFT;
    o->sub_solver = PFC_SUB_ILU0;
    o->precond_fp32 = 0;
    o->mass_project = 1;
    o->guess = PFC_GUESS_PREVIOUS;
    o->dt_min = o->dt_max = 0.1;
    o->eta = 0.0;
    o->max_retries = 4;
    o->timing = 0;
    o->precond_lag = 0;
    o->newton_rel_ref = 1;
    o->use_graph = 0;
    o->ilu_level = 2;
}

pfc_status pfc_create(const pfc_grid* gr, const pfc_model* md, const pfc_opts* op, void* stream,
                      pfc_ctx** out) {
    if (!gr || !md || !op || !out) return PFC_EINVAL;
    *out = nullptr;
    pfc_ctx* c = new pfc_ctx();
    c->grid = *gr;
    c->model = *md;
    c->opts = *op;
    c->stream = (hipStream_t)stream;
    auto bad = [&](const std::string& m) {
        c->err = m;
        return PFC_EINVAL;
    };
    pfc_status s = PFC_OK;
    const int dim = gr->dim;
    if (dim != 2 && dim != 3) s = bad("dim must be 2 or 3");
    if (s == PFC_OK && md->mobility != PFC_MOBILITY_1 && md->mobility != PFC_MOBILITY_1_MINUS_SQ)
        s = bad("unknown mobility");
    if (s == PFC_OK && md->boundary != PFC_BC_PERIODIC && md->boundary != PFC_BC_NEUMANN) s = bad("unknown boundary");
    for (int a = 0; s == PFC_OK && a < dim; ++a) {
        if (gr->n[a] < 8) s = bad("grid extent below 8");
        else if (!(gr->L[a] > 0)) s = bad("domain length must be positive");
        else if (op->sub[a] < 2 || gr->n[a] % op->sub[a] != 0) s = bad("sub[a] must be >= 2 and divide n[a]");
        else {
            const int e = gr->n[a] / op->sub[a] + 2 * op->overlap;
            if (e > gr->n[a] - 3 || e > 255) s = bad("extended subdomain too wide");
        }
    }
    if (s == PFC_OK && op->overlap < 0) s = bad("negative overlap");
    if (s == PFC_OK && (op->gmres_restart < 1 || op->gmres_restart > 60)) s = bad("gmres_restart must be 1..60");
    if (s == PFC_OK && (op->gmres_maxit < 1 || op->newton_maxit < 1)) s = bad("iteration limits must be >= 1");
    if (s == PFC_OK && op->precond_lag < -1) s = bad("precond_lag must be >= -1");
    if (s == PFC_OK && op->use_graph && !stream) s = bad("use_graph needs a non-default stream (graph capture)");
    if (s == PFC_OK && (op->ras_kind < PFC_RAS_LEFT || op->ras_kind > PFC_RAS_RIGHT)) s = bad("unknown ras_kind");
    if (s == PFC_OK && op->ras_kind != PFC_RAS_LEFT)   // boxes covering a cell, per axis, for the sum
        for (int a = 0; a < dim; ++a) {
            const int own = gr->n[a] / op->sub[a], R = (op->overlap + own - 1) / own;
            if (std::min(2 * R + 1, op->sub[a]) > 16) s = bad("overlap too wide for the AS / right-RAS sum");
        }
    if (s == PFC_OK && op->sub_solver != PFC_SUB_ILU0 && op->sub_solver != PFC_SUB_LU && op->sub_solver != PFC_SUB_ILUK)
        s = bad("bad sub_solver");
    if (s == PFC_OK && op->sub_solver == PFC_SUB_ILUK && (op->ilu_level < 0 || op->ilu_level > 4))
        s = bad("ilu_level must be 0..4");
    if (s == PFC_OK && op->sub_solver == PFC_SUB_LU && dim != 2) {
        c->err = "exact subdomain LU is built for 2-D only";
        s = PFC_EUNSUP;
    }
    if (s == PFC_OK && !(op->dt_min > 0 && op->dt_max >= op->dt_min)) s = bad("need 0 < dt_min <= dt_max");
    if (s == PFC_OK && (op->guess < PFC_GUESS_PREVIOUS || op->guess > PFC_GUESS_LEARNED)) s = bad("bad guess kind");
    if (s == PFC_OK && op->guess == PFC_GUESS_LEARNED && dim != 2) {
        c->err = "the learned guess is built for 2-D grids";
        s = PFC_EUNSUP;
    }
    if (s != PFC_OK) {
        pfc_status r = s;
        std::string msg = c->err;
        delete c;
        std::fprintf(stderr, "pfc_create: %s\n", msg.c_str());
        return r;
    }
    // geometry
    Geom& g = c->g;
    g.dim = dim;
    g.nx = gr->n[0];
    g.ny = gr->n[1];
    g.nz = dim == 3 ? gr->n[2] : 1;
    g.N = (long)g.nx * g.ny * g.nz;
    const double hx = gr->L[0] / g.nx, hy = gr->L[1] / g.ny, hz = dim == 3 ? gr->L[2] / g.nz : 1.0;
    g.ihx2 = 1.0 / (hx * hx);
    g.ihy2 = 1.0 / (hy * hy);
    g.ihz2 = dim == 3 ? 1.0 / (hz * hz) : 0.0;
    g.cell_volume = hx * hy * (dim == 3 ? hz : 1.0);
    Decomp& d = c->dec;
    d.ov = op->overlap;
    d.nsub = 1;
    d.next = 1;
    for (int a = 0; a < 3; ++a) {
        const bool act = a < dim;
        d.sub[a] = act ? op->sub[a] : 1;
        d.own[a] = act ? gr->n[a] / op->sub[a] : 1;
        d.ext[a] = act ? d.own[a] + 2 * d.ov : 1;
        d.nsub *= d.sub[a];
        d.next *= d.ext[a];
    }
    if (op->sub_solver == PFC_SUB_LU && d.ext[0] > 72) s = bad("exact LU needs a box x-extent of at most 72");
    if (s == PFC_OK && op->sub_solver == PFC_SUB_LU && lu_factor_lds_bytes(d.ext[0]) > 159 * 1024)
        s = bad("exact LU block too large for LDS");
    const size_t ilu_lds = (op->precond_fp32 ? 4 : 8) * ((size_t)d.next + 1);
    if (s == PFC_OK && op->sub_solver == PFC_SUB_ILU0 && ilu_lds > 160 * 1024) s = bad("subdomain too large for LDS");
    if (s != PFC_OK) {
        std::string msg = c->err;
        delete c;
        std::fprintf(stderr, "pfc_create: %s\n", msg.c_str());
        return s;
    }
    build_stencil_table(g, md->gamma, 1.0, &c->st);
    const long N = g.N;
    const int m = op->gmres_restart;
    const size_t esz = op->precond_fp32 ? sizeof(float) : sizeof(double);
    s = PFC_OK;
    auto A = [&](pfc_status r) {
        if (s == PFC_OK) s = r;
    };
    A(dalloc(c, &c->d_c, N));
    A(dalloc(c, &c->d_F, N));
    A(dalloc(c, &c->d_X, N));
    A(dalloc(c, &c->d_T, N));
    A(dalloc(c, &c->d_S, N));
    A(dalloc(c, &c->d_w, N));
    A(dalloc(c, &c->d_r, N));
    A(dalloc(c, &c->d_prev, N));
    A(dalloc(c, &c->d_V, (size_t)(m + 1) * N));
    A(dalloc(c, &c->d_Z, (size_t)m * N));
    if (dim == 3 || md->mobility != PFC_MOBILITY_1 || md->boundary != PFC_BC_PERIODIC)
        A(dalloc(c, &c->d_tmp3, 2 * (size_t)N));
    if (md->mobility == PFC_MOBILITY_1_MINUS_SQ) {
        A(dalloc(c, &c->d_u, N));
        A(dalloc(c, &c->d_mu, N));
    }
    A(dalloc(c, &c->d_part, 128 * (size_t)kRedBlocks + 64 * (size_t)c->dec.nsub));
    c->n_scal = SC_P + std::max({kRedBlocks, 3 * residual_partial_count(c), 2 * energy_partial_count(c)});
    A(dalloc(c, &c->d_scal, (size_t)c->n_scal));
    A(dalloc(c, &c->d_flag, 1));
    if (op->ras_kind != PFC_RAS_LEFT) A(dalloc(c, &c->d_zbox, (size_t)c->dec.nsub * c->dec.next));
    if (op->sub_solver == PFC_SUB_ILU0) {
        std::vector<int> lptr, lpts;
        build_ilu_schedule(c, &lptr, &lpts);
        c->nlev = (int)lptr.size() - 1;
        int widest = 0;
        for (int l = 0; l < c->nlev; ++l) widest = std::max(widest, lptr[l + 1] - lptr[l]);
        c->ilu_cells_per_lane = (widest + 63) / 64;
        if (c->ilu_cells_per_lane > kIluMaxCellsPerLane && s == PFC_OK)
            s = fail(c, PFC_EINVAL, "ILU(0) box has a wavefront level wider than 192 cells");
        A(dalloc(c, &c->d_level_ptr, lptr.size()));
        A(dalloc(c, &c->d_level_pts, lpts.size()));
        c->fac_elems = (size_t)d.nsub * d.next * ilu_fac_elems_per_cell(c->st.S);
        A(dalloc(c, &c->d_work, (size_t)d.nsub * d.next * c->st.S));
        if (s == PFC_OK) {
            hipMemcpy(c->d_level_ptr, lptr.data(), sizeof(int) * lptr.size(), hipMemcpyHostToDevice);
            hipMemcpy(c->d_level_pts, lpts.data(), sizeof(int) * lpts.size(), hipMemcpyHostToDevice);
        }
    } else if (op->sub_solver == PFC_SUB_ILUK) {
        std::string e;
        const pfc_status r = iluk_plan_create(c, op->ilu_level, &e);
        if (r != PFC_OK && s == PFC_OK) s = fail(c, r, e);
    } else {
        c->lu_W = d.ext[0];
        c->lu_H = d.ext[1];
        const size_t WW = (size_t)c->lu_W * c->lu_W;
        c->fac_elems = (size_t)d.nsub * c->lu_H * lu_factor_elems_per_block_row(c->lu_W);
        A(dalloc(c, &c->d_work, (size_t)d.nsub * lu_work_blocks(c->lu_W) * WW));
    }
    if (s == PFC_OK) {
        if (hipMalloc(&c->d_fac, esz * c->fac_elems) != hipSuccess) s = fail(c, PFC_ENOMEM, "factor allocation failed");
    }
    if (s == PFC_OK && (hipHostMalloc((void**)&c->h_pin, sizeof(double) * c->n_scal,
                                      hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
                        hipHostGetDevicePointer((void**)&c->d_hpin, c->h_pin, 0) != hipSuccess ||
                        hipHostMalloc((void**)&c->h_y, sizeof(double) * (SC_SHIFT - SC_Y + 1)) != hipSuccess))
        s = fail(c, PFC_ENOMEM, "pinned allocation failed");
    if (s == PFC_OK && (set_ilu_lds_limits() != hipSuccess || set_lu_lds_limits() != hipSuccess ||
                        set_iluk_lds_limits() != hipSuccess))
        s = fail(c, PFC_EHIP, "cannot raise the LDS limit");
    if (s == PFC_OK && hipMemset(c->d_scal, 0, sizeof(double) * c->n_scal) != hipSuccess)
        s = fail(c, PFC_EHIP, "memset");
    if (s != PFC_OK) {
        std::fprintf(stderr, "pfc_create: %s\n", c->err.c_str());
        free_all(c);
        delete c;
        return s;
    }
    *out = c;
    return PFC_OK;
}

void pfc_destroy(pfc_ctx* c) {
    if (!c) return;
    hipStreamSynchronize(c->stream);
    free_all(c);
    delete c;
}

const char* pfc_last_error(const pfc_ctx* c) { return c ? c->err.c_str() : "null context"; }

pfc_status pfc_residual(pfc_ctx* c, const double* Phi, const double* phi, double dt, const double* src, double* F,
                        double* norm) {
    if (!c || !Phi || !phi || !F || !(dt > 0)) return c ? fail(c, PFC_EINVAL, "bad argument") : PFC_EINVAL;
    return residual_impl(c, Phi, phi, dt, src, F, norm);
}

pfc_status pfc_jv(pfc_ctx* c, const double* Phi, const double* phi, double dt, const double* v, double* Jv) {
    if (!c || !Phi || !phi || !v || !Jv || !(dt > 0)) return c ? fail(c, PFC_EINVAL, "bad argument") : PFC_EINVAL;
    HIPCHK(launch_coef(c, Phi, phi, c->d_c));
    return jv_impl(c, v, dt, nullptr, nullptr, Jv);
}

pfc_status pfc_ras_setup(pfc_ctx* c, const double* Phi, const double* phi, double dt) {
    if (!c || !Phi || !phi || !(dt > 0)) return c ? fail(c, PFC_EINVAL, "bad argument") : PFC_EINVAL;
    return setup_impl(c, Phi, phi, dt);
}

pfc_status pfc_ras_apply(pfc_ctx* c, const double* r, double* z) {
    if (!c || !r || !z) return c ? fail(c, PFC_EINVAL, "bad argument") : PFC_EINVAL;
    return apply_impl(c, r, z);
}

pfc_status pfc_energy(pfc_ctx* c, const double* phi, double* e, double* m) {
    if (!c || !phi || !e || !m) return c ? fail(c, PFC_EINVAL, "bad argument") : PFC_EINVAL;
    return energy_impl(c, phi, e, m);
}

pfc_status pfc_gmres(pfc_ctx* c, const double* Phi, const double* phi, double dt, const double* b, double* x,
                     double rtol, double atol, int* its, double* res) {
    if (!c || !Phi || !phi || !b || !x || !its || !res || !(dt > 0))
        return c ? fail(c, PFC_EINVAL, "bad argument") : PFC_EINVAL;
    HIPCHK(launch_coef(c, Phi, phi, c->d_c));
    HIPCHK(hipMemcpyAsync(c->d_w, b, sizeof(double) * c->g.N, hipMemcpyDeviceToDevice, c->stream));
    const pfc_status s = fgmres(c, c->d_w, x, dt, rtol, atol, its, res);
    HIPCHK(hipStreamSynchronize(c->stream));
    return s;
}

pfc_status pfc_newton(pfc_ctx* c, const double* phi, double dt, double* Phi, pfc_step_stats* st) {
    if (!c || !phi || !Phi || !st || !(dt > 0)) return c ? fail(c, PFC_EINVAL, "bad argument") : PFC_EINVAL;
    std::memset(st, 0, sizeof(*st));
    double fref = 0.0;
    HIPCHK(hipMemcpyAsync(c->d_X, Phi, sizeof(double) * c->g.N, hipMemcpyDeviceToDevice, c->stream));
    pfc_status s = newton_impl(c, phi, dt, st, false, c->opts.newton_rel_ref != 0, &fref);
    st->res_ref = fref;
    HIPCHK(hipMemcpyAsync(Phi, c->d_X, sizeof(double) * c->g.N, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    st->dt = dt;
    return s;
}

pfc_status pfc_step(pfc_ctx* c, double* phi, pfc_step_stats* st) {
    if (!c || !phi || !st) return c ? fail(c, PFC_EINVAL, "bad argument") : PFC_EINVAL;
    std::memset(st, 0, sizeof(*st));
    const long N = c->g.N;
    const pfc_opts& o = c->opts;
    if (!c->have_energy) {
        double m0;
        CHK(energy_impl(c, phi, &c->F_n, &m0));
        c->have_energy = true;
    }
    double dt = o.dt_min;
    if (c->step > 0 && o.dt_max > o.dt_min) {
        const double fp = std::fabs(c->F_n - c->F_nm1) / c->dt_nm1;
        dt = std::max(o.dt_min, o.dt_max / std::sqrt(1.0 + o.eta * fp * fp));
    }
    pfc_status s = PFC_OK;
    for (int attempt = 0;; ++attempt) {
        // initial guess
        const int used = guess_kind(c, dt);
        CHK(make_guess(c, phi, dt, used));
        pfc_step_stats tmp;
        std::memset(&tmp, 0, sizeof(tmp));
        double fref = 0.0;
        const bool want_ref = o.newton_rel_ref && used != PFC_GUESS_PREVIOUS;
        const bool reuse = may_reuse_factors(c, dt);
        const long fac_before = c->fac_step;
        s = newton_impl(c, phi, dt, &tmp, reuse, want_ref, &fref);
        if (s != PFC_OK && reuse && (s == PFC_ENOTCONV || s == PFC_EKRYLOV)) {
            // lagged factors did not do: same dt, fresh factors
            st->newton_its += tmp.newton_its;
            st->gmres_its += tmp.gmres_its;
            CHK(make_guess(c, phi, dt, used));
            std::memset(&tmp, 0, sizeof(tmp));
            c->fac_valid = false;
            s = newton_impl(c, phi, dt, &tmp, false, want_ref, &fref);
        }
        if (s == PFC_OK && tmp.newton_its > 0) {
            const double gpn = (double)tmp.gmres_its / tmp.newton_its;
            if (c->fac_step != fac_before || c->fac_step == c->step) c->fac_gpn = gpn;
            c->last_gpn = gpn;
        }
        st->newton_its += tmp.newton_its;
        st->gmres_its += tmp.gmres_its;
        st->ls_cuts += tmp.ls_cuts;
        st->res0 = tmp.res0;
        st->res_final = tmp.res_final;
        st->res_ref = fref;
        st->guess_used = used;
        if (s == PFC_OK) break;
        if ((s != PFC_ENOTCONV && s != PFC_EKRYLOV) || attempt >= o.max_retries || dt <= o.dt_min / 16) return s;
        st->rejected++;
        dt = std::max(dt * 0.5, o.dt_min / 16);
    }
    // accept (phi^(n-1) <- phi^n, phi^n <- X) in the pass that forms the energy of X
    double e, m;
    CHK(energy_impl(c, c->d_X, &e, &m, phi, c->d_prev));
    c->have_prev = true;
    c->F_nm1 = c->F_n;
    c->F_n = e;
    c->dt_nm1 = dt;
    c->t += dt;
    c->step++;
    st->dt = dt;
    st->t = c->t;
    st->energy = e;
    st->mass = m;
    return PFC_OK;
}

pfc_status pfc_reset(pfc_ctx* c) {
    if (!c) return PFC_EINVAL;
    c->step = 0;
    c->F_n = c->F_nm1 = c->dt_nm1 = c->t = 0.0;
    c->have_prev = c->have_energy = false;
    c->fac_valid = false;
    c->fac_step = -1;
    c->fac_gpn = c->last_gpn = 0.0;
    CHK(timer_drain(c));
    for (int i = 0; i < 4; ++i) {
        c->timer.count[i] = 0;
        c->timer.total_ms[i] = 0.0;
    }
    c->graph_launches = 0;
    return PFC_OK;
}

namespace {
// checkpoint file: header, then phi (N doubles) and, if have_prev, phi^(n-1) (N doubles)
struct CkptHeader {
    char magic[8];                 // "PFCCKPT2"
    int32_t dim, n[3];
    double L[3], gamma;
    int32_t mobility, boundary;
    int64_t step;
    double t, F_n, F_nm1, dt_nm1;
    int32_t have_prev, have_energy;
};
const char kMagic[8] = {'P', 'F', 'C', 'C', 'K', 'P', 'T', '2'};
}  // namespace

pfc_status pfc_checkpoint_save(pfc_ctx* c, const double* phi, const char* path) {
    if (!c || !phi || !path) return c ? fail(c, PFC_EINVAL, "bad argument") : PFC_EINVAL;
    const size_t N = (size_t)c->g.N;
    std::vector<double> buf(N * (c->have_prev ? 2 : 1));
    HIPCHK(hipMemcpyAsync(buf.data(), phi, sizeof(double) * N, hipMemcpyDeviceToHost, c->stream));
    if (c->have_prev)
        HIPCHK(hipMemcpyAsync(buf.data() + N, c->d_prev, sizeof(double) * N, hipMemcpyDeviceToHost, c->stream));
    CHK(sync(c));
    CkptHeader h;
    std::memset(&h, 0, sizeof(h));
    std::memcpy(h.magic, kMagic, 8);
    h.dim = c->grid.dim;
    for (int a = 0; a < 3; ++a) {
        h.n[a] = c->grid.n[a];
        h.L[a] = c->grid.L[a];
    }
    h.gamma = c->model.gamma;
    h.mobility = c->model.mobility;
    h.boundary = c->model.boundary;
    h.step = c->step;
    h.t = c->t;
    h.F_n = c->F_n;
    h.F_nm1 = c->F_nm1;
    h.dt_nm1 = c->dt_nm1;
    h.have_prev = c->have_prev;
    h.have_energy = c->have_energy;
    FILE* f = std::fopen(path, "wb");
    if (!f) return fail(c, PFC_EINVAL, std::string("cannot open ") + path);
    const bool ok = std::fwrite(&h, sizeof(h), 1, f) == 1 && std::fwrite(buf.data(), sizeof(double), buf.size(), f) == buf.size();
    if (std::fclose(f) != 0 || !ok) return fail(c, PFC_EINVAL, std::string("cannot write ") + path);
    return PFC_OK;
}

pfc_status pfc_checkpoint_load(pfc_ctx* c, double* phi, const char* path) {
    if (!c || !phi || !path) return c ? fail(c, PFC_EINVAL, "bad argument") : PFC_EINVAL;
    FILE* f = std::fopen(path, "rb");
    if (!f) return fail(c, PFC_EINVAL, std::string("cannot open ") + path);
    CkptHeader h;
    bool ok = std::fread(&h, sizeof(h), 1, f) == 1 && std::memcmp(h.magic, kMagic, 8) == 0 && h.dim == c->grid.dim &&
              h.gamma == c->model.gamma && h.mobility == c->model.mobility && h.boundary == c->model.boundary &&
              (h.have_prev == 0 || h.have_prev == 1);
    for (int a = 0; ok && a < 3; ++a) ok = h.n[a] == c->grid.n[a] && h.L[a] == c->grid.L[a];
    const size_t N = (size_t)c->g.N;
    std::vector<double> buf;
    if (ok) {
        buf.resize(N * (h.have_prev ? 2 : 1));
        ok = std::fread(buf.data(), sizeof(double), buf.size(), f) == buf.size();
    }
    std::fclose(f);
    if (!ok) return fail(c, PFC_EINVAL, std::string("not a checkpoint of this grid and model: ") + path);
    HIPCHK(hipMemcpyAsync(phi, buf.data(), sizeof(double) * N, hipMemcpyHostToDevice, c->stream));
    if (h.have_prev)
        HIPCHK(hipMemcpyAsync(c->d_prev, buf.data() + N, sizeof(double) * N, hipMemcpyHostToDevice, c->stream));
    CHK(sync(c));
    c->step = h.step;
    c->t = h.t;
    c->F_n = h.F_n;
    c->F_nm1 = h.F_nm1;
    c->dt_nm1 = h.dt_nm1;
    c->have_prev = h.have_prev != 0;
    c->have_energy = h.have_energy != 0;
    c->fac_valid = false;
    c->fac_step = -1;
    c->fac_gpn = c->last_gpn = 0.0;
    return PFC_OK;
}

pfc_status pfc_kernel_time(pfc_ctx* c, int which, long* count, double* total_ms) {
    if (!c || which < 0 || which > 4 || !count || !total_ms) return PFC_EINVAL;
    if (which == 4) {
        *count = c->graph_launches;
        *total_ms = 0.0;
        return PFC_OK;
    }
    CHK(timer_drain(c));
    *count = c->timer.count[which];
    *total_ms = c->timer.total_ms[which];
    return PFC_OK;
}

pfc_status pfc_guess(pfc_ctx* c, int kind, const double* phi, const double* phi_prev, double dt, double dt_prev,
                     double* X) {
    if (!c) return PFC_EINVAL;
    if (!phi || !X || X == phi || X == phi_prev) return fail(c, PFC_EINVAL, "bad argument");
    if (kind < PFC_GUESS_PREVIOUS || kind > PFC_GUESS_LEARNED) return fail(c, PFC_EINVAL, "bad guess kind");
    if (kind != PFC_GUESS_PREVIOUS && (!phi_prev || !(dt > 0) || !(dt_prev > 0)))
        return fail(c, PFC_EINVAL, "the extrapolated and learned guesses need phi_prev and positive dt, dt_prev");
    if (kind == PFC_GUESS_LEARNED && !c->net) return fail(c, PFC_EINVAL, "no network attached");
    return guess_into(c, phi, phi_prev, dt, kind == PFC_GUESS_PREVIOUS ? 1.0 : dt / dt_prev, kind, X);
}

pfc_status pfc_attach_net(pfc_ctx* c, pfc_net* net, const double* scales, const double* dt_range) {
    if (!c) return PFC_EINVAL;
    if (!net) {
        c->net = nullptr;
        return PFC_OK;
    }
    if (c->g.dim != 2) return fail(c, PFC_EUNSUP, "the learned guess is built for 2-D grids");
    bool sc_ok = scales != nullptr;
    for (int i = 0; sc_ok && i < 6; ++i) sc_ok = std::isfinite(scales[i]) && (i >= 4 || scales[i] > 0);
    if (!sc_ok) return fail(c, PFC_EINVAL, "scales must be finite, s_a, s_b, s_o, s_c positive");
    if (!dt_range || !(dt_range[0] > 0) || !(dt_range[1] > 0) || !(dt_range[2] >= dt_range[1]) ||
        !std::isfinite(dt_range[0]) || !std::isfinite(dt_range[2]))
        return fail(c, PFC_EINVAL, "dt_range must be dt_ref > 0 and 0 < dt_lo <= dt_hi, finite");
    if (!c->netw.x) {
        const size_t N = (size_t)c->g.N;
        if (hipMalloc((void**)&c->netw.x, sizeof(float) * 2 * N) != hipSuccess ||
            hipMalloc((void**)&c->netw.a, sizeof(float) * kNetWorkFloats * N) != hipSuccess ||
            hipMalloc((void**)&c->netw.b1c, sizeof(float) * 32) != hipSuccess)
            return fail(c, PFC_ENOMEM, "out of device memory for the network buffers");
    }
    if (net_prepare(net) != PFC_OK) return fail(c, PFC_EHIP, std::string("network: ") + net_error(net));
    c->net = net;
    for (int i = 0; i < 6; ++i) c->net_scale[i] = scales[i];
    for (int i = 0; i < 3; ++i) c->net_dt[i] = dt_range[i];
    return PFC_OK;
}

}  // extern "C"
