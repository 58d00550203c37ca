/*
 * pfc.h -- C ABI of libpfc, a gfx950 (MI355X) implementation of the per-time-step
 * nonlinear solve of the energy-stable phase-field-crystal (PFC) scheme of
 * Li, Yang, Cai et al., "Parallel energy-stable phase field crystal simulations based
 * on domain decomposition methods" (arXiv:1703.01202).
 *
 * What is computed
 *   Each time step solves F(Phi) = 0 (Sec. 4, Eq. (17)) where F is the semi-implicit
 *   discrete-variational-derivative scheme of Sec. 3, Eq. (12) with M = 1 on a
 *   cell-centred periodic mesh:
 *       F(Phi) = (Phi - phi)/dt - Delta_d mu_d(Phi, phi),
 *       mu_d   = [(1-gamma) + 2 Delta_d + Delta_d^2] (Phi+phi)/2
 *                + (Phi^3 + Phi^2 phi + Phi phi^2 + phi^3)/4          (Eq. (11)),
 *   by inexact Newton with backtracking (Eqs. (18)-(20)), right-preconditioned flexible
 *   GMRES (Eq. (21)) and a restricted additive Schwarz preconditioner (Eqs. (22)-(26))
 *   whose subdomain problems carry phi = 0 on the three-layer ring around each
 *   extended subdomain, solved by ILU(0) or by exact LU.  The time step adapts by
 *   Eq. (16) from the discrete free energy of Eq. (8).
 *
 * Conventions (all entry points)
 *   - Every field is a DEVICE pointer to a contiguous FP64 array owned by the caller,
 *     laid out [nz][ny][nx] with x fastest (2-D: nz = 1).  No call keeps or frees a
 *     caller pointer.  Output arrays may not alias inputs of the same call.
 *   - Work is enqueued on the HIP stream given to pfc_create.  Calls that return host
 *     scalars (norms, energies, statistics) synchronise that stream; the others only
 *     enqueue.
 *   - Errors are returned as pfc_status, never thrown; pfc_last_error gives a message.
 *     A context is used from one host thread at a time.
 *   - Sizes: n[a] >= 8 per active axis; sub[a] >= 2 divides n[a]; the extended
 *     subdomain n[a]/sub[a] + 2*overlap is at most n[a] - 3 (so a box never meets
 *     itself through the periodic wrap within the stencil radius) and at most 255.
 *     Anything else is PFC_EINVAL at pfc_create.
 */
#ifndef PFC_H
#define PFC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PFC_OK = 0,
    PFC_EINVAL = -1,     /* bad argument, size or option */
    PFC_ENOMEM = -2,     /* device allocation failed */
    PFC_EHIP = -3,       /* a HIP runtime call failed */
    PFC_ENAN = -4,       /* a non-finite value appeared in a norm */
    PFC_ENOTCONV = -5,   /* Newton did not reach its tolerance (Sec. 4, Eq. (20)) */
    PFC_EKRYLOV = -6,    /* GMRES did not reach its tolerance (Table 1 "n/c") */
    PFC_EPIVOT = -7,     /* zero or non-finite pivot in a subdomain factorisation */
    PFC_EUNSUP = -8      /* option combination not built (e.g. exact LU in 3-D) */
} pfc_status;

/* Cell-centred periodic mesh (Sec. 3): n[0] = Nx (fastest), n[1] = Ny, n[2] = Nz;
 * L[a] domain length, mesh size L[a]/n[a].  dim is 2 or 3. */
typedef struct {
    int dim;
    int n[3];
    double L[3];
} pfc_grid;

/* Model (Sec. 2, Eq. (1)): gamma is the quench depth.
 * mobility: PFC_MOBILITY_1 (M = 1) or PFC_MOBILITY_1_MINUS_SQ (M(phi) = 1 - phi^2, taken at the
 *   averaged state (Phi + phi)/2 as Eq. (12) says, on a face as the mean of its two cells, Sec. 3).
 * boundary: PFC_BC_PERIODIC or PFC_BC_NEUMANN, the Neumann-type conditions of Sec. 2 read as zero
 *   normal differences: the ghost cell beyond a boundary face mirrors the cell inside it, for
 *   every field a difference operator acts on (so no flux crosses the boundary and mass is kept).
 * With a variable mobility or Neumann boundaries the residual, Jacobian action and energy are
 * exact; the Schwarz subdomain matrices stay those of M = 1 with periodic box gathers (a
 * preconditioner only: flexible GMRES converges to the same root). */
enum { PFC_MOBILITY_1 = 0, PFC_MOBILITY_1_MINUS_SQ = 1 };
enum { PFC_BC_PERIODIC = 0, PFC_BC_NEUMANN = 1 };
typedef struct {
    double gamma;
    int mobility;
    int boundary;
} pfc_model;

/* Schwarz preconditioners (Sec. 4): left-RAS (Eq. (23)): restrict with overlap, extend the owned
 * cells only; classical AS (Eq. (22)): restrict and extend with overlap, the boxes' solutions
 * added where they overlap; right-RAS (Eq. (24)): restrict the owned cells only, extend with
 * overlap and add.  The sums over overlapping boxes are formed per cell in a fixed order. */
enum { PFC_RAS_LEFT = 0, PFC_AS_CLASSICAL = 1, PFC_RAS_RIGHT = 2 };
/* Subdomain solvers (Sec. 4; Table 1): ILU(0) on the stencil pattern, exact LU (2-D), and
 * ILU(k) with k = pfc_opts.ilu_level levels of fill (k = 0 gives the ILU(0) factors through the
 * general-pattern kernels). */
enum { PFC_SUB_ILU0 = 0, PFC_SUB_LU = 1, PFC_SUB_ILUK = 2 };
enum { PFC_GUESS_PREVIOUS = 0, PFC_GUESS_EXTRAP = 1, PFC_GUESS_LEARNED = 2 };

typedef struct {
    double newton_rtol, newton_atol;  /* eps_r, eps_a of Eq. (20); defaults 1e-8, 1e-10 */
    double lin_rtol, lin_atol;        /* xi_r, xi_a of the linear test; defaults 1e-3, 1e-11 */
    int newton_maxit;                 /* default 50 */
    int gmres_restart;                /* default 30 */
    int gmres_maxit;                  /* per Newton step, default 300 */
    int sub[3];                       /* subdomains per axis (x, y, z) */
    int overlap;                      /* overlap in mesh layers (paper's delta = 3 layers) */
    int ras_kind;                     /* PFC_RAS_LEFT (default), PFC_AS_CLASSICAL or PFC_RAS_RIGHT */
    int sub_solver;                   /* PFC_SUB_ILU0, PFC_SUB_LU (2-D only) or PFC_SUB_ILUK */
    int precond_fp32;                 /* 1: factors stored and applied in FP32 */
    int mass_project;                 /* 1: zero-mean projection of guess and directions */
    int guess;                        /* PFC_GUESS_* */
    double dt_min, dt_max, eta;       /* Eq. (16); dt_min == dt_max gives a fixed step */
    int max_retries;                  /* dt halvings after a failed Newton solve, default 4 */
    int timing;                       /* bitmask of the launches timed with events (pfc_kernel_time):
                                         1 preconditioner apply, 2 residual, 4 Jacobian action,
                                         8 factorisation; 0 off */
    int precond_lag;                  /* -1: factor at every Newton step (Table 1's columns without
                                         reuse); 0: factor at the first Newton step of every time step (the
                                         paper's reuse); L > 0: pfc_step keeps the factors for up to L
                                         time steps while dt stays within 20% of the dt they were built
                                         with and GMRES iterations per Newton step stay at most twice
                                         (+1) those of the step that factored; a failed solve on lagged
                                         factors is retried with fresh ones */
    int newton_rel_ref;               /* reference of eps_r in Eq. (20): 1 (default) ||F(phi^n)||, the
                                         residual of the paper's initial guess Phi_0 = phi^n, whatever
                                         guess starts the iteration, so every guess meets the same
                                         target; 0: ||F|| at the guess actually used */
    int use_graph;                    /* 1: each Arnoldi step (preconditioner apply, J v, both Gram-Schmidt
                                         passes, which write the Hessenberg column to mapped host
                                         memory) is captured once per
                                         Krylov index and time step size as a HIP graph and replayed with
                                         one launch; needs a non-default stream (PFC_EINVAL otherwise) and
                                         is ignored while timing is on.  Results are bitwise those of the
                                         launches made one by one. */
    int ilu_level;                    /* levels of fill k of PFC_SUB_ILUK, 0..4 (default 2) */
} pfc_opts;

/* Per-step statistics.  res0 = ||F|| at the initial guess, res_final at the accepted
 * iterate, res_ref = ||F(phi^n)|| (the reference of the relative test; equals res0 for the
 * previous-step guess). */
typedef struct {
    int newton_its, gmres_its, ls_cuts, rejected, guess_used;
    double dt, t, energy, mass, res0, res_final, res_ref;
} pfc_step_stats;

typedef struct pfc_ctx pfc_ctx;

/* Fill *o with the defaults listed above (sub = 2x2(x2), overlap 2, ILU(0), FP64). */
void pfc_default_opts(pfc_opts* o);

/* Create a solver context for one grid.  stream is a hipStream_t (NULL: default
 * stream).  Allocates all device workspace (Krylov basis, factors); PFC_ENOMEM if the
 * device is out of memory, PFC_EINVAL for bad sizes or options.  Limits of the subdomain
 * solvers (PFC_EINVAL beyond them): an ILU(0) box's vector must fit in 160 KiB of LDS
 * (one spare element included) and its widest wavefront level (cells with equal
 * x + 3y + 7z) must hold at most 192 cells; exact LU is 2-D and bounds the box width by
 * the LDS its factorisation needs; ILU(k) needs a box of at most 65534 cells whose vector fits
 * in LDS and rows of at most 256 entries. */
pfc_status pfc_create(const pfc_grid* g, const pfc_model* m, const pfc_opts* o,
                      void* stream, pfc_ctx** out);
void pfc_destroy(pfc_ctx* ctx);
const char* pfc_last_error(const pfc_ctx* ctx);

/* Residual of Eq. (12): F = (Phi - phi)/dt - Delta_d mu_d(Phi, phi) - src.
 * src may be NULL (it is a time-averaged source for manufactured solutions).
 * If norm2 is not NULL the Euclidean norm of F is returned there (synchronises). */
pfc_status pfc_residual(pfc_ctx* ctx, const double* Phi, const double* phi, double dt,
                        const double* src, double* F, double* norm2);

/* Exact Jacobian action (Sec. 4, Eq. (19)) at (Phi, phi):
 * Jv = v/dt - Delta_d[(1-gamma)/2 v + Delta_d v + 1/2 Delta_d^2 v + c v],
 * c = (3 Phi^2 + 2 Phi phi + phi^2)/4. */
pfc_status pfc_jv(pfc_ctx* ctx, const double* Phi, const double* phi, double dt,
                  const double* v, double* Jv);

/* Assemble the subdomain matrices A_k = R_k J R_k^T (Eq. (25); equal to the zero-ring
 * subdomain problem of Eq. (26)) at (Phi, phi, dt) and factor them (ILU(0) on the
 * stencil pattern in natural order, or exact LU).  PFC_EPIVOT on a zero pivot. */
pfc_status pfc_ras_setup(pfc_ctx* ctx, const double* Phi, const double* phi, double dt);

/* z = sum_k (R_k^0)^T inv(A_k) R_k^delta r  (left-RAS, Eq. (23)) with the factors of the
 * last pfc_ras_setup; when mass_project is set, z is then shifted to zero mean. */
pfc_status pfc_ras_apply(pfc_ctx* ctx, const double* r, double* z);

/* Discrete free energy F_d (Eq. (8)) and mass sum(phi) * cell volume (synchronises). */
pfc_status pfc_energy(pfc_ctx* ctx, const double* phi, double* energy, double* mass);

/* Solve J x = b at (Phi, phi, dt) by right-preconditioned FGMRES(restart) from x = 0 with
 * the current factors, stopping at ||b - J x|| <= max(rtol ||b||, atol).  Returns the
 * iteration count and the final estimated residual norm (synchronises). */
pfc_status pfc_gmres(pfc_ctx* ctx, const double* Phi, const double* phi, double dt,
                     const double* b, double* x, double rtol, double atol,
                     int* iterations, double* res_norm);

/* One nonlinear solve (Sec. 4): Newton from the iterate in Phi (in/out) for the old
 * level phi and step dt; factors once at the first iteration and reuses them.
 * PFC_ENOTCONV if eps_r/eps_a are not met in newton_maxit iterations (synchronises). */
pfc_status pfc_newton(pfc_ctx* ctx, const double* phi, double dt, double* Phi,
                      pfc_step_stats* st);

/* One time step: dt from Eq. (16) and the stored energy history, initial guess, Newton,
 * energy and mass of the accepted solution.  phi holds phi^n on entry and phi^(n+1)
 * on return.  On a failed solve dt is halved (down to dt_min/16, max_retries times)
 * and the step retried from phi^n.  The first call after pfc_reset uses dt_min. */
pfc_status pfc_step(pfc_ctx* ctx, double* phi, pfc_step_stats* st);

/* The Newton initial guess Phi_0 of one step phi^n -> phi^(n+1) of size dt (Sec. 4: the
 * paper starts from the previous solution), from explicit history instead of the context's:
 *   kind PFC_GUESS_PREVIOUS: X = phi (phi_prev, dt, dt_prev ignored; may be NULL / 0);
 *   kind PFC_GUESS_EXTRAP:   X = phi + (dt/dt_prev) (phi - phi_prev);
 *   kind PFC_GUESS_LEARNED:  X = phi + s_o y, y = the attached network (include/pfc_net.h) at
 *                            x[0] = (phi - mean phi)/s_a, x[1] = (dt/dt_prev)(phi - phi_prev)/s_b.
 * When mass_project is set, the extrapolated and learned guesses are then shifted by a
 * constant to the mass of phi.  This is the computation pfc_step makes with its stored history
 * (there with the fallbacks described at pfc_step); it serves callers that run their own time
 * loop and tests.  phi, phi_prev, X: device FP64 fields of the context's grid; X aliases neither
 * input.  PFC_EINVAL for a bad kind, missing phi_prev or non-positive dt/dt_prev (kinds 1, 2),
 * or the learned kind without an attached network.  Enqueues only. */
pfc_status pfc_guess(pfc_ctx* ctx, int kind, const double* phi, const double* phi_prev, double dt,
                     double dt_prev, double* X);

/* Forget the time history (step counter, energies, previous solution). */
pfc_status pfc_reset(pfc_ctx* ctx);

/* Checkpoint: write phi (device) and the time history a restart needs (step count, t,
 * F^n, F^(n-1), dt_(n-1) of Eq. (16), and phi^(n-1) for the extrapolated and learned
 * guesses) to the file at path (binary, little-endian, with the grid and the model for
 * checking).  Factors are not saved: a restarted run factors at its first step.
 * pfc_checkpoint_load reads such a file into phi (device) and the context; PFC_EINVAL if the
 * file is not a checkpoint of this grid and model (the context is then unchanged).  A run
 * with precond_lag = 0 continues from a checkpoint exactly as it would have without one.
 * Both synchronise the stream. */
pfc_status pfc_checkpoint_save(pfc_ctx* ctx, const double* phi, const char* path);
pfc_status pfc_checkpoint_load(pfc_ctx* ctx, double* phi, const char* path);

/* The residual of pfc_residual (same kernel, bitwise the same F and norm) without a context
 * and without allocating: for callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc).  2-D grids only (PFC_EUNSUP for
 * dim 3, whose residual needs two grid-sized work vectors); M = 1 and periodic; n >= 8 per
 * axis, dt > 0, F aliasing neither input (PFC_EINVAL otherwise).  Phi, phi, src (nullable), F:
 * device FP64 [ny][nx]; stream: hipStream_t (NULL = default).  The kernel's per-block partial
 * sums of ||F||^2 (at most 1024) go to a fixed 8 KiB device array of the library, one per GPU,
 * kept until the process ends; calls that overlap on one GPU race on it.  With norm2 (host)
 * the call synchronises the stream and returns ||F||_2 (PFC_ENAN if not finite); without it,
 * it only enqueues.  PFC_EHIP on a HIP error. */
pfc_status pfc_residual_noalloc(const pfc_grid* g, const pfc_model* m, const double* Phi, const double* phi,
                                double dt, const double* src, double* F, double* norm2, void* stream);

/* Per-kernel timing (bit which of opts.timing): which = 0 preconditioner apply, 1 residual,
 * 2 Jacobian action, 3 factorisation.  Returns the launch count and the summed
 * event-measured duration in milliseconds since the last pfc_reset.  Single-kernel regions
 * (2-D residual and Jacobian action, every apply) are timed by the kernel dispatch itself
 * (hipExtLaunchKernel start/stop events); the others by events recorded around them.
 * Synchronises the context stream.  which = 4 gives the number of Arnoldi-step graph
 * launches (opts.use_graph) and 0 ms. */
pfc_status pfc_kernel_time(pfc_ctx* ctx, int which, long* count, double* total_ms);

#ifdef __cplusplus
}
#endif
#endif /* PFC_H */
