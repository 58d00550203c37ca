/*
 * pfc_net.h -- C ABI of the learned Newton initial guess in libpfc.
 *
 * The paper starts Newton at the previous solution (Sec. 4, Eqs. (17)-(20)); this part of
 * the library adds a small convolutional network that predicts the increment
 * phi^(n+1) - phi^n of one time step of size dt, trained on solver trajectories by the
 * library's own kernels.  Newton's residual test still decides when a step is solved
 * (Eq. (20)), so the accepted solution does not depend on the guess; only the iteration
 * count does.  The adaptive step of Sec. 3 (Eq. (16)) spans decades of dt, so dt is an input.
 *
 * Network (fixed architecture)
 *   input  x: two planes, [2][ny][nx] FP32, periodic in both axes, and a condition c (the
 *          log step size below), a constant third plane
 *   4 layers of 3x3 periodic cross-correlation, channels 2 (+ c) -> 32 -> 32 -> 32 -> 1,
 *   tanh after the first three, no activation on the output:
 *       z_l[o](y,x) = b_l[o] + sum_{c,dy,dx} bf16(W_l[o][c][dy][dx]) a_(l-1)[c](y+dy-1, x+dx-1)
 *   and z_1[o] gains c u1[o]: the taps of the constant plane sum to u1[o] (FP32).
 *   Convolution weights are rounded to bfloat16 (nearest, ties to even) for every use;
 *   accumulation is FP32; biases, u1 and the master weights stay FP32.  The two inner 32 -> 32
 *   layers run on the matrix cores with each FP32 activation split into two bfloat16
 *   parts (so the products carry about 16 significant bits of the activation); in a
 *   forward (inference) pass the output layer is formed the same way, as per-tap sums
 *   of the third layer's activations that are added up over the 3x3 neighbourhood.
 *   Parameters, flat FP32, PFC_NET_NPARAM of them, in this order:
 *       W1[32][2][3][3] b1[32] W2[32][32][3][3] b2[32] W3[32][32][3][3] b3[32] W4[1][32][3][3] b4[1]
 *       u1[32]
 *   Loss of one sample: mean over cells of (y - t)^2.
 *
 * Use as the initial guess (pfc_opts.guess = PFC_GUESS_LEARNED, after pfc_attach_net):
 *   l = ln(dt_n/dt_ref), g = exp(beta l + gamma l^2) (the typical size of one step's
 *   increment at dt_n relative to dt_ref), c = l/s_c,
 *   x[0] = (phi^n - mean phi^n)/s_a,  x[1] = (dt_n/dt_(n-1)) (phi^n - phi^(n-1))/(s_b g),
 *   Phi_0 = phi^n + s_o g y, shifted to the mass of phi^n.
 *   When there is no phi^(n-1) yet, or dt_n lies outside the range [dt_lo, dt_hi] the
 *   network was trained on, the guess falls back to linear extrapolation (or the previous
 *   solution on the first step).
 *
 * Conventions: device pointers are FP32 arrays owned by the caller; work is enqueued on
 * the stream given at creation; calls returning host values synchronise it.  Errors are
 * pfc_status codes (include/pfc.h); pfc_net_last_error gives a message.
 */
#ifndef PFC_NET_H
#define PFC_NET_H

#include "pfc.h"

#ifdef __cplusplus
extern "C" {
#endif

enum { PFC_NET_NPARAM = 19425, PFC_NET_CIN = 2, PFC_NET_WIDTH = 32 };

typedef struct pfc_net pfc_net;

/* Create a network with all parameters zero (stream: hipStream_t, NULL = default). */
pfc_status pfc_net_create(void* stream, pfc_net** out);
void pfc_net_destroy(pfc_net* net);
const char* pfc_net_last_error(const pfc_net* net);

/* Copy PFC_NET_NPARAM FP32 master parameters from / to HOST memory.  set_params also
 * resets the Adam moments and step counter. */
pfc_status pfc_net_set_params(pfc_net* net, const float* host_params);
pfc_status pfc_net_get_params(pfc_net* net, float* host_params);

/* y = network(x; c = cond).  x: device [2][ny][nx], y: device [ny][nx]; ny, nx >= 3; cond
 * finite.  Grows the activation workspace to the largest grid seen (PFC_ENOMEM on failure).
 * An inference pass: the activations are not kept (pfc_net_gradient runs its own). */
pfc_status pfc_net_forward(pfc_net* net, const float* x, double cond, int ny, int nx, float* y);

/* Gradient of scale * loss(network(x; c = cond), t) with respect to the parameters (taken at
 * the bfloat16-rounded weights; d/du1 = cond d/db1), written to (accumulate = 0) or added to
 * (accumulate = 1) the network's gradient buffer.  If loss is not NULL the unscaled loss is
 * returned (synchronises). */
pfc_status pfc_net_gradient(pfc_net* net, const float* x, double cond, const float* t, int ny, int nx,
                            double scale, int accumulate, double* loss);

/* Copy the gradient buffer to HOST memory (PFC_NET_NPARAM floats). */
pfc_status pfc_net_get_gradient(pfc_net* net, float* host_grad);

/* One Adam step (Kingma & Ba, Algorithm 1, bias-corrected) on the master parameters with
 * the gradient buffer: beta1, beta2, eps as given, lr the step size. */
pfc_status pfc_net_adam(pfc_net* net, double lr, double beta1, double beta2, double eps);

/* Attach a trained network to a solver context for PFC_GUESS_LEARNED (2-D grids only;
 * PFC_EUNSUP otherwise).  scales = {s_a, s_b, s_o, s_c, beta, gamma} (host, 6 doubles),
 * finite, the first four positive; dt_range = {dt_ref, dt_lo, dt_hi} (host, 3 doubles): the
 * reference step and the range of step sizes the guess is used in (0 < dt_lo <= dt_hi;
 * PFC_EINVAL otherwise).  Allocates the context's own inference buffers (~0.4 KB per cell), so
 * several contexts, on different streams and host threads, may share one network; it
 * prepares the network's inference copy of its parameters (synchronising the network's
 * stream).  The context keeps the pointer, not a copy: the network must outlive its use
 * and must not be trained while attached (a step then fails with PFC_EINVAL until the
 * network is attached again).  NULL detaches. */
pfc_status pfc_attach_net(pfc_ctx* ctx, pfc_net* net, const double* scales, const double* dt_range);

#ifdef __cplusplus
}
#endif
#endif /* PFC_NET_H */
