/*
 * pfc_batch.h -- many independent PFC instances of uneven size advanced together.
 *
 * Each instance is a full solver context (include/pfc.h) with its own grid, model and
 * options and its own HIP stream; a pool of host worker threads advances the instances one
 * time step per pfc_batch_step call (Sec. 3, Eq. (16) and the Newton-Krylov-Schwarz solve
 * of Sec. 4, per instance).  The solve of one instance synchronises its stream once per
 * Arnoldi step and per Newton test, so running the instances from several threads on
 * several streams keeps the GPU busy while any one instance waits on the host; instances
 * are handed out largest first.  Results are bitwise identical to stepping each instance
 * alone with pfc_step.
 *
 * Conventions as in pfc.h: fields are caller-owned FP64 device arrays; errors are
 * pfc_status codes; pfc_batch_last_error gives a message.  A batch is driven from one host
 * thread at a time.
 */
#ifndef PFC_BATCH_H
#define PFC_BATCH_H

#include "pfc.h"
#include "pfc_net.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pfc_batch pfc_batch;

/* Create count >= 1 instances: instance i has grids[i], models[i], opts[i] (validated as
 * by pfc_create; the first failure is returned and nothing is kept).  workers host threads
 * (1 <= workers <= 64, at most count) step them.  Streams are created by the library at
 * the default priority and destroyed with the batch. */
pfc_status pfc_batch_create(int count, const pfc_grid* grids, const pfc_model* models, const pfc_opts* opts,
                            int workers, pfc_batch** out);
void pfc_batch_destroy(pfc_batch* b);
const char* pfc_batch_last_error(const pfc_batch* b);

/* Advance every instance by one time step.  phis[i]: instance i's field on the device
 * (phi^n in, phi^(n+1) out).  st[i] and status[i] receive instance i's statistics and
 * status (both arrays of count entries, host memory).  Returns PFC_OK when every instance
 * succeeded, else the status of the first failed instance in index order; the other
 * instances are stepped regardless.  Returns after all instances finished. */
pfc_status pfc_batch_step(pfc_batch* b, double* const* phis, pfc_step_stats* st, pfc_status* status);

/* pfc_reset on every instance. */
pfc_status pfc_batch_reset(pfc_batch* b);

/* pfc_attach_net on every instance (one network shared read-only by all of them). */
pfc_status pfc_batch_attach_net(pfc_batch* b, pfc_net* net, const double* scales, const double* dt_range);

/* Instance i's context (owned by the batch; for pfc_energy, pfc_kernel_time and the like,
 * not to be destroyed by the caller). */
pfc_status pfc_batch_instance(pfc_batch* b, int i, pfc_ctx** out);

#ifdef __cplusplus
}
#endif
#endif /* PFC_BATCH_H */
