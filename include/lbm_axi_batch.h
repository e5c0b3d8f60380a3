/*
 * lbm_axi batch — many independent axisymmetric Shan–Chen lattices (uneven
 * sizes and parameters) advanced together on one MI355X.
 *
 * Each instance is the method of lbm_axi.h (Srivastava et al.,
 * arXiv:1310.1871, Sec. II) with its own lbm_axi_params; all instances of a
 * batch share the storage precision.  One step of the whole batch is one
 * launch of a persistent kernel whose workgroups stride over a work list of
 * (instance, tile) items; on a non-null stream the launches are captured
 * once into a HIP graph (two launches per graph, one per buffer parity) and
 * replayed.  The tile shape, the grid size and the work-list order come from
 * an autotuner that times the candidates on the batch itself.
 *
 * Memory: the caller provides one device workspace of
 * lbm_axi_batch_workspace_bytes bytes (256-byte aligned) holding every
 * instance's two population buffers, a backup buffer used by the autotuner
 * and the device tables; the library allocates no device memory.  Return
 * codes are those of lbm_axi.h.
 */
#ifndef LBM_AXI_BATCH_H
#define LBM_AXI_BATCH_H

#include <stddef.h>
#include <stdint.h>

#include "lbm_axi.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_axi_batch* lbm_axi_batch_t;

/* Bytes of device workspace for n_inst instances with parameters ps[0..n).
 * 0 if any parameter set is invalid or the precisions differ. */
size_t lbm_axi_batch_workspace_bytes(const lbm_axi_params* ps, int32_t n_inst);

/* Create the batch: validates ps, binds the workspace and stream, and
 * initialises instance k to f^eq(rho0[k], 0) from the device field
 * h_d_rho0[k] (a host array of n_inst device pointers to double[nr][nz]).
 * The stream must outlive the handle.  Returns LBM_AXI_WARN_STABILITY (the
 * batch is created) when an instance has G < -6 (lbm_axi_check_params). */
int lbm_axi_batch_create(const lbm_axi_params* ps, int32_t n_inst, const double* const* h_d_rho0,
                         void* d_workspace, size_t ws_bytes, void* hip_stream, lbm_axi_batch_t* out);

/* Advance every instance by n steps with the persistent kernel (graph
 * replay on a non-null stream, direct launches on the null stream).  On a
 * stream the caller is capturing into a graph, the launches go into that
 * graph and n must be even (LBM_AXI_EINVAL otherwise), as for
 * lbm_axi_step. */
int lbm_axi_batch_step(lbm_axi_batch_t b, int64_t n);

/* The same n steps with one ordinary launch per instance per step (the
 * baseline the persistent launch is compared with). */
int lbm_axi_batch_step_per_instance(lbm_axi_batch_t b, int64_t n);

/* Density and hydrodynamic velocity (FP64) of instance k into device
 * fields [nr_k][nz_k]; pointers may be NULL. */
int lbm_axi_batch_moments(lbm_axi_batch_t b, int32_t k, double* d_rho, double* d_uz, double* d_ur);

/* Device-to-device copy of instance k's populations (its lbm_axi_params'
 * storage type, plain layout [9][nr][nz]: 9 nz nr values, no padding
 * between the planes, which the batch's own buffers have) into d_dst. */
int lbm_axi_batch_get_state(lbm_axi_batch_t b, int32_t k, void* d_dst);

/* Instance k's populations f_i as FP64 into the device array
 * double[9][nr_k][nz_k]: the stored values, plus W_i rho_ref in FP32
 * shifted storage (decoded on the device, in double).  Asynchronous. */
int lbm_axi_batch_populations(lbm_axi_batch_t b, int32_t k, double* d_f);

/* Number of kernel configurations compiled for the batch's precision, and
 * the tile shape (z, r) and workgroup size of configuration c. */
int32_t lbm_axi_batch_num_configs(lbm_axi_batch_t b);
int lbm_axi_batch_config_info(lbm_axi_batch_t b, int32_t c, int32_t* h_tz, int32_t* h_tr, int32_t* h_threads);

/* Select configuration c, grid = grid_per_cu * (compute units) workgroups
 * (capped by the number of work items) and work-list order
 * (0: instance by instance, 1: largest instance first, 2: round robin over
 * instances).  Invalidates captured graphs. */
int lbm_axi_batch_set_schedule(lbm_axi_batch_t b, int32_t c, int32_t grid_per_cu, int32_t order);

/* Autotuner: times every (configuration, grid_per_cu in 1..4, order) on the
 * batch itself for steps_per_trial steps each (after one warm-up step),
 * restores the populations after every trial, and selects the fastest.
 * Writes the chosen (c, grid_per_cu, order) and its time per step in
 * microseconds to h_choice[0..2] and *h_us.  Synchronises the stream. */
int lbm_axi_batch_autotune(lbm_axi_batch_t b, int32_t steps_per_trial, int32_t* h_choice, double* h_us);

/* Total nodes of the batch (sum nz * nr). */
int64_t lbm_axi_batch_nodes(lbm_axi_batch_t b);

void lbm_axi_batch_destroy(lbm_axi_batch_t b);

#ifdef __cplusplus
}
#endif

#endif /* LBM_AXI_BATCH_H */
