/*
 * lbm_axi adjoint — reverse-mode derivative of the axisymmetric Shan–Chen
 * step and the interface-radius loss, FP64, on one MI355X.
 *
 * The forward step is the method of Srivastava et al. (arXiv:1310.1871,
 * Sec. II; see lbm_axi.h).  These entry points differentiate it by hand:
 * the vector-Jacobian product of one step with respect to the state and to
 * (G, tau), the derivative of the initial equilibrium with respect to the
 * initial density, and the ray-integral interface radius used as a shape
 * observable (a reading: the paper fixes no interface-shape observable; its
 * drop test measures the radial intercept A(t), Sec. IV.B).
 *
 * All arrays are FP64 device arrays unless the name starts with h_; states
 * and adjoints are [9][nr][nz] (the library's population layout), fields
 * [nr][nz].  The caller owns every buffer and the stream; calls are
 * asynchronous on hip_stream.  Return codes are the LBM_AXI_* codes of
 * lbm_axi.h.
 */
#ifndef LBM_AXI_ADJOINT_H
#define LBM_AXI_ADJOINT_H

#include <stddef.h>
#include <stdint.h>

#include "lbm_axi.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Bytes of FP64 scratch lbm_axi_adjoint_step and lbm_axi_adjoint_run need
 * for an nz x nr grid: the node fields that pass from one reverse kernel to
 * the next (the part of the density adjoint that goes through the psi
 * stencils; two sets of F-bar scaled by -G psi in two components and of
 * exp(-rho/rho0)) and two sums per tile for dL/dG and dL/dtau (56 B per node
 * and 32 B per tile of 16 x 16 nodes, or of 16 x 8 on grids with fewer than
 * 192 of the larger tiles); 0 if the size is invalid.  The adjoint needs
 * nz >= 4 and nr >= 6 (the psi window mirrors up to six rows at the axis
 * and the wall), nz (nr + 12) < 2^31, and one FP64 state, 72 nz nr bytes,
 * below 4 GiB (its kernels address a state with 32-bit byte offsets); other
 * sizes give 0 here and LBM_AXI_EINVAL from the calls. */
size_t lbm_axi_adjoint_workspace_bytes(int32_t nz, int32_t nr);

/* One reverse step.  With f' = step(f; G, tau) (post-streaming states,
 * lbm_axi_step's update), writes d_lam = (df'/df)^T d_lam_next and, if
 * d_grad_acc is not NULL, adds <d_lam_next, df'/dG> and
 * <d_lam_next, df'/dtau> to d_grad_acc[0] and d_grad_acc[1].  p must have
 * precision LBM_AXI_FP64 and flags 0 (LBM_AXI_EUNSUP otherwise).  d_lam must not alias
 * d_lam_next or d_f.  d_ws: at least lbm_axi_adjoint_workspace_bytes. */
int lbm_axi_adjoint_step(const lbm_axi_params* p, const double* d_f, const double* d_lam_next, double* d_lam,
                         double* d_grad_acc, void* d_ws, size_t ws_bytes, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * reverse step as lbm_axi_adjoint_step, with its scratch in a static device
 * array of LBM_AXI_NOALLOC_SCRATCH_BYTES (24 MiB) that the library holds on
 * every GPU it runs on until the process ends, instead of a workspace
 * argument.  Grids whose lbm_axi_adjoint_workspace_bytes exceed it (beyond
 * about 449 000 nodes, e.g. 768 x 512 fits; the 256 x 128 drop needs 1.9 MB) return
 * LBM_AXI_ENOMEM with a message.  The caller passes inputs and outputs as
 * for lbm_axi_adjoint_step.  Allocates nothing (no hipMalloc, hipFree or
 * allocating library call); the first call on a device looks the array's
 * address up.  Every call on one GPU uses that GPU's one array: calls that
 * overlap on a GPU (other streams, other threads) race and must be
 * serialised by the caller.  The array keeps the last call's contents; the
 * step overwrites everything it reads. */
#define LBM_AXI_NOALLOC_SCRATCH_BYTES (24u << 20)
int lbm_axi_adjoint_step_noalloc(const lbm_axi_params* p, const double* d_f, const double* d_lam_next, double* d_lam,
                                 double* d_grad_acc, void* hip_stream);

/* k reverse steps over a recorded segment (lbm_axi_record, FP64):
 * d_states holds f^{t0}, ..., f^{t0+k-1} ([k][9][nr][nz]).  On entry d_lam
 * holds lam^{t0+k} = dL/df^{t0+k}; on return it holds lam^{t0}, the same
 * values as k calls of lbm_axi_adjoint_step from the last state back to the
 * first.  d_tmp: scratch of 9 nz nr doubles (not aliasing d_lam).
 * d_grad_acc (may be NULL) accumulates dL/dG, dL/dtau over the k steps:
 * the per-tile partial sums run over the steps in the workspace and are
 * reduced once at the end, so these two values equal those of the single
 * steps up to the order of the additions.  Between steps lam stays split
 * in two parts (in d_tmp or d_lam, and in the workspace), which the next
 * step's gathers add; the last step adds them.  k >= 0 (0 leaves d_lam
 * unchanged). */
int lbm_axi_adjoint_run(const lbm_axi_params* p, const double* d_states, int32_t k, double* d_lam, double* d_tmp,
                        double* d_grad_acc, void* d_ws, size_t ws_bytes, void* hip_stream);

/* Adjoint of the initial equilibrium f_i = f^eq_i(rho0, u0) (appendix,
 * Eq. e_distribution): d_rho0_bar = sum_i d_lam0_i df^eq_i/drho0.
 * d_uz0 / d_ur0 may be NULL (zero initial velocity).  LBM_AXI_EINVAL for
 * NULL d_lam0 / d_rho0_bar or nz, nr < 1. */
int lbm_axi_init_vjp(const double* d_lam0, const double* d_uz0, const double* d_ur0, int32_t nz, int32_t nr,
                     double* d_rho0_bar, void* hip_stream);

/* rho = sum_i f_i of a state (Eq. hydro_var).  LBM_AXI_EINVAL for NULL
 * pointers or nz, nr < 1. */
int lbm_axi_density(const double* d_f, int32_t nz, int32_t nr, double* d_rho, void* hip_stream);

/* Host-side construction of the ray-integral interface radius
 *   r(theta_m) = sum_k ds * phi(zc + s_k cos theta_m, s_k sin theta_m),
 *   s_k = (k + 1/2) ds, k < floor(s_max / ds),
 * with phi the bilinear interpolant of node values (rows mirrored below row
 * 0, clamped above the last row, z periodic), as a sparse matrix in host
 * arrays: ray-major CSR (h_row_ptr[n_rays+1], h_col, h_val) and node-major
 * CSR (h_node_ptr[n_nodes+1], h_nodes, h_node_row, h_node_val).  Call once
 * with the array pointers NULL to get *h_nnz and *h_n_nodes, then with
 * arrays of capacity cap >= nnz (LBM_AXI_ENOMEM otherwise).  LBM_AXI_EINVAL
 * (message in lbm_axi_last_error) for ds <= 0, s_max < 0, non-finite zc,
 * ds, s_max or angle, |zc| + s_max > 1e9, more than 2^24 samples per ray,
 * or nz nr or nnz beyond 32-bit indices; LBM_AXI_ENOMEM when the host
 * allocation fails. */
int lbm_axi_ray_weights(int32_t nz, int32_t nr, double zc, const double* h_thetas, int32_t n_rays, double ds,
                        double s_max, int32_t cap, int32_t* h_row_ptr, int32_t* h_col, double* h_val,
                        int32_t* h_node_ptr, int32_t* h_nodes, int32_t* h_node_row, double* h_node_val,
                        int32_t* h_nnz, int32_t* h_n_nodes);

/* d_out[m] = sum_k val_mk (rho[col_mk] - rho_g) / (rho_l - rho_g) with the
 * ray-major matrix on the device (fixed-order FP64 reduction).
 * LBM_AXI_EINVAL for NULL pointers, n_rows < 0, or rho_l, rho_g not finite
 * or equal; n_rows = 0 does nothing. */
int lbm_axi_ray_forward(const double* d_rho, int32_t n_rows, const int32_t* d_row_ptr, const int32_t* d_col,
                        const double* d_val, double rho_l, double rho_g, double* d_out, void* hip_stream);

/* Adjoint of lbm_axi_ray_forward applied to rho = sum_i f_i:
 * d_lam_i(x) += sum_m d_rbar[m] w_mx / (rho_l - rho_g) for every direction
 * i, with the node-major matrix on the device (built by lbm_axi_ray_weights
 * for the same nz, nr: d_lam holds nine planes of nz nr values).
 * LBM_AXI_EINVAL for NULL pointers, n_nodes < 0, nz, nr < 1, nz nr beyond
 * 32-bit indices, or rho_l, rho_g not finite or equal. */
int lbm_axi_ray_vjp(const double* d_rbar, int32_t n_nodes, const int32_t* d_node_ptr, const int32_t* d_node_row,
                    const double* d_node_val, const int32_t* d_nodes, double rho_l, double rho_g, int32_t nz,
                    int32_t nr, double* d_lam, void* hip_stream);

/* *d_loss += sum_m (d_r[m] - d_target[m])^2 and, if d_rbar is not NULL,
 * d_rbar[m] = 2 (d_r[m] - d_target[m]) (FP64).  LBM_AXI_EINVAL for NULL
 * d_r, d_target, d_loss or m < 0. */
int lbm_axi_misfit(const double* d_r, const double* d_target, int32_t m, double* d_loss, double* d_rbar,
                   void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* LBM_AXI_ADJOINT_H */
