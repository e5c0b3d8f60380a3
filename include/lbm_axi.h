/*
 * lbm_axi — axisymmetric Shan–Chen lattice Boltzmann on one MI355X (gfx950).
 *
 * C ABI of the hot path of Srivastava, Perlekar, ten Thije Boonkkamp, Verma,
 * Toschi, "Axisymmetric Multiphase Lattice Boltzmann Method"
 * (arXiv:1310.1871): the fused per-timestep D2Q9 update on the (z, r)
 * half-plane.
 *
 * Geometry (paper Sec. II.E): node (k, j) sits at z = k (k = 0..nz-1,
 * periodic) and r = j + 1/2 (j = 0..nr-1).  The axis r = 0 is a mid-grid
 * specular reflector; the outer wall r = nr is mid-grid bounce-back
 * (no-slip) or mid-grid specular reflection (free-slip).
 *
 * Field arrays passed through this interface are double[nr][nz], row-major,
 * z contiguous, in device memory unless the argument name starts with h_.
 * The caller allocates every device buffer (including the workspace) and
 * owns the HIP stream; the library never frees caller memory and never
 * allocates device memory.  Calls are asynchronous on the handle's stream
 * unless stated otherwise.
 *
 * Return codes: LBM_AXI_OK (0) or a negative LBM_AXI_E* code; the message of
 * the last failure on the calling thread is lbm_axi_last_error().
 */
#ifndef LBM_AXI_H
#define LBM_AXI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_AXI_OK 0
#define LBM_AXI_EINVAL (-1)     /* invalid argument or parameter */
#define LBM_AXI_ENOMEM (-2)     /* workspace too small */
#define LBM_AXI_EHIP (-3)       /* HIP runtime error (message in last_error) */
#define LBM_AXI_ENONFINITE (-4) /* a reduced diagnostic is NaN or Inf */
#define LBM_AXI_EUNSUP (-5)     /* combination not supported */
/* Positive return: success with a warning (the call took effect; the
 * message is in lbm_axi_last_error()). */
#define LBM_AXI_WARN_STABILITY 1 /* G < -6: outside the stability rule of thumb of Sec. II.D */

#define LBM_AXI_WALL_NOSLIP 0   /* mid-grid bounce-back */
#define LBM_AXI_WALL_FREESLIP 1 /* mid-grid specular reflection */

#define LBM_AXI_FP64 0          /* populations stored and collided in FP64 */
#define LBM_AXI_FP32_SHIFTED 1  /* FP32 storage of f_i - W_i rho_ref, FP32 collision */

/* flags: force incorporation.  0 (default) is the Shan–Chen velocity shift
 * of the paper's scheme (Sec. II.A, Eqs. ueq and uhydro).  LBM_AXI_FLAG_GUO
 * selects the forcing of Guo, Zheng and Shi (Phys. Rev. E 65, 046308, 2002),
 * the scheme the paper compares against in Sec. IV.A and Table I: f^eq at
 * the hydrodynamic velocity u = (j + F/2)/rho plus, in the collision,
 * (1 - 1/(2 tau)) W_i [3 (c_i - u) + 9 (c_i . u) c_i] . F.  Forces, sources
 * and boundary rules are the same.  The adjoint supports the default only. */
#define LBM_AXI_FLAG_GUO 4
/* flags: LBM_AXI_FLAG_NO_WALL_DERIV selects the other reading of the
 * derivative rule at the outer wall (Sec. II.E only states that derivative
 * terms vanish at the non-axis boundaries, not how).  Default: every field is reflected evenly across the wall and the
 * stencils run unchanged.  With this flag: F^{gamma,sym} is zero on the 4
 * rows next to the wall (its stencils reach 4 rows) and the velocity
 * derivatives in H_z, H_r are zero on the 2 rows next to the wall; the
 * other terms are unchanged.  May be combined with LBM_AXI_FLAG_GUO. */
#define LBM_AXI_FLAG_NO_WALL_DERIV 2
/* flags: LBM_AXI_FLAG_ZWALLS closes both ends of z with no-slip walls
 * (mid-grid bounce-back at z = -1/2 and z = nz - 1/2, Sec. II.E; the two
 * discs of the radial-flow test of Sec. III) instead of joining them
 * periodically.  psi is mirrored evenly across them for the Shan–Chen sum,
 * and, as Sec. II.E asks at the boundaries other than the axis, the
 * derivative terms are zero where their stencils would reach across:
 * F^{gamma,sym} on the 4 columns and the velocity derivatives of H on the 2
 * columns next to each wall.  Requires nz >= 8.  May be combined with the
 * other flags. */
#define LBM_AXI_FLAG_ZWALLS 8
/* flags: LBM_AXI_FLAG_MIDLINK selects the other reading of where the source
 * h_i is evaluated.  Sec. II.C places it at the mid-link, mid-step point
 * without giving its discretisation; by default it is the node value
 * h_i(x, t).  With this flag it is the average over the link,
 * (h_i(x) + h_i(x + c_i)) / 2, with h_i(y) = W_i (mass(y) + 3 c_i . H(y))
 * from the fields at y (across the axis the mirror node with H_r reversed,
 * across the outer wall the mirror node).  Each step then runs two kernels:
 * a moments pass that writes H and the mass source of every node (3 nz nr
 * doubles more workspace), and the step, on its run-time option path.  Not
 * with LBM_AXI_FLAG_ZWALLS or open rows; not in a batch or the adjoint. */
#define LBM_AXI_FLAG_MIDLINK 16

typedef struct lbm_axi_params {
    int32_t nz;        /* nodes along z (>= 1) */
    int32_t nr;        /* nodes along r (>= 6: reach of the derivative stencils) */
    double G;          /* Shan–Chen coupling (Sec. II.A, Eq. scforce); G < -6 is outside the
                          stability rule of thumb of Sec. II.D */
    double tau;        /* BGK relaxation time (> 1/2); nu = (tau - 1/2)/3 */
    double psi_rho0;   /* rho_0 of psi = rho_0 (1 - exp(-rho/rho_0)) (> 0; the paper uses 1) */
    double gz;         /* body acceleration along +z (pipe-flow test, Sec. III.A) */
    int32_t wall;      /* LBM_AXI_WALL_NOSLIP or LBM_AXI_WALL_FREESLIP */
    int32_t axisym;    /* 1: axisymmetric method; 0: plain planar Shan–Chen (test mode) */
    int32_t precision; /* LBM_AXI_FP64 or LBM_AXI_FP32_SHIFTED */
    int32_t flags;     /* LBM_AXI_FLAG_GUO | LBM_AXI_FLAG_NO_WALL_DERIV | LBM_AXI_FLAG_ZWALLS |
                          LBM_AXI_FLAG_MIDLINK; other bits: LBM_AXI_EUNSUP */
    double rho_ref;    /* shift of the FP32 storage (ignored in FP64) */
} lbm_axi_params;

typedef struct lbm_axi_ctx* lbm_axi_t;

/* Validate p without touching a device (the checks create makes).  Returns
 * LBM_AXI_OK, a negative error code, or LBM_AXI_WARN_STABILITY when
 * G < -6: Sec. II.D gives as a rule of thumb that the scheme stays stable
 * up to a liquid/vapour density ratio of about 35, reached at G = -6;
 * stronger coupling is allowed but may diverge. */
int lbm_axi_check_params(const lbm_axi_params* p);

/* Bytes of device workspace lbm_axi_create needs for these parameters (two
 * population buffers, each plane padded by 8 KiB inside the library, plus
 * reduction scratch).  0 if the parameters are invalid. */
size_t lbm_axi_workspace_bytes(const lbm_axi_params* p);

/* Validate p, bind the caller's workspace and stream, and initialise the
 * populations to f_i = f^eq_i(rho0, u0) (appendix, Eq. e_distribution),
 * the post-streaming state at t = 0.  d_rho0/d_uz0/d_ur0 are device fields;
 * d_uz0 and d_ur0 may be NULL (zero velocity).  The workspace must be at
 * least lbm_axi_workspace_bytes(p) bytes and 256-byte aligned and stays owned
 * by the caller; it must outlive the handle.  hip_stream is a hipStream_t
 * (NULL: the null stream).  On success *out receives the handle; the
 * return value is LBM_AXI_OK, or LBM_AXI_WARN_STABILITY when G < -6 (see
 * lbm_axi_check_params; the handle is valid). */
int lbm_axi_create(const lbm_axi_params* p, const double* d_rho0, const double* d_uz0,
                   const double* d_ur0, void* d_workspace, size_t ws_bytes, void* hip_stream,
                   lbm_axi_t* out);

/* Advance n >= 0 full time steps (Sec. II, Eq. lbm2d_mod_new with the
 * Shan–Chen force of Eq. scforce, the axisymmetric extra force of
 * Eq. scAxisExtra, the source terms of Eqs. condition_h/H_terms and the
 * boundary rules of Sec. II.E).  Asynchronous.  On a stream the caller is
 * capturing into a graph, the step kernels go into that graph (the library
 * does not replay graphs of its own then) and n must be even
 * (LBM_AXI_EINVAL otherwise): the handle keeps which of its two buffers
 * holds the state on the host, and a replay runs the captured launches. */
int lbm_axi_step(lbm_axi_t h, int64_t n);

/* Density rho = sum f_i (Eq. hydro_var) and hydrodynamic velocity
 * u = (sum c_i f_i + F/2)/rho (Eq. uhydro, F the total force) of the current
 * state, in FP64, into device fields double[nr][nz].  Any pointer may be
 * NULL to skip that field.  Asynchronous. */
int lbm_axi_moments(lbm_axi_t h, double* d_rho, double* d_uz, double* d_ur);

/* FP64 global diagnostics of the current state, reduced on the device in a
 * fixed order and copied to host memory h_out[LBM_AXI_NREDUCE]:
 *   [0] 3D mass      sum 2 pi r rho           (Sec. II.B, Sec. II.C)
 *   [1] 3D z-momentum sum 2 pi r rho u_z
 *   [2] kinetic energy E_ke = pi sum r rho |u|^2   (Sec. III)
 *   [3] 2D mass      sum rho
 * Synchronises the stream.  Returns LBM_AXI_ENONFINITE (with h_out filled)
 * if any value is NaN or Inf. */
#define LBM_AXI_NREDUCE 4
int lbm_axi_reduce(lbm_axi_t h, double* h_out);

/* FP64 interface diagnostics of the current state (Sec. IV.A-IV.C).  In
 * every column z the interface radius R(z) is the outermost crossing of
 * rho = rho_mid along r, interpolated linearly between the two nodes around
 * it (nr - 1/2 if the top node is at or above rho_mid, 0 if no node of the
 * column is).  d_radius: device array of nz doubles for R(z), or NULL.
 * h_out[LBM_AXI_NINTERFACE] (host):
 *   [0] A = R(z_col): radial intercept of a drop centred at column z_col
 *       (the oscillation amplitude of Sec. IV.B)
 *   [1] min_z R(z): neck radius of a thread (Sec. IV.C)
 *   [2] max_z R(z)
 *   [3] min_z rho on the row next to the axis: below rho_mid the thread has
 *       broken (Sec. IV.C)
 *   [4] rho_in  = rho(z_col, row 0)
 *   [5] rho_out = rho(0, row nr - 1)
 *   [6] dp = p(rho_in) - p(rho_out) with p = rho/3 + (G/6) psi^2 (Sec. II.A,
 *       Eq. pressure): the Laplace pressure jump of Sec. IV.A
 * 0 <= z_col < nz.  Synchronises the stream. */
#define LBM_AXI_NINTERFACE 7
int lbm_axi_interface(lbm_axi_t h, double rho_mid, int32_t z_col, double* d_radius, double* h_out);

/* Open boundaries (Sec. II.E: a prescribed velocity or pressure is imposed
 * through the equilibrium populations, before streaming).  After every
 * collision the populations of row in_row become f^eq(rho_in, u_in(z)) with
 * u_in(z) = (d_uz_in[z], d_ur_in[z]) (device arrays of nz doubles, copied
 * into the workspace on the stream by this call), and those of row out_row
 * become f^eq(rho_out, u) with u the hydrodynamic velocity of the node one
 * row below (an open outlet at imposed pressure passes the interior velocity
 * on).  The flow domain is the rows between them; the rows outside still
 * step but take no part in it.  The derivative terms are zero on rows whose
 * stencils reach past an open row: F^{gamma,sym} within 3 rows inside it,
 * the velocity derivatives within 1 row inside it, and every row outside.
 * in_row = out_row = -1 turns both off (the default); either may be -1
 * alone.  -1 <= in_row < out_row < nr when both are set, out_row >= 1,
 * rho_in, rho_out > 0.  The step runs the kernel's run-time option path
 * while open rows are set.  Not supported by the adjoint. */
int lbm_axi_set_open(lbm_axi_t h, int32_t in_row, double rho_in, const double* d_uz_in, const double* d_ur_in,
                     int32_t out_row, double rho_out);

/* Drops on the axis once a thread has broken up (Sec. IV.C: the thread
 * breaks into two or more drops when kappa* < 1).  A drop is a maximal run
 * of consecutive columns, periodic in z, whose axis node (row 0) has
 * rho >= rho_mid.  Its 3D volume is sum_z pi R(z)^2, the solid of revolution
 * of the interface radius R(z) of lbm_axi_interface, and its centre the
 * volume-weighted mean column, counted from the first column with
 * rho < rho_mid on the axis onward and taken modulo nz.  Drops are listed in
 * that order.
 *   h_count (host): number of drops; 0 if no axis node reaches rho_mid; -1
 *     if every axis node does (an unbroken thread).
 *   h_volume[k], h_centre[k] (host, max_drops entries each) for
 *     k < min(count, max_drops).
 * 0 <= max_drops <= LBM_AXI_MAX_DROPS (h_volume and h_centre may be NULL
 * when it is 0).  Synchronises the stream. */
#define LBM_AXI_MAX_DROPS 64
int lbm_axi_drops(lbm_axi_t h, double rho_mid, int32_t max_drops, int32_t* h_count, double* h_volume,
                  double* h_centre);

/* The current populations f_i as FP64, into the device array
 * double[9][nr][nz] (d_f, 72 nz nr bytes): the stored values, plus
 * W_i rho_ref in FP32 shifted storage (the decode is done on the device, in
 * double).  Asynchronous. */
int lbm_axi_populations(lbm_axi_t h, double* d_f);

/* Size in bytes of the population state as the caller sees it: 9 nz nr
 * values of the storage type, structure of arrays [9][nr][nz] with no
 * padding between the planes (the library's own buffers pad them). */
size_t lbm_axi_state_bytes(lbm_axi_t h);

/* Device-to-device copy of the current state into d_dst / from d_src
 * (lbm_axi_state_bytes bytes, the plain [9][nr][nz] layout).
 * Checkpoint/resume.  Asynchronous. */
int lbm_axi_get_state(lbm_axi_t h, void* d_dst);
int lbm_axi_set_state(lbm_axi_t h, const void* d_src);

/* Record a trajectory segment: with the handle at state f^t, writes
 * f^t, f^{t+1}, ..., f^{t+n-1} to d_states (n consecutive blocks of
 * lbm_axi_state_bytes bytes each, the plain [9][nr][nz] layout) and leaves the
 * handle at f^{t+n-1} (n - 1 steps).  n >= 1.  For checkpointed reverse
 * sweeps, which need every state of a segment.  Asynchronous. */
int lbm_axi_record(lbm_axi_t h, int64_t n, void* d_states);

/* Step kernel selection (the arithmetic is the same; the organisation of
 * the work differs).  LBM_AXI_KERNEL_TILE: one workgroup per tile of nodes,
 * every tile recomputing a 6-node halo, each XCD walking a run of whole tile
 * rows.  LBM_AXI_KERNEL_STRIP: each workgroup walks a band of 64 columns up
 * a chunk of chunk_rows rows, keeping the halo rows it has computed (needs
 * nz >= 70; the Guo and wall-derivative options only, no open rows).
 * LBM_AXI_KERNEL_TILE_ALTERNATE: the tile kernel walking its runs from the
 * end on every other step (each step starts on the tiles the previous one
 * ended on).  LBM_AXI_KERNEL_TILE_COLUMNS: the tile kernel with each XCD
 * walking its rows of tiles column by column (where the runs are whole
 * rows).  LBM_AXI_KERNEL_TILE_PAIRS: the tile kernel with each thread
 * holding two z-adjacent nodes, moved in one 16-byte access per plane (8
 * bytes in FP32) where nz is even and z periodic; it applies to lattices of
 * at least 1024 tiles of 64 x 16 (smaller ones run the tile kernel).  The
 * tile variants give the same populations bit for bit; chunk_rows is read by
 * the strip only.  create selects the tile kernel, the fastest on MI355X
 * (4096 x 512 FP64: 75 us per step, against 77 us alternating, 78 us by
 * columns, 80 us with node pairs and 93 us for the strip with chunks of 43
 * rows); set_open leaves the strip for it.  Returns LBM_AXI_EUNSUP when the
 * strip does not apply. */
#define LBM_AXI_KERNEL_TILE 0
#define LBM_AXI_KERNEL_STRIP 1
#define LBM_AXI_KERNEL_TILE_ALTERNATE 2
#define LBM_AXI_KERNEL_TILE_COLUMNS 3
#define LBM_AXI_KERNEL_TILE_PAIRS 4
int lbm_axi_set_kernel(lbm_axi_t h, int32_t kind, int32_t chunk_rows);

/* Rebind the stream later calls are issued on. */
int lbm_axi_set_stream(lbm_axi_t h, void* hip_stream);

/* Replace G and tau of an existing handle (same validation as create,
 * including the LBM_AXI_WARN_STABILITY return). */
int lbm_axi_set_coupling(lbm_axi_t h, double G, double tau);

/* Release the handle (not the caller's workspace).  NULL is ignored. */
void lbm_axi_destroy(lbm_axi_t h);

/* Message of the last failed call on this thread ("" if none). */
const char* lbm_axi_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LBM_AXI_H */
