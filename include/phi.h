/* phi.h -- MI355X (gfx950) library for the radio-interferometric measurement
 * operator Phi = Theta G F Z, its adjoint, and the l2-ball data-fidelity dual
 * step of primal-dual forward-backward (PDFB) imaging.
 *
 * Paper: Thouvenin, Dabbech et al., "Parallel faceted imaging in radio
 * interferometry via proximal splitting (Faceted HyperSARA): II. Code and real
 * data proof of concept" (arXiv 2209.07604).
 *
 *   Section 2.1, eq. (1): y_l = Phi_l x_l + n_l,  Phi_l = Theta_l G_l F Z;
 *       Z zero-pads and scales the N-pixel image into the K-point grid, F is
 *       the 2-D DFT on that grid, G interpolates (one compact-support row per
 *       visibility, widened by DDE / w-kernel convolution: Sections 3.1-3.2),
 *       Theta whitens.  Visibilities are split into blocks (l, b).
 *   Section 2.2, eq. (2): one data-fidelity term per block, the indicator of
 *       B(y_{l,b}, eps_{l,b}) = {z : ||z - y_{l,b}||_2 <= eps_{l,b}}.
 *   Section 2.2.3: PDFB splits these terms; their dual update is
 *       Phi x~ -> l2-ball projection -> Phi^dagger.
 *
 * Conventions (all fixed here; the paper leaves them open):
 *   - Image x_l: float32, row-major [Ny][Nx]; pixel (p, q) has offsets
 *     pbar = p - Ny/2, qbar = q - Nx/2 from the phase centre.
 *   - Grid: Ky = 2 Ny, Kx = 2 Nx (2x oversampling).  Z puts
 *     s_y[p] s_x[q] x[p][q] at cell (pbar mod Ky, qbar mod Kx); F is the
 *     unnormalised forward DFT exp(-2 pi i k.n / K); the adjoint uses the
 *     unnormalised inverse DFT (no 1/K).
 *   - G: row m is a dense S_m x S_m window (S_m odd, 1..21) whose entry
 *     (i, j) multiplies grid cell ((b_y + i) mod Ky, (b_x + j) mod Kx).
 *   - Theta: one real positive scalar theta_b per block.
 *   - Visibilities: complex64 (float re, float im) interleaved.
 *   - phi_adjoint returns the adjoint for real images: Re(Z^T F^H G^H Theta v).
 *
 * Order of visibilities.  Hot calls read and write visibility vectors in
 * *plan order*: blocks in channel-major order, and inside each block the
 * order the plan chose (sorted by window position).  Convert user-order
 * vectors once with phi_to_plan_order / phi_from_plan_order.
 *
 * Memory.  The caller owns every buffer.  Device buffers (prefix d_) are
 * allocated by the caller (e.g. PyTorch); the plan's own device state lives
 * in one caller-allocated workspace whose size phi_plan_workspace_size gives.
 * Host buffers (prefix h_) are read during the call only.  The library makes
 * no device allocations of its own.
 *
 * Streams.  `stream` is a hipStream_t passed as void*; every device call is
 * asynchronous on it.  A plan must not be used from two streams at once.
 *
 * Errors.  Functions return phi_status and never throw.  Argument checks run
 * before any HIP call.  On error no output is guaranteed.
 */
#ifndef PHI_H_
#define PHI_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct phi_plan_s* phi_plan;

typedef enum {
  PHI_OK = 0,
  PHI_ERR_ARG = -1,          /* null pointer or invalid enum/flag            */
  PHI_ERR_SHAPE = -2,        /* sizes inconsistent (odd Ny, block counts...) */
  PHI_ERR_RANGE = -3,        /* value out of range (S, base, theta, eps...)  */
  PHI_ERR_WORKSPACE = -4,    /* workspace missing, too small or misaligned   */
  PHI_ERR_NONFINITE = -5,    /* a device-side norm was NaN / Inf             */
  PHI_ERR_HIP = -6,          /* a HIP runtime call failed                    */
  PHI_ERR_UNSUPPORTED = -7,  /* size beyond what the kernels are built for   */
  PHI_ERR_STATE = -8         /* call order (e.g. G not loaded, not bound)    */
} phi_status;

/* Storage of the G coefficients on the device.  Arithmetic is FP32 in all
 * cases; the per-block norms and projection scale are FP64. */
typedef enum {
  PHI_G_C64 = 0,   /* complex float32                                   */
  PHI_G_F16 = 1,   /* complex float16 (RNE from the host values)        */
  PHI_G_BF16 = 2,  /* complex bfloat16 (RNE from the host values)       */
  PHI_G_KB = 3     /* no stored G: direction-independent Kaiser-Bessel
                      rows psi(kappa_y - b_y - i) psi(kappa_x - b_x - j),
                      psi(d) = I0(beta sqrt(1 - (2d/J)^2)) / I0(beta),
                      evaluated in the kernels (FP32, I0 by Abramowitz &
                      Stegun 9.8.1-9.8.2) from per-visibility kappa - b
                      loaded with phi_plan_load_kb.  J = S of every
                      visibility (one of 3, 5, 7, 9, 11), beta from Beatty
                      et al. (2005) at 2x oversampling:
                      pi sqrt((J/2)^2 1.5^2 - 0.8).                     */
} phi_gprec;

/* Host window element type accepted by phi_plan_load_g. */
typedef enum { PHI_HOST_C128 = 0, PHI_HOST_C64 = 1 } phi_host_type;

/* Execution flags. */
enum {
  PHI_PER_CHANNEL = 1,  /* launch every stage per channel (the plain form)
                           instead of one launch over all channels/blocks  */
  PHI_GRAPH = 2,        /* replay the dual step from a captured hipGraph    */
  PHI_PERSISTENT = 4,   /* G stages run as a persistent grid over work items */
  PHI_FUSED_GH = 8,     /* dual step in one pass over G (c and G^H c from
                           the same taps; sigma * scale applied to v+, and
                           times theta in the merge) instead of a G pass
                           and a G^H pass; used with stored G where the
                           item's grid tile and one accumulator per wave
                           fit a work-group's LDS (e.g. 16-cell tiles)      */
  PHI_DR = 16           /* at plan creation only: also build the plan of the
                           visibility-gridding reduction (phi_dr_setup) in
                           the same workspace; stored G only, kept in
                           complex64 (g_prec applies to the reduced rows)    */
};

typedef struct {
  int32_t n_channels;          /* L >= 1                                     */
  int32_t ny, nx;              /* image size, even, 8 <= n <= 4096           */
  const int32_t* h_n_blocks;   /* [L] blocks per channel, >= 1               */
  const int64_t* h_n_vis;      /* [sum B] visibilities per block (>= 0),
                                  channel-major                              */
  const int32_t* h_base;       /* [M_tot][2] window origin (b_y, b_x),
                                  0 <= b_y < Ky, 0 <= b_x < Kx; user order   */
  const uint8_t* h_stencil;    /* [M_tot] window size S, odd, 1 <= S <= 21
                                  (PHI_G_KB: one J in {3, 5, 7, 9, 11})      */
  const double* h_theta;       /* [sum B] whitening theta_b > 0 (NULL => 1)  */
  const double* h_scale_y;     /* [Ny] Z scale s_y (deapodisation)           */
  const double* h_scale_x;     /* [Nx] Z scale s_x                           */
  int32_t g_prec;              /* phi_gprec                                  */
  int32_t flags;               /* PHI_PER_CHANNEL | PHI_GRAPH | ...          */
  int32_t tile;                /* uv tile edge T for G^H binning: 16, 32 or 64;
                                  0 picks 32                                 */
  int32_t persist_blocks;      /* work-groups of a persistent G stage (0 =>
                                  4 per compute unit when PHI_PERSISTENT)    */
} phi_desc;

typedef struct {
  int64_t n_vis_total;         /* M_tot                                      */
  int64_t n_taps;              /* sum_m S_m^2                                */
  int64_t n_items;             /* G work items (tile x visibility range)     */
  int64_t n_blocks_total;      /* sum B                                      */
  int64_t g_bytes;             /* device bytes of packed G                   */
  int64_t partial_bytes;       /* device bytes of the G^H tile partials      */
  int64_t workspace_bytes;     /* total workspace                            */
  double alg_bytes_dual_step;  /* algorithmic HBM bytes of one dual step     */
  double alg_bytes_gather;     /* ... of the G gather stage                  */
  double alg_bytes_scatter;    /* ... of the G^H scatter stage               */
  int32_t ky, kx, tile, n_stages;
  int32_t persist_blocks;      /* persistent G-stage grid in use (0 = one
                                  work-group per item)                       */
  int32_t fused;               /* 1 if the dual step runs in one pass over G
                                  (PHI_FUSED_GH set and usable)              */
  int32_t pitch_classes;       /* launches of the one-pass step over all
                                  channels: items grouped by tile pitch, each
                                  group with LDS sized for its pitch, largest
                                  items first.  Pitches are grouped from the
                                  smallest up until a group holds 8192 items
                                  (environment PHI_PITCH_CLASS_ITEMS, read at
                                  phi_plan_create, overrides; >= 1)          */
  /* plans created with PHI_DR: the reduced rows and their stored taps, to be
     weighed against n_vis_total and n_taps (the reduction pays only when the
     rows of Lam H hold fewer bytes than G)                                   */
  int64_t dr_rows;             /* M' = sum_b |S_b| (0 without PHI_DR)        */
  int64_t dr_taps;             /* sum over reduced rows of s^2               */
  int64_t dr_bytes;            /* device bytes of the reduced rows           */
  int32_t dr_max_window;       /* largest reduced-row window edge s          */
  int32_t reduced;             /* 1 on the handle phi_dr_plan returns        */
  int32_t fft_image_first;     /* 1 if the 2-D DFT runs columns first, on the
                                  image (grids of 3072 ... 8192 rows with
                                  Nx / 2 a multiple of 8), else rows first   */
  int32_t reserved;
} phi_info;

/* Validate `desc`, sort visibilities and build the work lists (host only,
 * no HIP call).  Host arrays are read during the call.  On success *out owns
 * a plan that phi_plan_destroy releases. */
phi_status phi_plan_create(const phi_desc* desc, phi_plan* out);
phi_status phi_plan_destroy(phi_plan plan);

/* Bytes of device workspace the plan needs (256-byte aligned start). */
phi_status phi_plan_workspace_size(phi_plan plan, size_t* bytes);

/* Attach the caller's workspace and upload plan metadata, twiddles and the
 * Z scales.  The workspace must stay allocated while the plan is used. */
phi_status phi_plan_bind(phi_plan plan, void* d_workspace, size_t bytes, void* stream);

/* Pack the windows of block `block` (0 <= block < sum B) into the device
 * G store, converting to the plan's g_prec with round-to-nearest-even.
 * h_windows holds that block's windows in user order, each S*S row-major,
 * back to back, as complex128 or complex64 (phi_host_type).  Synchronous
 * with respect to h_windows (it can be freed on return). */
phi_status phi_plan_load_g(phi_plan plan, int64_t block, const void* h_windows,
                           int32_t host_type, void* stream);

/* Kaiser-Bessel mode (g_prec = PHI_G_KB): load block `block`'s continuous
 * grid coordinates h_kappa [n][2] = (kappa_y, kappa_x) (host FP64, user
 * order, kappa = omega K / (2 pi) in grid cells, any period).  The window
 * origin floor(kappa - J/2) + 1 of every visibility must equal, mod K, the
 * origin given at plan creation, else PHI_ERR_RANGE (nothing is loaded);
 * non-finite kappa: PHI_ERR_RANGE.  The plan keeps kappa - b in FP32.  On a
 * plan with stored G this call returns PHI_ERR_STATE, as phi_plan_load_g
 * does on a Kaiser-Bessel plan.  Synchronous with respect to h_kappa. */
phi_status phi_plan_load_kb(phi_plan plan, int64_t block, const double* h_kappa, void* stream);

/* ---------------------------------------------------------------------------
 * Device-side G builder (Sections 3.1-3.2: each row of G is the
 * interpolation kernel convolved with the Fourier kernels of the w-term and
 * of the antenna pair's DDEs).  Rows are computed in FP64 on the GPU from
 * per-visibility tables and stored, rounded once (RNE) to the plan's
 * precision, into block `block`'s G in plan order: the same result
 * phi_plan_load_g gives for the same FP64 windows.
 *
 * Row of visibility m (user order within the block):
 *   psi(d) = I0(beta sqrt(1 - (2d/J)^2)) / I0(beta) (0 outside |d| <= J/2),
 *     beta = pi sqrt((J/2)^2 1.5^2 - 0.8), sampled per axis at
 *     kappa - (b + i), i = 0..J-1, b = floor(kappa - J/2) + 1;
 *   w-kernel per axis, k = -h..h: c_k = cos^2(pi k / (2 (h + 1)))
 *     exp(-i pi k^2 / (4 max(a, 1/2))), divided by sum_k c_k (h = 0: 1);
 *   u = psi (*) c per axis (length J + 2h), window = outer(u_y, u_x),
 *   then, with DDEs, window (*) (d_i (*) conj(flip(d_j))) (d: the antennas'
 *     sa x sa kernels, pair edge sd = 2 sa - 1; sd = 1 without DDE);
 *   S = J + 2h + sd - 1, first cell b - h - (sd - 1)/2 per axis (mod K).
 * S and the first cell must equal those declared for the visibility at plan
 * creation, else PHI_ERR_RANGE (the block's G is then undefined and the block
 * counts as not loaded).  Synchronous.  Not available on PHI_G_KB plans
 * (PHI_ERR_STATE).
 */
typedef struct {
  int32_t J;       /* Kaiser-Bessel width: odd, 3..11                        */
  int32_t n_ant;   /* antennas in d_dde (0 without DDEs)                     */
  int32_t sa;      /* antenna kernel edge: odd, 1..7 (ignored without DDEs)  */
  int32_t reserved;
} phi_gbuild;

/* d_kappa: float64 [n][2] device, (kappa_y, kappa_x) in grid cells, user
 * order of the block (n = its visibility count); d_h: int32 [n] w half-widths
 * >= 0; d_a: float64 [n] w-chirp parameters; d_ant: int32 [n][2] antenna
 * indices (i, j) in [0, n_ant), or (-1, -1) for a row without DDE, or NULL
 * for no DDEs at all; d_dde: complex128 [n_ant][sa][sa] (NULL iff d_ant is
 * NULL).  All device pointers, read on `stream`. */
phi_status phi_plan_build_g(phi_plan plan, int64_t block, const phi_gbuild* desc, const double* d_kappa,
                            const int32_t* d_h, const double* d_a, const int32_t* d_ant, const void* d_dde,
                            void* stream);

/* Copy block `block`'s stored G to host memory in user order, S*S taps per
 * visibility back to back, converted exactly from the stored precision to
 * host_type (PHI_HOST_C128 or PHI_HOST_C64).  Synchronous.  PHI_ERR_STATE on
 * a Kaiser-Bessel plan or a block not loaded. */
phi_status phi_plan_read_g(phi_plan plan, int64_t block, void* h_windows, int32_t host_type, void* stream);

/* Replace the per-block whitening scalars (host [sum B], > 0). */
phi_status phi_plan_set_theta(phi_plan plan, const double* h_theta, void* stream);

phi_status phi_plan_get_info(phi_plan plan, phi_info* info);

/* Change the execution flags (PHI_PER_CHANNEL | PHI_GRAPH | PHI_PERSISTENT)
 * of a plan; the data it holds is unchanged.  Drops a cached graph. */
phi_status phi_plan_set_flags(phi_plan plan, int32_t flags);

/* Permute a complex64 visibility vector [M_tot] between user order (blocks
 * concatenated, each in the caller's order) and plan order. */
phi_status phi_to_plan_order(phi_plan plan, const void* d_user, void* d_plan, void* stream);
phi_status phi_from_plan_order(phi_plan plan, const void* d_plan, void* d_user, void* stream);

/* y = Phi x for every block (eq. 1).  d_x: float32 [L][Ny][Nx];
 * d_y: complex64 [M_tot], plan order. */
phi_status phi_forward(phi_plan plan, const float* d_x, void* d_y, void* stream);

/* x = sum_b Re Phi_{l,b}^dagger v_b for every channel.  d_v: complex64
 * [M_tot] plan order; d_x: float32 [L][Ny][Nx] (overwritten). */
phi_status phi_adjoint(phi_plan plan, const void* d_v, float* d_x, void* stream);

/* Data-fidelity dual step of PDFB for every block (l, b) (eq. 2), with
 * c = v/sigma + Phi x~ - y:
 *   rho_b = ||c||_2,  res_b = ||Phi x~ - y||_2            (FP64)
 *   v+    = sigma (1 - eps/rho) c if rho > eps, else 0    (= v + sigma Phi x~
 *           - sigma P_B(y, eps)((v + sigma Phi x~)/sigma), the Moreau form)
 *   grad_l = sum_b Re Phi_{l,b}^dagger v+_b
 * d_xt: float32 [L][Ny][Nx]; d_v: complex64 [M_tot] plan order, in/out
 * (v on entry, v+ on return); d_y: complex64 [M_tot] plan order;
 * d_eps: float64 [sum B]; d_sigma: float64 [sum B] or NULL (=> 1);
 * d_grad: float32 [L][Ny][Nx]; d_rho, d_res: float64 [sum B] (may be NULL).
 * A NaN or Inf norm is recorded and reported by phi_plan_check. */
phi_status l2ball_dual_step(phi_plan plan, const float* d_xt, void* d_v, const void* d_y,
                            const double* d_eps, const double* d_sigma, float* d_grad,
                            double* d_rho, double* d_res, void* stream);

/* Synchronise `stream` and report PHI_ERR_NONFINITE if any dual step since
 * the last check produced a non-finite norm (the flag is then cleared). */
phi_status phi_plan_check(phi_plan plan, void* stream);

/* Set the tuning choices by hand (what phi_plan_autotune picks): the tile
 * edge (one the plan was created with: 16/32/64 where they divide the grid,
 * or only desc->tile if one was given) and the persistent G-stage grid size
 * (0 = one work-group per item). */
phi_status phi_plan_set_tuning(phi_plan plan, int32_t tile, int32_t persist_blocks, void* stream);

/* Per-stage timing with HIP events recorded on `stream` around each stage
 * of the calls that follow (enable = 1), or off (enable = 0). */
phi_status phi_plan_set_timing(phi_plan plan, int32_t enable);
/* Synchronise and return accumulated milliseconds per stage and the number
 * of timed calls; names[i] are static strings.  n_stages <= max_stages. */
phi_status phi_plan_get_timing(phi_plan plan, int32_t max_stages, double* ms,
                               const char** names, int32_t* n_stages, int64_t* n_calls);

/* Time the candidate tile edges (16, 32, 64, where they divide the grid),
 * G-stage launch shapes (one work-group per item, or a persistent grid of 4
 * work-groups per compute unit) and, with stored G where its LDS fits, the
 * one-pass dual step against the two passes, on the bound plan with its
 * loaded G: `reps` rounds of the G stages + merge on scratch vectors inside
 * the workspace.  Keeps the fastest combination (sets or clears
 * PHI_FUSED_GH).  Overwrites the grid buffers.  Synchronous. */
phi_status phi_plan_autotune(phi_plan plan, void* stream, int32_t reps);

/* ---------------------------------------------------------------------------
 * Per-channel analysis quantities, all channels at once, asynchronous on
 * `stream`.  They reuse the plan's forward and adjoint stages and its
 * visibility scratch (calls on one plan must not overlap).
 *
 * PSF and its normalisation (the paper's residual-image definition among its
 * evaluation metrics): delta is the image that is 1 at the phase centre
 * (Ny/2, Nx/2) and 0 elsewhere; the PSF of channel l is Phi_l^dagger Phi_l
 * delta and eta_l = 1 / (its value at the phase centre) makes it peak at 1.
 * d_psf: float32 [L][Ny][Nx] out; d_peak: float64 [L] out (may be NULL).
 */
phi_status phi_psf(phi_plan plan, float* d_psf, double* d_peak, void* stream);

/* Residual image r_l = eta_l Re Phi_l^dagger (y_l - Phi_l x_l) (same passage).
 * d_x: float32 [L][Ny][Nx]; d_y: complex64 [M_tot] plan order; d_eta: float64
 * [L] or NULL (=> 1); d_r: float32 [L][Ny][Nx] out. */
phi_status phi_residual_image(phi_plan plan, const float* d_x, const void* d_y, const double* d_eta,
                              float* d_r, void* stream);

/* Power method for ||Phi_l||^2, the largest eigenvalue of Phi_l^dagger Phi_l
 * (the bound on the step sizes of the primal-dual iteration, Section 2.2):
 * x_l <- x_l / ||x_l||, then n_iter times x_l <- A x_l / ||A x_l|| with
 * nu_l = ||A x_l|| (norms in FP64).  d_x: float32 [L][Ny][Nx], the start
 * vector in (nonzero in every channel) and the last unit iterate out; d_tmp:
 * float32 [L][Ny][Nx] scratch (distinct from d_x); d_nu: float64 [L] out;
 * n_iter >= 1 (else PHI_ERR_RANGE). */
phi_status phi_power_iteration(phi_plan plan, float* d_x, float* d_tmp, int32_t n_iter, double* d_nu,
                               void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the power
 * method of phi_power_iteration with its scratch image in a fixed device
 * array of 32 MiB per GPU (held from library load until the process ends)
 * instead of d_tmp.  It allocates nothing; the plan must be bound.  Channels
 * x pixels (L Ny Nx) above 8 Mi (32 MiB of float32) return
 * PHI_ERR_UNSUPPORTED.  Every call on one GPU shares that GPU's array, so
 * calls that overlap on one GPU race (serialise them on one stream). */
phi_status phi_power_iteration_static(phi_plan plan, float* d_x, int32_t n_iter, double* d_nu, void* stream);

/* ---------------------------------------------------------------------------
 * Regularizer-free primal-dual forward-backward (PDFB) loop: eq. (2) with the
 * regularization reduced to the non-negativity constraint on the image cube
 * (Section 2.2), i.e. find x_l >= 0 with ||Phi_{l,b} x_l - y_{l,b}|| <=
 * eps_{l,b}.  One iteration, data-fidelity dual update first:
 *   v+  = l2ball_dual_step at x~ (gives grad_l = sum_b Re Phi_{l,b}^H v+_b)
 *   x+  = max(x - tau_l grad_l, 0),  x~ = 2 x+ - x,  x <- x+
 *   eps = phi_eps_update(...)        (only with an adaptive rule)
 * It converges for tau_l ||sum_b sigma_b Phi_{l,b}^H Phi_{l,b}|| < 1, e.g.
 * sigma_b = 1 / ||Phi_l||^2 (phi_power_iteration) and tau_l < 1.
 *
 * Adaptive l2 bounds (effective noise estimation, Section 3.3: update the
 * noise-level estimates and l2 bounds during the iteration, fix them once the
 * bounds are satisfied), with the update rule of Dabbech et al. (2018) that
 * the paper cites for it.  Per block b of channel l whose bound is not fixed,
 * after the primal update: since_b += 1; if freeze and res_b <= lambda_hi
 * eps_b the bound is fixed; otherwise, if ||x+ - x||^2 < var_tol^2 ||x+||^2
 * (channel l; a zero image never counts as settled), since_b >= min_gap and
 * res_b is outside [lambda_lo eps_b, lambda_hi eps_b]:
 *   eps_b <- lambda_mix res_b + (1 - lambda_mix) eps_b, since_b <- 0,
 *   count_b += 1.
 * res_b is the residual ||Phi_b x~ - y_b|| of the same iteration's dual step.
 * Valid rules: 0 < lambda_lo <= 1 <= lambda_hi, 0 < lambda_mix <= 1,
 * var_tol >= 0, min_gap >= 0, all finite (else PHI_ERR_RANGE).
 */
typedef struct {
  double lambda_lo;    /* lower edge of the accepted band (e.g. 0.99)      */
  double lambda_hi;    /* upper edge; also the fixing threshold (1.01)     */
  double lambda_mix;   /* weight of the residual in the update (0.618)     */
  double var_tol;      /* relative image variation that counts as settled  */
  int32_t min_gap;     /* iterations between two updates of one block      */
  int32_t freeze;      /* nonzero: fix a bound once res_b <= lambda_hi eps */
} phi_eps_rule;

/* Primal step for every channel (FP32 image arithmetic, NaN propagates):
 * x+ = max(x - tau_l grad_l, 0), x~ = 2 x+ - x, then x <- x+.
 * d_x, d_xt: float32 [L][Ny][Nx] in/out (x~ is only written);
 * d_grad: float32 [L][Ny][Nx]; d_tau: float64 [L] (>= 0, not checked on the
 * device); d_var: float64 [L][2] out, (||x+ - x||^2, ||x+||^2) in FP64 with a
 * fixed summation order, or NULL.  d_x, d_xt and d_grad must be distinct. */
phi_status phi_pdfb_primal(phi_plan plan, float* d_x, float* d_xt, const float* d_grad, const double* d_tau,
                           double* d_var, void* stream);

/* One application of the adaptive rule to every block.  d_res: float64
 * [sum B] (res_b); d_var: float64 [L][2] from phi_pdfb_primal; d_eps:
 * float64 [sum B] in/out; d_state: int32 [sum B][3] in/out (since, fixed,
 * count), zero at the start of a run; rule: host struct, read during the
 * call. */
phi_status phi_eps_update(phi_plan plan, const double* d_res, const double* d_var, const phi_eps_rule* rule,
                          double* d_eps, int32_t* d_state, void* stream);

/* n_iter >= 1 PDFB iterations (above), asynchronous on `stream`, no host
 * synchronisation.  d_x, d_xt: float32 [L][Ny][Nx] in/out (x~ = x at the
 * start of a run); d_v: complex64 [M_tot] plan order, in/out; d_y, d_eps,
 * d_sigma, d_rho, d_res: as for l2ball_dual_step (d_eps is updated in place
 * when rule != NULL); d_tau: float64 [L]; d_grad: float32 [L][Ny][Nx]
 * scratch (last iteration's grad on return); d_var: float64 [L][2] out;
 * rule: NULL for fixed bounds, else d_state (int32 [sum B][3]) is required.
 * d_rho, d_res and d_var hold the last iteration's values. */
phi_status phi_pdfb_run(phi_plan plan, float* d_x, float* d_xt, void* d_v, const void* d_y, double* d_eps,
                        const double* d_sigma, const double* d_tau, int32_t n_iter, const phi_eps_rule* rule,
                        int32_t* d_state, float* d_grad, double* d_rho, double* d_res, double* d_var,
                        void* stream);

/* ---------------------------------------------------------------------------
 * Visibility-gridding dimensionality reduction (Section 3.4, eqs. 4-5), per
 * data block b with whitening theta_b, computed on the device from the
 * plan's stored G:
 *   H = G^H Theta^H Theta G (Hermitian), S_b = {p : H_pp > 0} (M'_b cells),
 *   Lam_p = H_pp^(-1/2) on S_b, y' = Lam G^H Theta^H y, Phi' = Lam H F Z,
 * and the l2 ball of the reduced data has radius eps' (the caller's choice,
 * e.g. eps'^2 = M' + 2 sqrt(M'), the chi-square rule with M' points).
 *
 * A plan created with PHI_DR computes, at creation and on the host, the
 * support of every block (the cells its windows cover) and, for every
 * support cell p, the window of row p of Lam H: the smallest odd square
 * holding every window that covers p (edge s from S to 2 S - 1).  Those rows
 * form the reduced plan: same channels, blocks and theta, M'_b rows per
 * block, stored in g_prec.  The plan's own G is then kept in complex64
 * whatever g_prec says: Lam rescales each row by its windows' taps at p,
 * which at the support's edge are the windows' smallest taps, and FP16 /
 * BF16 storage would not keep their relative precision.  Creation fails with
 * PHI_ERR_UNSUPPORTED where a row's window would exceed 21 x 21 (dense
 * coverage with S > 11) or the grid is smaller than 42 cells; with
 * PHI_ERR_ARG for g_prec = PHI_G_KB.  phi_plan_workspace_size then covers
 * both plans, which share the grid buffers (calls on the two must not
 * overlap), and phi_plan_get_info reports M', the reduced taps and bytes.
 * Reduced-order vectors hold the rows in the reduced plan's order.
 */

/* Row values and gridded data (the device set-up of the reduction).  The
 * plan must be bound with every block's G loaded.  Row p of Lam H is
 * theta_b Lam0_p (H0)_pq with H0 = G^H G and Lam0 = H0_pp^(-1/2): the rows
 * store Lam0 H0 (rounded once to the plan's precision) and the reduced plan
 * applies theta_b; y' = Lam0 G^H y.  Sums run in FP64 in a fixed order
 * (windows covering p in plan order).  d_y: complex64 [M_tot] plan order
 * (NULL: y' = 0); d_yred: complex64 [M'] reduced order, out; h_m_red: host
 * int64 [sum B] out, M'_b (may be NULL).  Asynchronous on `stream`.
 * PHI_ERR_STATE without PHI_DR, unbound or with G not loaded. */
phi_status phi_dr_setup(phi_plan plan, const void* d_y, void* d_yred, int64_t* h_m_red, void* stream);

/* The reduced data-fidelity dual step: l2ball_dual_step of Phi' on the
 * reduced plan (same arguments and semantics with M' rows: d_vred and
 * d_yred complex64 [M'] reduced order, d_eps_red and d_sigma [sum B];
 * grad_l = sum_b Re Phi'_{l,b}^dagger v'+_b).  PHI_ERR_STATE before
 * phi_dr_setup. */
phi_status l2ball_dual_step_dr(phi_plan plan, const float* d_xt, void* d_vred, const void* d_yred,
                               const double* d_eps_red, const double* d_sigma, float* d_grad, double* d_rho,
                               double* d_res, void* stream);

/* The reduced plan as a handle owned by `plan` (destroyed with it; it is not
 * bound, destroyed or loaded on its own: those calls return PHI_ERR_STATE).
 * Every other call applies to it: phi_forward is Phi', phi_adjoint
 * Re Phi'^dagger, phi_plan_autotune, phi_plan_set_flags and timing tune and
 * time the reduced step, phi_plan_read_g reads its rows. */
phi_status phi_dr_plan(phi_plan plan, phi_plan* reduced);

/* Host copies, in reduced order, of each row's cell p = p_y Kx + p_x
 * (h_cells, int64 [M']), its window origin (h_base, int32 [M'][2]) and edge
 * (h_stencil, uint8 [M']); any pointer may be NULL.  Host only (works before
 * phi_plan_bind). */
phi_status phi_dr_rows(phi_plan plan, int64_t* h_cells, int32_t* h_base, uint8_t* h_stencil);

const char* phi_status_string(phi_status s);

#ifdef __cplusplus
}
#endif
#endif /* PHI_H_ */
