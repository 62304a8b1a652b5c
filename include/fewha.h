/*
 * fewha.h -- C ABI of the MI355X (gfx950) implementation of the FEWHA tomography hot path:
 * the matrix-free Jacobi-PCG solve of the wavelet-domain MAP normal equations
 *
 *     (W Ahat^T C_eta^-1 Ahat W^T + alpha D) c = W Ahat^T C_eta^-1 s        (Eq. (fewha))
 *
 * followed by deformable-mirror fitting (Alg. 1), after Stadler, Biasi, Manetti, Ramlau,
 * "Real-time implementation of an iterative solver for atmospheric tomography" (arXiv 2009.00946).
 *
 * Conventions shared by every call
 * --------------------------------
 * Pointers named d_* are DEVICE pointers (HIP global memory on the plan's GPU) holding
 * contiguous arrays of the plan's precision (float for FEWHA_FP32, double for FEWHA_FP64)
 * unless stated otherwise.  Pointers named h_* are host pointers.  `stream` is a hipStream_t
 * passed as void* (NULL = the default stream).  The caller owns every buffer it passes; the
 * library never keeps a pointer to a caller buffer after a call returns.
 *
 * Vector layouts (sizes from fewha_sizes):
 *   coefficient vector c (n_coef): layers concatenated in configuration order, each n x n
 *     row-major (row = y, column = x) in the Mallat in-place pyramid: top-left LL, top-right
 *     x-high/y-low, bottom-left x-low/y-high, bottom-right HH, recursing J times into LL.
 *   layer vector (n_coef): the same concatenation of n x n row-major nodal values (finite
 *     element domain; node (k, l) of layer i at ((l - n/2) spacing, (k - n/2) spacing)).
 *   slope vector s (n_slopes): per guide star the s^x plane then the s^y plane, each
 *     n_sub x n_sub row-major; entries of inactive subapertures are ignored on input and
 *     written as 0 on output.
 *   actuator vector a (n_act): DMs concatenated, each n_act x n_act row-major; actuator (i, j)
 *     at ((j - (n_act-1)/2) pitch, (i - (n_act-1)/2) pitch).
 *
 * Execution: fewha_plan_create and fewha_plan_bind are synchronous.  Every other call that
 * takes a stream only enqueues kernels on it and returns (no host synchronisation, no device
 * allocation), so a sequence of calls can be captured into a HIP graph.  A plan may be used by
 * one stream at a time; calls on one plan from two streams at once race on its workspace.
 *
 * Errors: every call returns FEWHA_OK (0) or a negative fewha_status; nothing is thrown across
 * the ABI.  Numerical failures inside a solve (PCG breakdown, non-finite reductions) are
 * recorded in a device status word that fewha_last_status reads (it synchronises the device).
 * With the environment variable FEWHA_DEBUG set, a FEWHA_ERR_HIP return also prints the failing
 * HIP call or launch, its source location and HIP's error string on stderr.
 *
 * HIP runtime: the library must run on the HIP runtime of the process that owns the device.
 * Loaded into a process that already has one (e.g. PyTorch's), it binds to it through the
 * shared soname; the Python binding imports torch before loading the library for that reason.
 */
#ifndef FEWHA_H
#define FEWHA_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fewha_plan fewha_plan;

typedef enum {
    FEWHA_OK = 0,
    FEWHA_ERR_INVALID_ARG = -1, /* null pointer, bad size, not a power of two, sigma <= 0, ... */
    FEWHA_ERR_GEOMETRY = -2,    /* a projected node or actuator leaves its layer grid, LGS below a layer */
    FEWHA_ERR_UNSUPPORTED = -3, /* configuration outside the implemented limits (see fewha_plan_create) */
    FEWHA_ERR_HIP = -4,         /* a HIP runtime call or kernel launch failed */
    FEWHA_ERR_WORKSPACE = -5,   /* plan not bound, or workspace too small / misaligned */
    FEWHA_ERR_BREAKDOWN = -6,   /* PCG denominator mu - rho beta / alpha_old <= 0 (device status) */
    FEWHA_ERR_NONFINITE = -7    /* NaN or Inf in a PCG reduction (device status) */
} fewha_status;

typedef enum { FEWHA_FP32 = 0, FEWHA_FP64 = 1 } fewha_precision;

/* PCG start flags for fewha_pcg_solve */
#define FEWHA_COLD 0 /* c = b_prev = r_prev = 0 before the frame */
#define FEWHA_WARM 1 /* warm restart from the caller's c and the plan's b_prev, r_prev */
#define FEWHA_REFRESH 2 /* warm restart from the caller's c with the residual recomputed as
                           b - M c (one application of M more) instead of carried by
                           (b - b_prev) + r_prev: clears the rounding a long FP32 chain of
                           carried residuals accumulates (about 1e-7 of |b| per frame) */

/* One Shack-Hartmann wavefront sensor / guide star (Sec. 2.1). */
typedef struct {
    int n_sub;        /* subapertures per side (>= 1); subaperture size d = D / n_sub */
    double theta_x;   /* guide-star direction, rad */
    double theta_y;
    double gs_height; /* m; 0 = natural guide star at infinity, > 0 = laser guide star height H */
    double sigma;     /* noise standard deviation per slope (rad); C_eta^-1 = sigma^-2 on active slopes */
} fewha_wfs;

/* One turbulent layer, discretised on an n x n node grid (Table 1, Table 2). */
typedef struct {
    double height;     /* m */
    double cn2_weight; /* fractional Cn2 weight gamma (> 0) */
    double spacing;    /* node spacing delta, m */
    int n;             /* power of two, n >= max(2, 2^J) */
} fewha_layer;

/* One deformable mirror (Alg. 1 fitting target). */
typedef struct {
    double height; /* conjugation height, m */
    double pitch;  /* actuator pitch, m */
    int n_act;     /* actuators per side (>= 2) */
} fewha_dm;

typedef struct {
    double D;           /* telescope diameter, m */
    double obstruction; /* central obstruction as a fraction of D, in [0, 1) */
    int n_wfs, n_layers, n_dms;
    int J;              /* wavelet decomposition levels (>= 1) */
    const fewha_wfs *wfs;
    const fewha_layer *layers;
    const fewha_dm *dms;
    double alpha_reg;   /* regularisation weight alpha of Eq. (fewha), > 0 */
    int precision;      /* fewha_precision */
} fewha_config;

/* Validate a configuration and size a plan (host only; touches no GPU).  The configuration is
 * copied.  Geometry rules (Sec. 2.1): WFS node x_j = -D/2 + j d; a ray from node (x, y) towards
 * guide star g meets layer l at (sigma x + theta_x h, sigma y + theta_y h) with sigma = 1 - h/H
 * (LGS) or 1 (NGS); every such point and every fitting actuator must lie inside its layer grid.
 * Limits: n_layers <= 64, n_wfs <= 64, n_dms <= 16, J <= 12, layer n <= 512, n_sub <= 4096.
 * Returns FEWHA_ERR_INVALID_ARG, FEWHA_ERR_GEOMETRY or FEWHA_ERR_UNSUPPORTED on rejection. */
int fewha_plan_create(const fewha_config *cfg, fewha_plan **out);

/* Bytes of device workspace the plan needs (tables, intermediates, b_prev, r_prev, PCG vectors). */
size_t fewha_workspace_bytes(const fewha_plan *p);

/* Attach a caller-allocated device workspace (>= fewha_workspace_bytes, 256-byte aligned, owned
 * by the caller and kept alive until fewha_plan_destroy) on the current HIP device, upload the
 * geometry tables, zero the warm-restart state and build the preconditioner of Sec. 3.4 by
 * probing the data term (one application of A per (layer, level, orientation) band).
 * Synchronous.  May be called again with another workspace (the state is reset). */
int fewha_plan_bind(fewha_plan *p, void *d_workspace, size_t bytes, void *stream);

/* Free the host side of the plan (the workspace stays the caller's). */
int fewha_plan_destroy(fewha_plan *p);

/* Vector lengths, the dimensions of Table 1 (Sec. 2.2): n_coef = sum over layers of n_l^2 wavelet
 * coefficients (= layer nodes; the paper's 2^(2 J_l) per layer), n_slopes = sum over sensors of
 * 2 n_sub^2 dense slopes (Gamma's rows), n_act = sum over DMs of n_act^2 actuators.  Any output
 * may be NULL.  Host only; FEWHA_ERR_INVALID_ARG for a null plan. */
int fewha_sizes(const fewha_plan *p, size_t *n_coef, size_t *n_slopes, size_t *n_act);

/* s = mask Gamma P W^T c: wavelet coefficients to slopes (Eq. (atmo) in the wavelet domain). */
int fewha_apply_A(const fewha_plan *p, const void *d_c, void *d_s, void *stream);

/* c = W P^T Gamma^T mask s: the exact adjoint A^T of the wavelet-domain tomography operator of
 * Eq. (atmo) (A = mask Gamma P W^T), the product that forms the right-hand side of Eq. (fewha)
 * (there weighted by C_eta^-1).  d_s: n_slopes (inactive entries are ignored), d_c: n_coef, not
 * aliasing d_s.  Uses the plan's workspace intermediates (node grids, layer grid). */
int fewha_apply_At(const fewha_plan *p, const void *d_s, void *d_c, void *stream);

/* y = M c = W P^T Gamma^T C_eta^-1 Gamma P W^T c + alpha D c (left-hand side of Eq. (fewha)). */
int fewha_apply_M(const fewha_plan *p, const void *d_c, void *d_y, void *stream);

/* c = W x: layer nodal values to wavelet coefficients (periodic Daubechies-3, J levels). */
int fewha_dwt_forward(const fewha_plan *p, const void *d_layers, void *d_c, void *stream);

/* c = W x as fewha_dwt_forward, for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, hosts that forbid hipMalloc): this call allocates nothing
 * and needs no bound workspace, only a created plan.  Its scratch (the level-kf approximation
 * of every layer, (n_coef / 4 + 4) values rounded up to a multiple of 4) sits in a device array of
 * the library, 8 MiB on every GPU the library runs on, held until the process ends; a plan needing
 * more returns FEWHA_ERR_UNSUPPORTED before touching the device.  The first call on a device looks
 * the array up there (and sets the kernels' LDS limits), so it must run with that device current.
 * All calls on one GPU share the array: two calls that overlap in time on one GPU (on different
 * streams, or from different threads) race on it and must be ordered by the caller.  Results are
 * bitwise those of fewha_dwt_forward.  d_layers, d_c: n_coef values each, not aliasing. */
int fewha_dwt_forward_noalloc(const fewha_plan *p, const void *d_layers, void *d_c, void *stream);

/* x = W^T c = W^-1 c: wavelet coefficients to layer nodal values (the reconstructed layers). */
int fewha_dwt_inverse(const fewha_plan *p, const void *d_c, void *d_layers, void *stream);

/* One reconstruction frame of Alg. 1 up to the PCG: b = W Ahat^T C_eta^-1 s; residual update
 * r = (b - b_prev) + r_prev; n_iter passes of Alg. 2 with the Jacobi preconditioner; then
 * b_prev = b, r_prev = r (kept in the workspace).  d_c holds c^(0) on entry (ignored for
 * FEWHA_COLD, which starts from c = b_prev = r_prev = 0) and c^(1) on return.  FEWHA_REFRESH
 * forms the same residual as b - M c^(0), the left-hand form of Alg. 1's residual line.  d_resnorm
 * (optional, n_iter doubles on the device) receives sqrt((r, J^-1 r)) at the start of every pass
 * that ran.  A zero residual ends the passes early (not an error); breakdown or non-finite
 * reductions stop the passes and set the device status word (fewha_last_status). */
int fewha_pcg_solve(fewha_plan *p, const void *d_s, void *d_c, int n_iter, int flags, double *d_resnorm,
                    void *stream);

/* Fitting and open-loop gain of Alg. 1: a = (1 - gain) a_prev + gain F W^T c, where F samples each
 * layer on-axis at the actuators of the DM nearest in altitude (ties to the lower DM) by bilinear
 * interpolation and sums the layers sharing a DM.  d_a_prev may be NULL (taken as 0).  d_a must
 * not alias d_c; it may alias d_a_prev. */
int fewha_fit_dm(const fewha_plan *p, const void *d_c, const void *d_a_prev, double gain, void *d_a,
                 void *stream);

/* One whole frame of Alg. 1 in one call: fewha_pcg_solve, then fewha_fit_dm of its c (arguments
 * and results as theirs, bit for bit).  d_a must not alias d_c or d_s. */
int fewha_reconstruct(fewha_plan *p, const void *d_s, void *d_c, int n_iter, int flags, double *d_resnorm,
                      const void *d_a_prev, double gain, void *d_a, void *stream);

/* Differentiation support (the adjoint state of Eq. (fewha)).  Solve M c = b for a right-hand
 * side b given in the wavelet domain (n_coef values), from c = 0, with n_iter passes of Alg. 2
 * and the Jacobi preconditioner of Sec. 3.4; d_resnorm as in fewha_pcg_solve.  The residual
 * starts at W (W^T b), equal to b up to rounding.  Uses the workspace's residual and PCG vectors,
 * so it overwrites the warm-restart state (b_prev = b, r_prev = the final residual): save it
 * with fewha_state_get first when a frame chain continues.  d_b must not alias d_c. */
int fewha_solve_M(fewha_plan *p, const void *d_b, void *d_c, int n_iter, double *d_resnorm, void *stream);

/* s = C_eta^-1 mask Gamma P W^T c: fewha_apply_A weighted by the inverse noise variance
 * sigma_g^-2 of each guide star (Eq. (MAP)), the map from coefficients to the weighted data
 * residual of the MAP functional. */
int fewha_apply_CA(const fewha_plan *p, const void *d_c, void *d_s, void *stream);

/* Per layer l: d_out[l] = sum over the layer's coefficients k of x_k (alpha D)_k y_k, in FP64 and
 * fixed order (d_out: n_layers doubles on the device).  alpha D is the prior of Eq. (fewha) per
 * (layer, level); since D_l is proportional to 1/gamma_l (the Cn^2 weight), dM/dgamma_l is
 * -(alpha D)_l / gamma_l on layer l and zero elsewhere. */
int fewha_prior_dot(const fewha_plan *p, const void *d_x, const void *d_y, double *d_out, void *stream);

/* The gradient of a loss L(c) of the MAP-FEWHA solution c = M^-1 b of Eq. (fewha) with respect to
 * the layers' Cn^2 weights gamma_l, by the implicit-function rule: with lambda = M^-1 dL/dc (e.g.
 * from fewha_solve_M), d_out[l] = dL/dgamma_l = lambda_l^T (alpha D)_l c_l / gamma_l, since the
 * prior of Eq. (fewha) scales as D_l ~ 1/gamma_l (so dM/dgamma_l = -(alpha D)_l / gamma_l on layer
 * l) and b does not depend on gamma.  d_lambda, d_c: n_coef values of the plan's precision;
 * d_out: n_layers doubles on the device, each summed in FP64 in a fixed order over its layer. */
int fewha_cn2_gradient(const fewha_plan *p, const void *d_lambda, const void *d_c, double *d_out, void *stream);

/* Closed loop (Alg. 1).  Pseudo-open-loop slopes s_pol = mask (s + Gamma P_DM a_m1): the DMs'
 * correction as the sensors see it added to the measured residual slopes, with a_m1 = a^(-1),
 * the DM shape two frames back (two-step delay).  Alg. 1 prints the update as s + Gamma a^(-1);
 * it is read with the projection P_DM of the DM surfaces onto the sensor grids: DM m is the
 * piecewise bilinear surface over its actuators (Sec. 4.1; actuator (i, j) at ((j - (n_a-1)/2)
 * pitch, (i - (n_a-1)/2) pitch), zero beyond the outermost actuators), met by each guide star's
 * rays at the DM's altitude as a layer is (cone factor, shift).  Inactive slopes are written 0.
 * d_s_pol may alias d_s. */
int fewha_pol_slopes(const fewha_plan *p, const void *d_s, const void *d_a_m1, void *d_s_pol, void *stream);

/* Closed-loop control of Alg. 1: a = a0 + gain (F W^T c - a_m1), with F the fitting of
 * fewha_fit_dm, a0 = a^(0) and a_m1 = a^(-1).  d_a must alias neither d_c nor d_a_m1; it may
 * alias d_a0. */
int fewha_fit_dm_closed(const fewha_plan *p, const void *d_c, const void *d_a0, const void *d_a_m1, double gain,
                        void *d_a, void *stream);

/* Least-squares DM fitting for more layers than DMs, then the open-loop gain:
 * a = (1 - gain) a_prev + gain a_ls.  Sec. 4.1 says that with more layers than DMs the fit becomes
 * a minimisation of its own, which it leaves unstated.  Reading: a_ls minimises, over the 25 probe
 * directions of the quality evaluation grid (theta_x, theta_y in {-60, -30, 0, 30, 60} arcsec)
 * and the nodes (-D/2 + j d, -D/2 + i d), d = D / n_sub of the first guide star, inside the closed
 * pupil annulus obstruction D/2 <= r <= D/2, along natural-star rays,
 *   sum_theta sum_x (sum_l U_l(x + theta h_l) - sum_m S_m(x + theta h_m))^2 + eps |a|^2,
 * U_l = the layers W^T c and S_m = the DMs, each the piecewise bilinear (hat) surface over its grid,
 * zero beyond it; a_ls is n_cg plain CG steps on the normal equations from 0 (a step whose
 * residual norm is 0 leaves a_ls unchanged).  d_c: n_coef coefficients; d_a_prev: n_act or NULL
 * (taken as 0); d_a: n_act, must not alias d_c, may alias d_a_prev.  Device pointers of the plan's
 * precision.  Uses workspace vectors of the plan (calls on one plan do not overlap).  Returns
 * FEWHA_ERR_INVALID_ARG for a null d_c or d_a, d_a == d_c, n_cg < 0, a non-finite gain, or eps
 * negative or non-finite. */
int fewha_fit_dm_ls(const fewha_plan *p, const void *d_c, const void *d_a_prev, double gain, int n_cg, double eps,
                    void *d_a, void *stream);

/* The warm-restart state of Alg. 1: the previous frame's right-hand side b^(0) and residual
 * r^(0), which the residual line combines with the new right-hand side as (b^(1) - b^(0)) + r^(0)
 * (n_coef each, coefficient layout).  state_get copies them out of the workspace, state_set
 * into it (e.g. to resume a chain, to run several chains on one plan, or to refresh r^(0) =
 * b^(0) - M c^(0)).  Enqueued on the stream like every other call. */
int fewha_state_get(const fewha_plan *p, void *d_b_prev, void *d_r_prev, void *stream);
int fewha_state_set(fewha_plan *p, const void *d_b_prev, const void *d_r_prev, void *stream);

/* Host copy of the preconditioner: h_jdiag[(l * (J + 1) + s) * 4 + o] = alpha D + tau for layer l,
 * level s in 1..J (1 finest) and orientation o (0 LL, only at s = J; 1 x-high; 2 y-high; 3 HH);
 * unused entries are 0.  h_jdiag holds n_layers * (J + 1) * 4 doubles.  Requires a bound plan. */
int fewha_precond_table(const fewha_plan *p, double *h_jdiag);

/* Batches of frames of one geometry.  Each stage of the path runs as one launch over every frame
 * of the batch (the frames are independent reconstructions: each has its own right-hand side,
 * warm-restart state and Alg. 2 scalars; only the geometry tables and the preconditioner are
 * shared).  fewha_plan_set_batch(p, max_batch) sizes the workspace for max_batch frames
 * (1 <= max_batch <= 1024); call it before fewha_workspace_bytes and fewha_plan_bind (it unbinds
 * a bound plan).  The single-frame calls act on frame 0.  In the _batch calls every vector
 * argument holds nbatch frames back to back, frame-major ([nbatch][n_coef], [nbatch][n_slopes],
 * [nbatch][n_act]; d_resnorm [nbatch][n_iter]), 1 <= nbatch <= max_batch, and frame f uses the
 * workspace state of frame f; otherwise each behaves as its single-frame counterpart. */
int fewha_plan_set_batch(fewha_plan *p, int max_batch);
int fewha_apply_A_batch(const fewha_plan *p, int nbatch, const void *d_c, void *d_s, void *stream);
int fewha_apply_At_batch(const fewha_plan *p, int nbatch, const void *d_s, void *d_c, void *stream);
int fewha_apply_M_batch(const fewha_plan *p, int nbatch, const void *d_c, void *d_y, void *stream);
int fewha_pcg_solve_batch(fewha_plan *p, int nbatch, const void *d_s, void *d_c, int n_iter, int flags,
                          double *d_resnorm, void *stream);
int fewha_fit_dm_batch(const fewha_plan *p, int nbatch, const void *d_c, const void *d_a_prev, double gain,
                       void *d_a, void *stream);
int fewha_reconstruct_batch(fewha_plan *p, int nbatch, const void *d_s, void *d_c, int n_iter, int flags,
                            double *d_resnorm, const void *d_a_prev, double gain, void *d_a, void *stream);
int fewha_pol_slopes_batch(const fewha_plan *p, int nbatch, const void *d_s, const void *d_a_m1, void *d_s_pol,
                           void *stream);
int fewha_fit_dm_closed_batch(const fewha_plan *p, int nbatch, const void *d_c, const void *d_a0, const void *d_a_m1,
                              double gain, void *d_a, void *stream);
/* Status words of frames 0..nbatch-1 after the last enqueued solve (synchronises the device). */
int fewha_last_status_batch(const fewha_plan *p, int nbatch, int *h_status);

/* Stages of one PCG pass, for timing a single launch (fewha_stage_launch). */
typedef enum {
    FEWHA_STAGE_WT = 0,   /* u = W^T J^-1 r: inverse DWT of the preconditioned residual (Alg. 2;
                             Kernel 1, Sec. 3.3) */
    FEWHA_STAGE_PROJ = 1, /* v = Gamma^T C_eta^-1 Gamma P u on every guide star, with the partial
                             sums of C (Gamma P u)^2 (Kernel 2, Sec. 3.3) */
    FEWHA_STAGE_PT = 2,   /* x = P^T v on every layer (Kernel 3, Sec. 3.3), with the Alg. 2 scalar
                             step in one extra workgroup */
    FEWHA_STAGE_FWD = 3   /* y = W x + alpha D z, all levels, with the PCG update of Alg. 2 and the
                             next pass's partial sums, applied to workspace scratch copies of r, p,
                             q, c (Kernel 3, Sec. 3.3) */
} fewha_stage;

/* Enqueue one launch of one stage of the PCG pass on the plan's current workspace contents
 * (the vectors the previous stage left there), for timing and profiling a single kernel.  The
 * stages read and write only workspace intermediates (u, v, x, partial sums, scratch vectors):
 * the caller's vectors, the warm-restart state and the published PCG scalar state are untouched,
 * so a later fewha_pcg_solve is unaffected.  Returns FEWHA_ERR_INVALID_ARG for an unknown stage. */
int fewha_stage_launch(const fewha_plan *p, int stage, void *stream);

/* fewha_stage_launch over frames 0..nbatch-1 of a batched plan (one launch, grid y = frame), for
 * timing the stage kernels in the batched regime of fewha_pcg_solve_batch.  Same contract per
 * frame; FEWHA_ERR_INVALID_ARG if nbatch is outside 1..max_batch or the stage is unknown. */
int fewha_stage_launch_batch(const fewha_plan *p, int nbatch, int stage, void *stream);

/* Launch shapes of a plan that change no result beyond the order of the PCG reductions' partial
 * sums (Sec. 3.4 asks for as few, and as well-shaped, kernel calls as the hardware allows; these
 * shapes are chosen per geometry, see fewha_autotune). */
typedef struct {
    int kf;         /* forward-DWT levels done on tiles over the whole GPU (1 or 2, at most J); the
                       levels beyond run per layer in one workgroup */
    int tq;         /* level-kf quads per edge of a fine forward-DWT tile: 1, 2, 4 or 8 (a tile
                       covers (tq 2^kf)^2 layer nodes) */
    int chunk_wt;   /* per tile kernel (W^T, projection, P^T, fine W): tiles per XCD chunk of the
                       workgroup order, 0..256; 0 = one contiguous run of tiles per XCD */
    int chunk_proj;
    int chunk_pt;
    int chunk_fwd;
    int fold;       /* 1: the coarse forward-DWT levels (kf+1..J) of the right-hand side and of
                       every PCG pass but the last run inside the next pass's inverse DWT (every
                       tile recomputes them from the level-kf approximation and updates its own
                       share), saving one launch per pass; FP32 plans with kf = 2, J > 2 and
                       layers up to 256 x 256 */
} fewha_tuning;

/* The plan's current launch shapes (defaults after fewha_plan_create: kf = min(2, J), tq the
 * largest of 8, 4, 2, 1 that fits the smallest layer, chunk_pt 16, other chunks 0, fold where it
 * applies). */
int fewha_get_tuning(const fewha_plan *p, fewha_tuning *h_tuning);

/* Set the launch shapes (host only; the plan stays bound, its workspace layout is unchanged).
 * FEWHA_ERR_INVALID_ARG for values outside the ranges above, FEWHA_ERR_UNSUPPORTED when the
 * split does not fit the coarse workgroup's LDS or the partial-sum buffer; the plan is then
 * unchanged.  Must not be called while work of the plan is in flight. */
int fewha_set_tuning(fewha_plan *p, const fewha_tuning *h_tuning);

/* Autotuner: times the PCG-pass stage kernels (fewha_stage_launch over nbatch frames, each
 * timing a HIP graph of back-to-back launches on a private stream) for every valid (kf, tq), then
 * the fold against none (on the inverse and forward DWT stages together), then every chunk in
 * {0, 4, 8, 16, 32} of each tile kernel, and keeps the fastest of each; the
 * result is set on the plan and returned in *h_best.  h_us (nullable, 4 values) receives the
 * tuned per-launch microseconds of the stages wt, proj, pt, fwd.  Synchronous; needs a bound
 * plan; resets the warm-restart state and the PCG scalars (as fewha_plan_bind leaves them), so it
 * belongs before the first frame.  nbatch in 1..max_batch. */
int fewha_autotune(fewha_plan *p, int nbatch, fewha_tuning *h_best, double *h_us);

/* The device status word of the last enqueued solve: FEWHA_ERR_BREAKDOWN when a pass of Alg. 2
 * met a non-positive denominator mu - rho beta / alpha_old (the step-size line; M is SPD, so only
 * rounding or corrupted input can cause it), FEWHA_ERR_NONFINITE when its reductions (rho, mu)
 * were NaN or Inf, else FEWHA_OK.  Synchronises the whole device first (hipDeviceSynchronize),
 * so the word is final whichever stream the solve was enqueued on.  FEWHA_ERR_WORKSPACE if
 * unbound, FEWHA_ERR_HIP if the synchronisation or the read fails. */
int fewha_last_status(const fewha_plan *p);

/* Static description of a status code. */
const char *fewha_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* FEWHA_H */
