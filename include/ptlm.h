/*
 * ptlm.h -- C ABI of the MI355X (gfx950) matrix-free Levenberg-Marquardt
 * ptychography library.
 *
 * The calls follow the problem statement of Kandel et al., "Efficient
 * ptychographic phase retrieval via a matrix-free Levenberg-Marquardt
 * algorithm" (arXiv 2103.01767): far-field model of Sec. 2
 * (eq:exit_wave, eq:expected_count), magnitude-based metrics of Sec. 4.1
 * (eq:magnitude, eq:ell_magnitude), the GGN matrix eq:ggn_magnitude used
 * matrix-free (App. A), the analytic diagonal of App. B, and the truncated LM
 * iteration alg:lm_inexact with the PCG stopping rule
 * eq:lma_termination_magnitude / eq:lma_termination_eta.
 *
 * Conventions shared by every call
 * --------------------------------
 * - Pointers named d_* or typed as device arrays are DEVICE pointers (HIP
 *   global memory) owned by the caller; pointers named h_* are host pointers.
 * - Arrays are row-major.  Complex arrays are interleaved (re, im) float pairs
 *   (complex64).  Object: ny x nx.  Probe: my x mx.  Per-measurement arrays:
 *   K x my x mx, position-major, detector pixels in FFT order (no shift).
 * - Positions are int32 pairs (row, col): the top-left object pixel of the
 *   probe window, 0 <= row <= ny-my, 0 <= col <= nx-mx.
 * - A real vector of R^(2n) is stored as the complex array whose real and
 *   imaginary parts are its two halves (Sec. 3 real coordinates).  Real
 *   diagonals of R^(2n) are float arrays of 2n entries interleaved the same
 *   way (one weight per real coordinate).  Gradients are real-coordinate
 *   gradients (twice the Wirtinger gradient of App. B).
 * - The 2D DFT F is unitary.
 * - Every call that takes a stream is asynchronous on that stream and never
 *   synchronises unless its comment says so.  No call allocates device memory:
 *   the caller passes one workspace sized by ptlm_workspace_bytes.
 * - Status codes are returned; no exception crosses the ABI.  On a non-OK
 *   status ptlm_last_error() returns a message (thread-local).
 * - A handle may be used from one host thread at a time.  Calls on one handle
 *   share its workspace and must be ordered on one stream.
 */
#ifndef PTLM_H
#define PTLM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PTLM_OK = 0,
  PTLM_ENOTACCEPTED = 1, /* LM: every retry of the outer iteration was rejected (not an error) */
  PTLM_EINVAL = -1,      /* invalid argument: sizes, positions, null pointers, unsupported shape */
  PTLM_EWORKSPACE = -2,  /* workspace missing or smaller than ptlm_workspace_bytes */
  PTLM_EHIP = -3,        /* a HIP runtime call failed */
  PTLM_ENUMERIC = -4     /* non-finite loss or gradient: iterate left at its last accepted value */
} ptlm_status;

typedef enum { PTLM_GAUSS = 0, PTLM_POISSON = 1 } ptlm_metric; /* eq:ell_magnitude */
typedef enum { PTLM_OBJECT = 0, PTLM_JOINT = 1 } ptlm_mode;    /* SPR eq:cdp / BPR eq:bp */
typedef enum { PTLM_GGN_MAGNITUDE = 0, PTLM_GGN_INTENSITY = 1 } ptlm_ggn;
/* How the GGN-vector product applies F and groups its tiles (a project choice,
 * ptlm_set_transform). */
typedef enum { PTLM_TRANSFORM_FFT = 0, PTLM_TRANSFORM_MFMA = 1, PTLM_TRANSFORM_FFT_WIDE = 2 } ptlm_transform;

/* Problem description.  Probe sides my, mx must each be 16, 32, 64 or 128, or both 48, 96 or 256. */
typedef struct {
  int32_t ny, nx;     /* object shape */
  int32_t my, mx;     /* probe shape */
  int32_t K;          /* number of scan positions (>= 1) */
  int32_t metric;     /* ptlm_metric */
  int32_t mode;       /* ptlm_mode: PTLM_JOINT optimises object and probe */
  float background;   /* b > 0 of eq:expected_count, per detector pixel */
  int32_t ggn;        /* GGN of the LM model: PTLM_GGN_MAGNITUDE (eq:ggn_magnitude, the paper's
                         choice) or PTLM_GGN_INTENSITY (eq:ggn_intensity, the ablation of App. C:
                         the same f and gradient, the Hessian of the metric taken in the
                         intensity h; its weight is floored at 1e-30 where it vanishes, y = 0) */
  int32_t seg_len;    /* launch shape (a project choice, no effect on the method): 0 cuts the
                         positions over the workgroups the GPU keeps resident; n > 0 also cuts
                         them into at most ceil(K / n) segments, about n positions each, so that
                         a problem that shares the GPU in a batch keeps fewer, longer segments
                         (less overlap-add and probe-partial traffic).  Results depend on it
                         only through FP32 summation order.  Must be >= 0. */
} ptlm_desc;

/* LM hyper-parameters (alg:lm_inexact; defaults of Sec. 5 via ptlm_lm_default_params). */
typedef struct {
  double mu0, mu_min, kappa, nu, rho_min;
  double beta;        /* eq:lma_termination_eta: 0.1 Gaussian, 0.9 Poisson */
  double diag_floor;  /* floor of D and of the Jacobi diagonal, relative to the block maximum */
  int32_t cg_max;     /* cap on PCG products per solve */
  int32_t retry_max;  /* cap on rejected attempts per outer iteration */
  int32_t scaling;    /* 0: D = I, 1: D = Dg(G) (App. B diagonal) */
  int32_t precond;    /* 0: none, 1: Jacobi Dg(G + lambda D), 2: learned diagonal + lambda D,
                         3: exact diagonal of G + lambda D (one more transform per linearisation),
                         4: stochastic estimate of diag(G) + lambda D (stoch_samples inverse
                         transforms per linearisation); 3 and 4 floored like D */
  int32_t warm_start; /* 1: PCG starts from the last accepted step */
  int32_t surrogate_T;  /* App. E surrogate metric: outer iterations with sigma_t > 0 (0: off) */
  double surrogate_s0;  /* sigma_0; sigma_t = s0 * 1e-6^(t / (T - 1)) for t < T, then 0 */
  int32_t project;      /* 1: alg:projected_LM plug-in after every accepted step, decided on the
                           device (projection, Armijo line search of at most ls_max sizes) */
  int32_t ls_max;       /* backtracking halvings of its line search before the iterate is kept */
  double o_max, p_max;  /* eq:constraints: |O| <= o_max (1), |P| <= p_max (1e8) */
  double sigma_ls;      /* eq:armijo_criterion constant (1e-4) */
  double gamma, tau_s, p_s; /* alg:projected_LM constants (1e-6, 1e-8, 2.1; Sec. 5) */
  int32_t alternate;    /* 1: alg:alt_LM_ptycho (joint problems only): every outer iteration
                           runs the attempts of alg:lm_inexact on the object with the probe fixed,
                           then on the probe with the new object fixed, each block with its own
                           damping mu and warm start; 0: joint update */
  int32_t stoch_samples;  /* precond 4: draws of the stochastic diagonal per linearisation */
  uint64_t stoch_seed;    /* precond 4: SplitMix64 seed; outer iteration t uses draws
                             t*stoch_samples .. (t+1)*stoch_samples - 1 (ptlm_diag_stochastic) */
} ptlm_lm_params;

/* LM state, FP64, in DEVICE memory (written by the library, read by the caller). */
typedef struct {
  double f;          /* f(z_t) at the current linearisation */
  double f_trial;    /* f(z_t + Delta) of the last attempt */
  double mu, lambda, rho, eta;
  double gnorm;      /* ||g|| = ||J^T grad ell|| */
  double resid_norm; /* ||grad_zeta ell|| */
  double pred;       /* predicted reduction of the last attempt */
  double rz, rr, alpha, beta_cg, pap; /* PCG scalars */
  double sigma;      /* surrogate term added to the background in the current outer iteration */
  double ls_alpha;   /* step size of the last projected plug-in (0: iterate kept) */
  double mu_alt;     /* alternating update: damping of the block not running (mu: running block) */
  int32_t t;         /* outer iterations completed (both sub-steps, alternating update) */
  int32_t cg_iters;  /* products with A in the last solve */
  int32_t cg_total;  /* products with A since ptlm_lm_init */
  int32_t accepted;  /* last attempt accepted */
  int32_t cg_active; /* internal: PCG loop still running */
  int32_t retries;   /* rejected attempts in the current outer iteration (sub-step) */
  int32_t nonfinite; /* a non-finite value was met */
  int32_t products;  /* GGN-vector products since ptlm_lm_init (PCG and warm starts) */
  int32_t attempts;  /* LM attempts (trial points) since ptlm_lm_init */
  int32_t need_lin;  /* internal: the next attempt starts by linearising */
  int32_t lin_now;   /* internal: the current attempt linearises */
  int32_t use_warm;  /* internal: the current solve starts from the last accepted step */
  int32_t alive;     /* internal: the current attempt runs (t < t_max, no numeric failure) */
  int32_t prev_valid;/* accepted steps exist for the PCG warm start: bit 0 object (all variables
                        for the joint update), bit 1 probe (alternating update) */
  int32_t t_max;     /* outer iterations to run: INT32_MAX after ptlm_lm_init, T in batches */
  int32_t status;    /* PTLM_OK, PTLM_ENOTACCEPTED (last outer iteration) or PTLM_ENUMERIC */
  int32_t iter_done; /* internal: the last attempt ended an outer iteration */
  int32_t ls_branch; /* last projected plug-in: 0 projected LM step, 1 line search along the
                        projected step, 2 projected gradient, -1 none */
  int32_t block;     /* alternating update: block of the current sub-step (0 object, 1 probe);
                        0 for the joint update */
  int32_t acc_o;     /* internal: the last attempt accepted a step of the object */
  int32_t acc_p;     /* internal: the last attempt accepted a step of the probe */
  int32_t tile_now;  /* internal: the current attempt evaluates the linearisation (0 when it
                        adopts the one computed at the accepted trial point) */
  int32_t ls_dir;    /* internal, projected plug-in: the projected step is to be tested as a
                        search direction */
  int32_t ls_neg;    /* internal, projected plug-in: the search runs along -grad f instead */
  int32_t ls_on;     /* internal, projected plug-in: the line search still runs */
  int32_t ls_take;   /* internal, projected plug-in: the trial buffer becomes the iterate */
  int32_t ls_keep;   /* internal, projected plug-in: no step size passed, z_t stays the iterate */
  int32_t ls_proj;   /* internal, projected plug-in: candidates are projected (gradient branch) */
  int32_t ls_iter;   /* internal, projected plug-in: step sizes tried */
} ptlm_lm_state;

typedef struct ptlm_handle ptlm_handle;

/* Fill p with the paper's values: mu0=1e-5, mu_min=1e-8, nu=1, rho_min=1e-4, kappa=4
 * (Sec. 5), beta=0.1 (Sec. 4.2), cg_max=10, retry_max=10, D=I, no preconditioner. */
void ptlm_lm_default_params(ptlm_lm_params* p);

/* Host only.  Bytes of device workspace needed for this problem.  h_pos: K (row, col)
 * pairs, host memory.  Returns PTLM_EINVAL for unsupported shapes or positions. */
ptlm_status ptlm_workspace_bytes(const ptlm_desc* desc, const int32_t* h_pos, size_t* bytes);

/* Create a handle.  Validates desc and every position (0 <= r <= n - m), copies the
 * positions and constant tables into the workspace on `stream` and returns without
 * waiting.  d_ws must stay valid until ptlm_destroy; the handle owns host metadata and,
 * for ptlm_lm_step's PCG and line-search look-ahead and for ptlm_autotune, 258 ints of
 * pinned host memory and 131 HIP events (made here, so that no later call allocates).  On
 * the first handle of a device it also takes that device's address of the static scratch
 * of ptlm_loss_noalloc. */
ptlm_status ptlm_create(const ptlm_desc* desc, const int32_t* h_pos, void* d_ws, size_t ws_bytes,
                        void* stream, ptlm_handle** out);
ptlm_status ptlm_destroy(ptlm_handle* h);

/* zeta = (|F(P * S_k O)|^2 + b)^(1/2) for every position (eq:exit_wave, eq:expected_count,
 * eq:magnitude).  d_O: ny*nx complex, d_P: my*mx complex, d_zeta: K*my*mx float. */
ptlm_status ptlm_forward(ptlm_handle* h, const float* d_O, const float* d_P, float* d_zeta, void* stream);

/* f = sum ell(zeta, y) (eq:error_metric_magnitude), accumulated in FP64 into d_f[0].
 * d_y: K*my*mx float counts >= 0.  d_resid (nullable): ell'(zeta), K*my*mx float. */
ptlm_status ptlm_loss(ptlm_handle* h, const float* d_O, const float* d_P, const float* d_y,
                      double* d_f, float* d_resid, void* stream);

/* For callers that cannot allocate (code under HIP graph capture, tight serving loops):
 * ptlm_loss with its only scratch -- the FP64 partial sums of the loss kernel, 4 doubles per
 * workgroup -- in a static device array of 8192 x 4 doubles (256 KiB, held by every device
 * the library runs on until the process ends) instead of the handle's workspace.  Same
 * arguments, results and rounding as ptlm_loss; allocates nothing and calls no allocating
 * routine.  The handle's device must be current.  PTLM_EINVAL for a 256 x 256 probe (its
 * transform tiles live in the workspace) or a handle with more than 8192 workgroups.  All
 * calls on one device share the array: calls that overlap in time on one device race (order
 * them on one stream). */
ptlm_status ptlm_loss_noalloc(ptlm_handle* h, const float* d_O, const float* d_P, const float* d_y,
                              double* d_f, float* d_resid, void* stream);

/* Linearise at (O, P): f (FP64, d_f[0]), ||grad_zeta ell||^2 (d_f[1]) and the gradient
 * g = J^T grad_zeta ell (App. A step 1) into d_gO (ny*nx complex) and, in PTLM_JOINT mode,
 * d_gP (my*mx complex; nullable in PTLM_OBJECT mode).  Stores the linearisation
 * (O, P and the per-pixel weighted phasor field) in the workspace for ptlm_jvp, ptlm_vjp,
 * ptlm_ggn_vp and ptlm_diag. */
ptlm_status ptlm_linearize(ptlm_handle* h, const float* d_O, const float* d_P, const float* d_y,
                           double* d_f, float* d_gO, float* d_gP, void* stream);

/* J v at the last linearisation: d zeta along v (App. A, JVP).  d_vP ignored (may be null)
 * in PTLM_OBJECT mode.  d_out: K*my*mx float. */
ptlm_status ptlm_jvp(ptlm_handle* h, const float* d_vO, const float* d_vP, float* d_out, void* stream);

/* J^T w at the last linearisation (eq:arbitrary_jtvp_sequence).  d_w: K*my*mx float.
 * d_outP nullable in PTLM_OBJECT mode. */
ptlm_status ptlm_vjp(ptlm_handle* h, const float* d_w, float* d_outO, float* d_outP, void* stream);

/* (G + lambda D) v at the last linearisation, G = J^T grad^2_zeta ell J (eq:ggn_magnitude,
 * App. A steps 2-4).  d_dO (2*ny*nx floats) / d_dP (2*my*mx) give D; null means D = I.
 * d_vP / d_outP ignored in PTLM_OBJECT mode. */
ptlm_status ptlm_ggn_vp(ptlm_handle* h, const float* d_vO, const float* d_vP, double lambda,
                        const float* d_dO, const float* d_dP, float* d_outO, float* d_outP,
                        void* stream);

/* Choose how the GGN-vector product (ptlm_ggn_vp and the products inside ptlm_lm_step /
 * ptlm_lm_solve) applies the 2D DFT F of eq:expected_count: PTLM_TRANSFORM_FFT, the tile
 * kernels' radix-16 FFT; PTLM_TRANSFORM_MFMA, F X F as two complex L x L matrix products on the
 * FP32 matrix cores (v_mfma_f32_16x16x4_f32 / v_mfma_f32_32x32x2_f32), for 16 x 16 and 32 x 32
 * probes only; PTLM_TRANSFORM_FFT_WIDE, the radix-16 FFT with workgroups of twice the tiles
 * (512 threads) over the same segments, for probe sides of 16 to 128 with at most 4096 pixels.
 * All give the product to FP32 rounding; MFMA differs from the FFT in the last bits, the wide
 * grouping gives the FFT's bits.  A handle starts with PTLM_TRANSFORM_MFMA for 16 x 16 probes,
 * PTLM_TRANSFORM_FFT_WIDE for 32 x 32 and PTLM_TRANSFORM_FFT otherwise; ptlm_autotune may
 * change it.  Batches run each shape's starting choice, but the standard grouping in place of
 * the wide one (same bits).  Takes effect from the next call; enqueues
 * nothing.  PTLM_EINVAL for an unknown value, a value the probe shape does not have, or the
 * handle of a batch's problem (ptlm_batch_problem). */
ptlm_status ptlm_set_transform(ptlm_handle* h, int32_t transform);

/* The two stages of ptlm_ggn_vp, for timing the per-position kernel on its own.
 * stage = 1: per-position kernel only (accumulates into workspace strips);
 * stage = 2: the finishing reductions only (writes d_outO / d_outP and clears the strips);
 * stage = 3: both (identical to ptlm_ggn_vp).  A stage-2 call finishes the most recent
 * stage-1 call on the handle; any other product in between replaces its partial sums. */
ptlm_status ptlm_ggn_vp_stage(ptlm_handle* h, const float* d_vO, const float* d_vP, double lambda,
                              const float* d_dO, const float* d_dP, float* d_outO, float* d_outP,
                              int32_t stage, void* stream);

/* Diagonal of G at the last linearisation, per real coordinate (2*ny*nx and 2*my*mx floats).
 * exact = 0: the paper's analytic approximation (App. B, eq:ggn_diag_mat converted by
 * eq:ggn_coord_trans; equal Re/Im weights).  exact = 1: the exact diagonal
 * sum_j ell''_j J_ji^2.  d_dP nullable in PTLM_OBJECT mode. */
ptlm_status ptlm_diag(ptlm_handle* h, float* d_dO, float* d_dP, int32_t exact, void* stream);

/* Stochastic estimate of the same diagonal from vector-Jacobian products alone (the matrix-free
 * route the paper names for problems without an analytic diagonal, end of Sec. 6): the mean
 * over `samples` draws of the squared real coordinates of J^T diag(sqrt(W)) r, W the GGN
 * weight of the linearisation and r a sign field over the K*M measurements; E[(J^T W^1/2 r)
 * (J^T W^1/2 r)^T] = G, so the estimate is unbiased.  Draw d gives measurement j (position k,
 * detector pixel m row-major, j = k*M + m) the sign of the top bit of output d*K*M + j + 1 of
 * SplitMix64 seeded with `seed`; the call uses draws draw0 .. draw0 + samples - 1.  Output
 * layout as ptlm_diag.  Overwrites the LM vector z of the workspace.  Costs `samples`
 * inverse transforms per position. */
ptlm_status ptlm_diag_stochastic(ptlm_handle* h, int32_t samples, uint64_t seed, uint64_t draw0, float* d_dO,
                                 float* d_dP, void* stream);

/* Autotuner of the tile-kernel launch (a project addition).  Times the GGN-vector product
 * (reps calls after one warm-up) with the positions cut into 0.5x, 1x and 2x as many
 * segments (workgroups) as the GPU keeps resident, for each transform the probe shape has
 * (PTLM_TRANSFORM_FFT always, PTLM_TRANSFORM_MFMA at 16 x 16 and 32 x 32,
 * PTLM_TRANSFORM_FFT_WIDE up to 4096 pixels), and keeps the fastest pair.  Results do not
 * depend on the choice beyond FP32 rounding.  Synchronises the stream.  h_ms (9 host doubles,
 * nullable) receives the time per call at [transform * 3 + scale index], -1 where the
 * transform does not apply; h_scale (nullable) the chosen scale,
 * h_transform (nullable) the chosen transform.  The workspace of ptlm_workspace_bytes covers
 * every candidate.  Overwrites the output buffers of the LM (call it before ptlm_lm_init or
 * between LM runs), not the linearisation.  PTLM_EINVAL for the handle of a batch's problem,
 * whose launch shape the batch fixes. */
ptlm_status ptlm_autotune(ptlm_handle* h, int32_t reps, double* h_ms, double* h_scale, int32_t* h_transform,
                          void* stream);

/* Truncated LM (alg:lm_inexact).  ptlm_lm_init resets d_state (mu = mu0, t = 0) on the
 * stream.  ptlm_lm_step runs one outer iteration in place on d_O (and d_P in PTLM_JOINT
 * mode): linearise, then up to retry_max attempts of {lambda, PCG solve, trial loss, gain
 * ratio, mu update}.  It synchronises the stream once per attempt to read the acceptance
 * flag.  Returns PTLM_OK when a step was accepted, PTLM_ENOTACCEPTED when all retries were
 * rejected (iterate unchanged), PTLM_ENUMERIC on a non-finite loss (iterate unchanged).
 * Without params->project the trial point of every attempt is evaluated as a full
 * linearisation into spare buffers; when the step is accepted the next outer iteration adopts
 * it instead of linearising again (same kernels on the same values: results are unchanged).
 * It is not adopted when O or P differ from the accepted point at the next call (the caller
 * changed them), when d_y is another pointer, after ptlm_linearize on the handle, or when the
 * surrogate term changes; the contents of d_y must not change between calls of one run.
 * With params->alternate (PTLM_JOINT only, else PTLM_EINVAL) the outer iteration is the
 * object sub-step and then the probe sub-step of alg:alt_LM_ptycho, each linearising at its
 * own start and running up to retry_max attempts on its block; PTLM_ENOTACCEPTED then means
 * that the attempts of at least one sub-step were all rejected (that block unchanged).
 * With params->precond == 2 the PCG preconditioner is d + lambda D, where d is the network's
 * learned diagonal (ptlm_lm_set_cnn, refreshed every outer iteration) or, if no network is
 * registered, the caller's d_precond (2n floats).
 * ptlm_lm_solve runs T outer iterations, stopping early on PTLM_ENUMERIC. */
ptlm_status ptlm_lm_init(ptlm_handle* h, const ptlm_lm_params* params, ptlm_lm_state* d_state,
                         void* stream);
ptlm_status ptlm_lm_step(ptlm_handle* h, float* d_O, float* d_P, const float* d_y,
                         const ptlm_lm_params* params, ptlm_lm_state* d_state,
                         const float* d_precond, void* stream);
ptlm_status ptlm_lm_solve(ptlm_handle* h, float* d_O, float* d_P, const float* d_y,
                          const ptlm_lm_params* params, int32_t T, ptlm_lm_state* d_state,
                          const float* d_precond, void* stream);

/* ---------------------------------------------------------------------------------------
 * Learned diagonal preconditioner (a project addition; the paper preconditions PCG with the
 * analytic diagonal Dg(G + lambda D) of App. B and mentions stochastic diagonal estimates).
 * A small CNN of `layers` 3x3 "same" convolutions (zero padding, ReLU between layers) maps
 * 3 feature maps on the object grid -- illumination overlap sum_k S_k^T |P|^2, overlap-
 * weighted |P|^2 and overlap-weighted arg P (ptlm_cnn_features) -- to 2 maps r; the learned
 * object diagonal is s * exp(r) per real coordinate (positive by construction), where the
 * scale s is the largest entry of the App. B object diagonal: the network predicts the shape
 * of Dg(G), trained on the exact diagonals of LM iterates (an untrained network, whose last
 * layer is zero, gives the constant s: the iterates of unpreconditioned CG).  The probe part
 * (joint mode) stays the App. B diagonal.  Tensors are NCHW float32 device arrays;
 * parameters are one float array: per layer W (Cout, Cin, 3, 3) then b (Cout).
 * ------------------------------------------------------------------------------------- */
typedef struct {
  int32_t n, h, w;            /* batch and spatial size */
  int32_t cin, cmid, cout;    /* channels: input, hidden, output (each 2, 3, 4, 8, 16 or 32) */
  int32_t layers;             /* number of conv layers, 1..15 */
} ptlm_cnn_desc;

ptlm_status ptlm_cnn_param_count(const ptlm_cnn_desc* d, size_t* count);           /* host only */
ptlm_status ptlm_cnn_workspace_bytes(const ptlm_cnn_desc* d, size_t* bytes);        /* host only */
/* d_out: n x cout x h x w (the log-diagonal r). */
ptlm_status ptlm_cnn_forward(const ptlm_cnn_desc* d, const float* d_params, const float* d_x, float* d_out,
                             void* d_ws, size_t ws_bytes, void* stream);
/* Loss L = sum_mask (r - t)^2 / (2 count) (mask > 0 selects pixels) into d_loss[0] (FP64)
 * and dL/dparams into d_grad (param_count floats). */
ptlm_status ptlm_cnn_loss_grad(const ptlm_cnn_desc* d, const float* d_params, const float* d_x, const float* d_t,
                               const float* d_mask, double* d_loss, float* d_grad, void* d_ws, size_t ws_bytes,
                               void* stream);
/* One Adam step (Kingma & Ba) on `count` parameters; step counts from 1. */
ptlm_status ptlm_cnn_adam(size_t count, float* d_params, const float* d_grad, float* d_m, float* d_v,
                          int32_t step, float lr, float beta1, float beta2, float eps, void* stream);
/* The 3 input maps (3 x ny x nx floats) at the last linearisation of the handle. */
ptlm_status ptlm_cnn_features(ptlm_handle* h, float* d_feat, void* stream);
/* Learned PCG diagonal (2n floats, interleaved like ptlm_diag) from r (2 x ny x nx) at the
 * last linearisation: object part s * exp(r) with r clamped to [log 1e-6, 2] and s the largest
 * App. B object entry; probe part the App. B diagonal floored at 1e-6 of its block maximum. */
ptlm_status ptlm_learned_precond(ptlm_handle* h, const float* d_r, float* d_precond, void* stream);
/* Register a network for ptlm_lm_step with params->precond == 2: after every linearisation
 * the step recomputes features -> network -> learned diagonal (as ptlm_learned_precond, with
 * params->diag_floor, 1e-6 by default, in place of 1e-6).
 * d = NULL unregisters.  The
 * desc must be n = 1, h x w = the object shape, cin = 3, cout = 2; d_params and d_ws
 * (ptlm_cnn_workspace_bytes) stay owned by the caller and must outlive their use. */
ptlm_status ptlm_lm_set_cnn(ptlm_handle* h, const ptlm_cnn_desc* d, const float* d_params, void* d_ws,
                            size_t ws_bytes);
/* How often ptlm_lm_step re-runs the registered network: every `every`-th linearisation
 * (default 1), or only at the first one after registration (every = 0).  Between runs the
 * learned diagonal is rebuilt from the kept network output and the new App. B scale.  A
 * batch (ptlm_batch_bind) runs each network from the bound probe, and again at each
 * ptlm_batch_cnn_refresh. */
ptlm_status ptlm_lm_set_cnn_refresh(ptlm_handle* h, int32_t every);

/* ---------------------------------------------------------------------------------------
 * Batched LM over independent problems of uneven sizes (a project addition: many
 * reconstructions share the GPU; the method per problem is alg:lm_inexact unchanged).
 * Each problem keeps its own plan, workspace region and LM state, and its handle
 * (ptlm_batch_problem) serves every single-problem call.  One attempt of the batch launches
 * each step of an LM attempt once for all problems (tile kernels once per probe shape
 * present); a problem's blocks and reduction order are those it has alone, so its iterates
 * in a batch equal those of ptlm_lm_step on it alone.
 * ------------------------------------------------------------------------------------- */
typedef struct ptlm_batch ptlm_batch;

/* Host only.  Bytes of device workspace for n problems (descs[i], positions h_pos[i]). */
ptlm_status ptlm_batch_workspace_bytes(int32_t n, const ptlm_desc* descs, const int32_t* const* h_pos,
                                       size_t* bytes);
/* Create the batch on d_ws (caller-owned, valid until ptlm_batch_destroy).  Uploads every
 * problem's tables on `stream`.  PTLM_EINVAL names the first invalid problem. */
ptlm_status ptlm_batch_create(int32_t n, const ptlm_desc* descs, const int32_t* const* h_pos, void* d_ws,
                              size_t ws_bytes, void* stream, ptlm_batch** out);
/* Handle of problem i (owned by the batch), NULL when out of range. */
ptlm_handle* ptlm_batch_problem(ptlm_batch* b, int32_t i);
/* Fix every problem's iterate d_O[i] / d_P[i] (updated in place), data d_y[i] and state
 * d_states[i] (n consecutive device states), the shared LM parameters and the number T of
 * outer iterations, and reset the states (mu = mu0, t = 0).  use_graph = 1: attempts after
 * the first are replayed from one captured HIP graph.  With params->precond == 2 every
 * problem needs a registered network (ptlm_lm_set_cnn on its handle); with params->alternate
 * every problem must be PTLM_JOINT.  With params->precond 3 or 4 each
 * problem's diagonal comes from its own launches of the single-problem kernels, in the same
 * attempt sequence (one tile launch, or one per draw, per problem).  Pointers must stay
 * valid until the next bind or ptlm_batch_destroy. */
ptlm_status ptlm_batch_bind(ptlm_batch* b, float* const* d_O, float* const* d_P, const float* const* d_y,
                            ptlm_lm_state* d_states, const ptlm_lm_params* params, int32_t T, int32_t use_graph,
                            void* stream);
/* Enqueue one LM attempt for every problem still running (no host synchronisation). */
ptlm_status ptlm_batch_attempt(ptlm_batch* b, void* stream);
/* Learned preconditioner of a batch (params->precond == 2): re-run every problem's registered
 * network on its features from its current probe (the bound d_P), on `stream`, between two
 * attempts.  The next linearisation of each problem builds its learned diagonal from the new
 * output; the linearisation state itself is not touched.  The network's inputs follow the
 * probe, which the joint LM updates, so a caller refreshes them every few outer iterations (a
 * refresh costs one network run per problem).  PTLM_EINVAL if the batch is not bound or a
 * problem has no network. */
ptlm_status ptlm_batch_cnn_refresh(ptlm_batch* b, void* stream);
/* Attempts until every problem has run T outer iterations (or met a non-finite value),
 * reading the states every check_every attempts, at most max_attempts.  Returns PTLM_OK,
 * PTLM_ENUMERIC (some problem failed; the others finished) or PTLM_ENOTACCEPTED (budget
 * spent).  *attempts_done (nullable) receives the attempts enqueued. */
ptlm_status ptlm_batch_solve(ptlm_batch* b, int32_t max_attempts, int32_t check_every, int32_t* attempts_done,
                             void* stream);
ptlm_status ptlm_batch_destroy(ptlm_batch* b);

/* Thread-local message describing the last non-OK status on this thread. */
const char* ptlm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PTLM_H */
