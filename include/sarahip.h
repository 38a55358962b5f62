/*
 * sarahip.h -- C ABI of the MI355X (gfx950) SARA/SDMM library.
 *
 * Carrillo, McEwen & Wiaux, "Why CLEAN when you can PURIFY?" (arXiv:1502.05037)
 * images the sky x >= 0 from visibilities y = Phi x + n by solving the
 * weighted-l1 problem (1), split into R data blocks as in (2) and solved in the
 * blocked form (3) by SDMM; SARA repeats (1)/(3) with re-computed weights.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Image x: n x n float32, row-major x[r*n + c]; pixel offsets r - n/2, c - n/2.
 *  - Visibilities: M complex64, interleaved (re, im) float32 pairs.  "User order"
 *    is the order of the uv array given to sh_op_create; data blocks are the
 *    contiguous ranges [block_offsets[i], block_offsets[i+1]) of that order.
 *  - (Phi x)_m = sum_{r,c} x[r,c] exp(-i (u_m (r - n/2) + v_m (c - n/2))),
 *    computed by an alpha-times oversampled NUFFT with a J x J Kaiser-Bessel
 *    interpolation kernel; Phi^dagger is the real adjoint Re(Phi^H v).
 *  - Coefficients: q planes of n x n float32 (plane 0 Dirac, then db1..db8 in
 *    bit order of the basis mask), each a 2D periodic DWT in Mallat layout.
 *  - Device pointers are HIP device memory owned by the caller (e.g. torch
 *    tensors); host pointers are ordinary host memory owned by the caller.  The
 *    library never frees or retains caller memory past a call.
 *  - `stream` is a hipStream_t (NULL = default stream).  Calls marked async only
 *    enqueue work; all others synchronise on `stream` before returning.
 *  - Errors: every call returns an sh_status.  Arguments are validated on the
 *    host before any launch; an invalid argument returns SH_EINVAL and enqueues
 *    nothing.  sh_last_error() gives a thread-local message for the last failure.
 *    No exception or abort crosses this boundary.
 */
#ifndef SARAHIP_H
#define SARAHIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SH_OK = 0,
  SH_EINVAL = -1,        /* invalid argument, nothing enqueued */
  SH_ENOMEM = -2,        /* device or host allocation failed */
  SH_EDEVICE = -3,       /* a HIP runtime call or kernel launch failed */
  SH_ENONFINITE = -4,    /* non-finite input or residual */
  SH_EUNSUPPORTED = -5   /* valid but not supported by this build */
} sh_status;

typedef struct sh_op_s* sh_op;    /* measurement operator: packed uv, tile plan, tables, scratch */
typedef struct sh_psi_s* sh_psi;  /* SARA dictionary: filter taps, level scratch */

/* Message for the last non-OK status on this thread (never NULL). */
const char* sh_last_error(void);
/* Device memory the library holds (live_bytes; a caller's workspaces are not counted) and the cap on it
 * (cap_bytes: the environment variable SH_MAX_DEVICE_BYTES, a positive byte count, read at every allocation;
 * -1 = none).  An allocation that would take the library past the cap fails with SH_ENOMEM.  Either
 * pointer may be NULL (not both). */
sh_status sh_device_bytes(int64_t* live_bytes, int64_t* cap_bytes);

/* Library version string. */
const char* sh_version(void);

/* ---------------------------------------------------------------------------
 * Measurement operator Phi (measurement equation y = Phi x + n; blocks (2)).
 * ------------------------------------------------------------------------- */

/* Plan Phi for M uv points (host, M x 2 row-major float64 (u, v) in radians
 * per pixel, each in [-pi, pi)), image side n (power of two, 16..4096),
 * oversampling alpha (2) and even kernel width J (2..16).  block_offsets (host,
 * R+1 int64, 0 = b_0 < b_1 < ... < b_R = M) gives the data blocks of (2).
 * The library converts uv to fixed-point grid coordinates in float64, sorts the
 * visibilities by uv tile inside each block and builds the gridding work list.
 * Synchronous.  Errors: SH_EINVAL (range, sizes, offsets), SH_ENOMEM. */
sh_status sh_op_create(const double* uv, int64_t M, int32_t n, int32_t oversample, int32_t kernel_width,
                       const int64_t* block_offsets, int32_t R, sh_op* out);
/* Same plan with explicit tiling (the autotuner's knobs): tile side T in {8, 16, 32} cells
 * (0 = automatic: 16, or alpha*n/4 when smaller) and the most visibilities per work item, 64..2^20 (0 = 4096).  The grid
 * side alpha*n must hold at least 3 tiles.  Results agree with sh_op_create to rounding. */
sh_status sh_op_create_tuned(const double* uv, int64_t M, int32_t n, int32_t oversample, int32_t kernel_width,
                             const int64_t* block_offsets, int32_t R, int32_t tile, int32_t chunk, sh_op* out);
/* sh_op_create_tuned with the plan's uploads on the caller's stream (hipStream_t, NULL = the null stream):
 * each upload is enqueued on it and waited for before the call returns, so the host arrays may go at once.
 * Synchronous with respect to that stream.  Errors as sh_op_create_tuned. */
sh_status sh_op_create_stream(const double* uv, int64_t M, int32_t n, int32_t oversample, int32_t kernel_width,
                              const int64_t* block_offsets, int32_t R, int32_t tile, int32_t chunk, void* stream,
                              sh_op* out);
sh_status sh_op_destroy(sh_op op);

/* One plan for P independent problems of the same image side, oversampling and kernel width
 * (many small fields imaged at once: the launches then cover all of them).  Problem p has M_p[p]
 * visibilities and R_p[p] blocks; uv (host, M x 2, M = sum M_p) and block_offsets (host, R+1,
 * R = sum R_p) concatenate the problems in order, so problem p's blocks are consecutive and cover
 * exactly its visibilities.  Every map of the plan then acts on all problems at once: images are
 * P x n x n (problem-major), visibilities M (problem-major), blocks R; problem p's visibilities
 * are measured from problem p's image only.  Errors as sh_op_create_tuned, plus SH_EINVAL when a
 * problem's blocks do not cover its visibilities exactly or P is outside [1, 4096]. */
sh_status sh_op_create_batched(const double* uv, const int64_t* M_p, int32_t P, int32_t n, int32_t oversample,
                               int32_t kernel_width, const int64_t* block_offsets, const int32_t* R_p,
                               int32_t tile, int32_t chunk, sh_op* out);

/* Autotuned plan (batched form; P = 1 for one problem).  The kernel width J is the smallest even
 * width whose aliasing estimate (sh_kb_alias_error) is <= accuracy, e.g. 1e-5; the gridding tile
 * side and item cap are then chosen by timing `reps` Phi + Phi^dagger pairs of candidate plans on
 * `stream` (tile sides 8, 16, 32, then item caps 1024 and 16384 for the fastest tile).  The choice
 * is cached for the process under a hash of the inputs; a repeated call only re-plans.  With the
 * environment variable SH_TUNE_CACHE naming a file, choices also persist across processes: a choice the
 * process has not made yet is looked up there first, and each new one is appended as a text line
 * "sarahip-tune-1 <key> <J> <tile> <chunk> <ms>" (the key starts with the library version; the last
 * valid line of a key wins; a file that cannot be read or written is ignored).  result (host) receives
 * the choice and its timing.  Synchronous; allocates and frees candidate plans.
 * Errors as sh_op_create_batched, plus SH_EINVAL for accuracy outside (0, 1) or unreachable. */
typedef struct {
  double accuracy;     /* the target given */
  double alias_error;  /* estimate for the chosen J */
  double ms_pair;      /* best measured Phi + Phi^dagger time (ms) */
  int32_t J;           /* chosen kernel width */
  int32_t tile;        /* chosen tile side */
  int32_t chunk;       /* chosen most visibilities per work item */
  int32_t candidates;  /* plans timed by this call (0 when cached) */
  int32_t cached;      /* 0 timed now, 1 from the process cache, 2 from the SH_TUNE_CACHE file */
} sh_tune_result;
sh_status sh_op_autotune(const double* uv, const int64_t* M_p, int32_t P, int32_t n, int32_t oversample,
                         double accuracy, const int64_t* block_offsets, const int32_t* R_p, int32_t reps,
                         sh_tune_result* result, sh_op* out, void* stream);
/* Forgets the process cache of sh_op_autotune (the SH_TUNE_CACHE file is left as it is). */
sh_status sh_tune_cache_clear(void);
/* Aliasing estimate of the J-wide Kaiser-Bessel interpolation on an alpha-times oversampled grid:
 * the RMS over image frequencies of sqrt(sum_{l != 0} psi_hat(xi + l)^2) / psi_hat(xi), times
 * sqrt(2) for two axes -- the expected relative error of Phi against the exact sum for a white
 * image.  Host only. */
sh_status sh_kb_alias_error(int32_t kernel_width, int32_t oversample, double* err_out);

/* Query plan sizes: out[0]=M, out[1]=n, out[2]=grid side K, out[3]=J, out[4]=R,
 * out[5]=number of gridding work items, out[6]=tile side, out[7]=max items per tile,
 * out[8]=number of problems P, out[9]=work items degridded one thread per visibility (all of them). */
sh_status sh_op_query(sh_op op, int64_t out[10]);

/* Block offsets in internal order (host, R+1 int64).  Internal order permutes
 * visibilities only inside each block, so these equal the user offsets. */
sh_status sh_op_block_offsets(sh_op op, int64_t* offsets_out);

/* Permutation: perm_out[i] = user index of internal visibility i (host, M int64). */
sh_status sh_op_permutation(sh_op op, int64_t* perm_out);

/* vis = Phi x in user order.  x: device P*n*n float32 (P = 1 unless batched); vis: device M
 * complex64.  Async. */
sh_status sh_phi_fwd(sh_op op, const float* x, float* vis, void* stream);
/* x = Re(Phi^H vis) from user-order visibilities.  Async. */
sh_status sh_phi_adj(sh_op op, const float* vis, float* x, void* stream);
/* The same two maps on internal-order visibilities (the order sdmm uses).  Async. */
sh_status sh_phi_fwd_internal(sh_op op, const float* x, float* vis, void* stream);
sh_status sh_phi_adj_internal(sh_op op, const float* vis, float* x, void* stream);
/* Reorder visibilities between user and internal order (device M complex64 each, distinct).  Async. */
sh_status sh_vis_to_internal(sh_op op, const float* user, float* internal, void* stream);
sh_status sh_vis_to_user(sh_op op, const float* internal, float* user, void* stream);

/* ||Phi||_2 of the real-linear map R^N -> C^M by power iteration on Re(Phi^H Phi)
 * from the caller's start image x0 (device P*n*n float32, e.g. a seeded Gaussian),
 * at most `iters` steps or until every problem's eigenvalue estimate changes by <= tol
 * relative.  Norms and Rayleigh quotients are reduced in float64.  nu_out: host, P values
 * (one per problem of a batched plan).  Synchronous. */
sh_status sh_op_norm(sh_op op, const float* x0, int32_t iters, double tol, double* nu_out, void* stream);

/* ---------------------------------------------------------------------------
 * SARA dictionary Psi = (1/sqrt q)[Psi_1 .. Psi_q] (SARA paragraph).
 * ------------------------------------------------------------------------- */

/* basis_mask: bit 0 = Dirac, bit b = Daubechies db_b (b = 1..8); SARA = 0x1FF.
 * n must be divisible by 2^levels (levels 1..8).  Filters are computed on the
 * host in float64 by spectral factorisation.  Synchronous. */
sh_status sh_psi_create(int32_t n, int32_t levels, uint32_t basis_mask, sh_psi* out);
/* The same dictionary applied to `batch` images per call (1..4096): x is batch x n x n and the
 * coefficients batch x q x n x n, image-major.  Pairs with a batched plan of P = batch problems. */
sh_status sh_psi_create_batched(int32_t n, int32_t levels, uint32_t basis_mask, int32_t batch, sh_psi* out);
sh_status sh_psi_destroy(sh_psi psi);
/* The same dictionary on caller-provided device memory (e.g. a torch tensor): its scratch (two LL
 * ping-pong buffers of batch x wavelet planes x (n/2)^2 float32) is carved from `workspace` (device,
 * 256-byte aligned, at least sh_psi_workspace_bytes bytes, owned by the caller, and to outlive the
 * handle).  The library then allocates no device memory for the handle.  Errors: SH_EINVAL (size,
 * alignment, arguments as sh_psi_create_batched). */
sh_status sh_psi_workspace_bytes(int32_t n, int32_t levels, uint32_t basis_mask, int32_t batch, size_t* bytes);
sh_status sh_psi_create_ws(int32_t n, int32_t levels, uint32_t basis_mask, int32_t batch, void* workspace,
                           size_t bytes, sh_psi* out);
/* Number of planes q (D = q*n*n coefficients). */
sh_status sh_psi_planes(sh_psi psi, int32_t* q_out);
/* The float64 scaling filter of db_p (2p taps) as used by the library (host). */
sh_status sh_daubechies(int32_t p, double* h_out);
/* x = Psi coeffs (synthesis).  coeffs: device q*n*n float32; x: device n*n.  Async. */
sh_status sh_psi_fwd(sh_psi psi, const float* coeffs, float* x, void* stream);
/* coeffs = Psi^dagger x (analysis).  Async. */
sh_status sh_psi_adj(sh_psi psi, const float* x, float* coeffs, void* stream);

/* ---------------------------------------------------------------------------
 * Proximal steps of SDMM on (3), each fused with its dual update.  All async.
 * ------------------------------------------------------------------------- */

/* Weighted soft threshold + dual: t = s + z; y = sign(t) max(|t| - gamma w, 0);
 * z <- t - y; v_out = y - z (the next x-update's input).  W may be NULL (w = 1).
 * Length D float32 each (device). */
sh_status sh_prox_l1(int64_t D, const float* s, float* z, const float* W, float gamma, float* v_out,
                     void* stream);
/* Positive orthant + dual: t = s + z; y = max(t, 0); z <- t - y; v_out = y - z.  Length N. */
sh_status sh_prox_pos(int64_t N, const float* s, float* z, float* v_out, void* stream);
/* Per-block l2-ball projection + dual on internal-order visibilities:
 * t = s + z; rho_i = ||t_i - yhat_i||_2 (float64); y_i = yhat_i + (t_i - yhat_i) min(1, eps_i/rho_i);
 * z <- t - y; v_out = y - z.  Also writes resid_out[i] = ||s_i - yhat_i||_2 (device float64, R).
 * s, z, yhat, v_out: device M complex64; eps: device float64 R. */
sh_status sh_prox_ball(sh_op op, const float* s, float* z, const float* yhat, const double* eps, float* v_out,
                       double* resid_out, void* stream);

/* The same projection for callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc): it calls no allocating routine and does not
 * synchronise (async, so it can be captured).  The per-block norms live in a fixed device array of
 * SH_BALL_NOALLOC_MAX_BLOCKS float64 values, one per GPU for the life of the process, shared by every
 * call on that GPU: calls that overlap on one GPU (several streams or threads) race and must be
 * serialised by the caller, as must calls on the same plan.  Arguments and results as sh_prox_ball.
 * Errors: SH_EINVAL (NULL argument, or a plan with more than SH_BALL_NOALLOC_MAX_BLOCKS blocks). */
#define SH_BALL_NOALLOC_MAX_BLOCKS 65536
sh_status sh_prox_ball_noalloc(sh_op op, const float* s, float* z, const float* yhat, const double* eps, float* v_out,
                               double* resid_out, void* stream);

/* SARA weights w = delta / (delta + |c|) (device D float32 in and out). */
sh_status sh_reweight(int64_t D, const float* c, double delta, float* W_out, void* stream);
/* Population standard deviation of c (float64 reduction).  Synchronous. */
sh_status sh_std(int64_t D, const float* c, double* std_out, void* stream);

/* ---------------------------------------------------------------------------
 * Real normal operator of the measurement model (measurement-equation
 * paragraph), the matrix of the x-update (Q in the SDMM paragraph):
 *   (T x)_p = scale_q Re(Phi^H Phi x)_p = scale_q sum_r k(p - r) x_r,
 *   k(d) = Re sum_m exp(i u_m . d)   (sum over problem q's visibilities),
 * a 2D convolution, applied as a circulant on the plan's K x K grid (K >= 2n):
 * zero-pad, FFT, product with the kernel's spectrum, inverse FFT, crop.  The
 * kernel comes from four adjoint NUFFTs of modulated unit visibilities, so T
 * matches the NUFFT pair Phi^dagger Phi to the interpolation's accuracy.
 * ------------------------------------------------------------------------- */
/* Density estimate of 1 / ||Phi_b|| for every block b of the plan (host R float64): with count_b the
 * largest number of block b's visibilities in an alpha x alpha window of grid cells (side 2 pi / n in the
 * uv plane, every cell offset, periodic), ||Phi_b||^2 ~ n^2 count_b and b_out[b] = 1 / (n sqrt(count_b)).
 * Cells are the plan's float64 cells floor(u K / 2 pi) mod K.  Synchronous.  Errors: SH_EINVAL, SH_ENOMEM. */
sh_status sh_block_weights(sh_op op, double* b_out, void* stream);

typedef struct sh_toep_s* sh_toep;
/* Build T for every problem of `op` (which must outlive it).  scale: host P float64 > 0, or NULL
 * (all 1).  Holds P*K*K float32 (spectrum) and P*n*K complex64 (scratch) of device memory; needs
 * M complex64 + P*n*n + 4*P*K*K float32 more while building.  Synchronous.
 * Errors: SH_EINVAL (NULL, scale <= 0 or non-finite, K < 2n), SH_ENOMEM, SH_EDEVICE. */
sh_status sh_toeplitz_create(sh_op op, const double* scale, sh_toep* out, void* stream);
/* The same operator on caller-provided device memory: its spectrum and scratch, and the build's
 * temporaries, are carved from `workspace` (device, 256-byte aligned, at least
 * sh_toeplitz_workspace_bytes, owned by the caller and to outlive the handle); the library allocates
 * no device memory for it.  Errors as sh_toeplitz_create, plus SH_EINVAL for a small or unaligned
 * workspace. */
sh_status sh_toeplitz_workspace_bytes(sh_op op, size_t* bytes);
sh_status sh_toeplitz_create_ws(sh_op op, const double* scale, void* workspace, size_t bytes, sh_toep* out,
                                void* stream);
/* out = T x for P images x (device P*n*n float32 each; out may not alias x).  Uses the plan's FFT
 * scratch, like sh_phi_fwd/adj: calls on one plan must not overlap.  Async. */
sh_status sh_toeplitz_apply(sh_toep t, const float* x, float* out, void* stream);
sh_status sh_toeplitz_destroy(sh_toep t);

/* ---------------------------------------------------------------------------
 * SDMM solve of (3) with SARA reweighting (PURIFY paragraph; SARA paragraph).
 * ------------------------------------------------------------------------- */

typedef struct {
  double gamma;        /* l1 prox step; <= 0: 1e-4 max|Psi^dagger Phi_hat^dagger y_hat| per problem */
  double nu;           /* norm used to normalise (see block_norm); <= 0: power iteration from ones
                          (at most 200 steps, to a relative change of 1e-6) */
  double tol_rel;      /* stop when ||x_n - x_{n-1}||/||x_n|| <= tol_rel and all blocks feasible;
                          0 = run max_iter every pass (fixed schedule) */
  double eps_slack;    /* feasibility test ||y_i - Phi_i x|| <= eps_i (1 + eps_slack) */
  double rw_beta;      /* delta_{t+1} = rw_beta * delta_t.  Between passes W = delta / (delta + |Psi^dagger x|),
                          and W = 1 where both are 0 (a pass that ended at x = 0 gives delta = 0) */
  double rw_delta0;    /* > 0: delta of the weights W passed in (warm start); else delta_1 = std */
  int32_t max_iter;    /* SDMM iterations per pass */
  int32_t cg_iters;    /* conjugate-gradient steps per x-update */
  int32_t passes;      /* weighted-l1 solves, the first with W (or identity) */
  int32_t check_every; /* host reads the stopping flags every this many iterations (>= 1) */
  int32_t graph;       /* 1: capture one iteration as a HIP graph and replay it; 0: plain launches.
                          Same arithmetic either way; kernel timing (sh_profile_enable) forces 0 */
  int32_t w_from_x0;   /* 1 (needs x0, W NULL): first-pass weights from the warm start by the
                          reweighting rule, delta_1 = std(Psi^dagger x0) per problem and
                          W = delta_1 / (delta_1 + |Psi^dagger x0|), as if x0 ended a pass */
  int32_t toeplitz;    /* 1: the CG steps apply Re(Phi_hat^H Phi_hat) through its Toeplitz embedding
                          (sh_toeplitz_create, built once per solve); 0: a Phi, Phi^dagger pair.
                          The right-hand side, the residuals and the stopping test always use Phi */
  int32_t block_norm;  /* normalisation of the data splits: Phi_hat_b = c_b Phi_b, y_hat_b = c_b y_b,
                          eps_hat_b = c_b eps_b with c_b = a_b / nu_p (b a block of problem p), where
                          a_b = 1 (0) or the density estimate of 1 / ||Phi_b|| (1, sh_block_weights),
                          and nu_p = nu if given, else the norm of problem p's a-weighted operator
                          sum_b a_b^2 Re(Phi_b^H Phi_b).  Any c_b > 0 keeps the solution set */
  double tol_dual;     /* > 0 (with tol_rel > 0): the stopping test also needs the relative dual residual
                          ||sum_j L_j^T z_j|| / max_j ||L_j^T z_j|| (sh_sdmm_info.kkt_dual) <= tol_dual,
                          evaluated at the checks where the relative change and feasibility already
                          hold; 0 = not tested */
  int32_t z_from_x0;   /* 1 (needs x0): the duals of the warm start also come from x0, from the optimality
                          conditions of the weighted problem at x0: y_psi = soft(c, gamma W) and
                          z_psi = c - y_psi for c = Psi^dagger x0, z_+ = 0, and per data block z_i = lambda (y_i - y_hat_i) with y_i the projection
                          of Phi_hat_i x0 onto the block's ball and one lambda >= 0 per problem minimising
                          ||Psi z_psi + Phi_hat^dagger z_phi||; 0: zero duals */
  double block_fraction; /* < 1: block-subset iterations (SDMM paragraph: iterations that use only a subset
                          of the data blocks y_i): in iteration k (counted from the session's start) block b
                          takes part when u(k R + b) < block_fraction, u(c) the c-th output of the SplitMix64
                          sequence seeded with block_seed taken to [0, 1) by its top 53 bits; only those
                          blocks are degridded, projected and gridded (their change to Phi_hat^T (y - z)),
                          the others keep their split variables.  The x-update still uses every block
                          (its right-hand side holds Phi_hat^T (y - z) as a running image, its matrix the
                          Toeplitz product).  The stopping test evaluates every block's residual at x_n.
                          Needs toeplitz = 1 and z_from_x0 = 0.  1 = every block every iteration */
  uint64_t block_seed;
  int32_t synthesis;   /* 1: the synthesis prior (SDMM paragraph: the solver handles various sparsity priors):
                          min ||W alpha||_1 over coefficients alpha (D = q n^2) subject to the same blocked
                          constraints on x = Psi alpha and x >= 0; the image returned is Psi alpha and the
                          weights follow alpha.  SDMM splits L = {I, Phi_hat Psi, Psi}, CG on alpha with
                          Q = I + Psi^dagger (I + Re(Phi_hat^H Phi_hat)) Psi through the Toeplitz product.
                          A warm start x0 starts from alpha = Psi^dagger x0.  Needs toeplitz = 1,
                          z_from_x0 = 0 and block_fraction = 1.  0: the analysis prior ||W Psi^dagger x||_1 */
} sh_sdmm_params;

/* Defaults: gamma -1, nu -1, tol_rel 0, eps_slack 1e-4, rw_beta 0.5, rw_delta0 0,
 * max_iter 300, cg_iters 2, passes 1, check_every 10, graph 1, w_from_x0 0, toeplitz 1, block_norm 1,
 * tol_dual 1e-2, z_from_x0 0, block_fraction 1, block_seed 0, synthesis 0.  With a batched plan, a given
 * gamma or nu applies to every problem; otherwise each problem gets its own. */
void sh_sdmm_default_params(sh_sdmm_params* p);

#define SH_PASS_RECORD 16   /* passes whose iteration counts sh_sdmm_info records */

typedef struct {
  int32_t iters_total;   /* SDMM iterations over all passes */
  int32_t passes_done;
  int32_t converged;     /* last pass met the stopping test (not an error when 0) */
  int32_t iters_last;    /* iterations of the last pass */
  double rel_change;     /* ||x_n - x_{n-1}|| / ||x_n|| at exit */
  double objective;      /* ||W Psi^dagger x||_1 (synthesis: ||W alpha||_1) with the last pass's weights */
  double gamma;          /* step actually used */
  double nu;             /* normalisation actually used (nu_p of block_norm) */
  double delta;          /* reweighting delta of W_out */
  double seconds;        /* wall time inside the call */
  double kkt_primal;     /* ||(s_j - y_j)_j|| / ||(s_j)_j|| of the state at exit: split images s_j = L_j x
                            (L = Psi^dagger, the normalised blocks Phi_hat_i, I) against their proximal points */
  double kkt_dual;       /* ||sum_j L_j^T z_j|| / max_j ||L_j^T z_j|| of the state at exit (stationarity) */
  int32_t pass_iters[SH_PASS_RECORD];   /* iterations of each pass (the first SH_PASS_RECORD passes), up to
                            the stopping iteration of this problem; 0 for passes not run */
} sh_sdmm_info;

/* Solve SARA/(3).  y: device M complex64, user order.  eps: host R float64 (user
 * units).  W: device D float32 weights of the first pass or NULL (identity).
 * x0: device n*n float32 warm start or NULL (zero start).  x_out: device n*n.
 * W_out: device D float32 (the weights after the last reweighting, i.e. those a
 * further pass would use) or NULL.  block_resid: host R float64 receiving
 * ||y_i - Phi_i x|| at exit, or NULL.  info: host, one entry per problem, or NULL.
 * Batched plans (P problems, psi with batch P) solve all problems together: images, weights and
 * coefficients are P times larger (problem-major) and every problem keeps its own nu, gamma,
 * CG scalars, reweighting delta and stopping test; the pass ends when every problem meets the
 * test.  In the last pass each problem's image, residuals, relative change, objective and W_out
 * are those of the iteration at which it first met the test (info[p].iters_last), as if it had
 * been solved alone.  Synchronous.
 * Errors: SH_EINVAL, SH_ENONFINITE (non-finite y/eps or residual), SH_ENOMEM, SH_EDEVICE. */
sh_status sh_sdmm_solve(sh_op op, sh_psi psi, const float* y, const double* eps, const float* W,
                        const float* x0, const sh_sdmm_params* params, float* x_out, float* W_out,
                        double* block_resid, sh_sdmm_info* info, void* stream);

/* Device memory of a solve or session with plan op, dictionary psi and these parameters: the solver state
 * (for M visibilities, N pixels and D coefficients about 40 M + 36 N + 16 D bytes, more with the Toeplitz
 * spectrum, the synthesis prior or block-subset iterations) plus the largest of the set-up's temporaries
 * (block-weight counters, the Toeplitz build, the power iteration).  Host only. */
sh_status sh_workspace_bytes(sh_op op, sh_psi psi, const sh_sdmm_params* params, size_t* bytes);
/* sh_sdmm_solve with every device allocation of the solve carved from `workspace` (device, 256-byte aligned,
 * at least sh_workspace_bytes bytes, owned by the caller): all device memory can then come from the caller
 * (e.g. torch).  Results are those of sh_sdmm_solve, bit for bit.  Errors as sh_sdmm_solve, plus SH_EINVAL
 * for a small or unaligned workspace. */
sh_status sh_sdmm_solve_ws(sh_op op, sh_psi psi, const float* y, const double* eps, const float* W,
                           const float* x0, const sh_sdmm_params* params, float* x_out, float* W_out,
                           double* block_resid, sh_sdmm_info* info, void* workspace, size_t bytes, void* stream);

/* Session form of the same solver, for callers that drive the iterations themselves
 * (benchmarks, checkpointed runs).  sh_sdmm_create validates as sh_sdmm_solve, copies the data
 * to device (internal order, normalised by nu), resolves nu and gamma, sets the zero or warm
 * state and synchronises.  It keeps pointers to op and psi (which must outlive the session) but
 * not to y, eps, W or x0. */
typedef struct sh_sdmm_s* sh_sdmm;
sh_status sh_sdmm_create(sh_op op, sh_psi psi, const float* y, const double* eps, const float* W,
                         const float* x0, const sh_sdmm_params* params, sh_sdmm* out, void* stream);
/* The session on a caller's workspace (as sh_sdmm_solve_ws); the workspace must outlive the session. */
sh_status sh_sdmm_create_ws(sh_op op, sh_psi psi, const float* y, const double* eps, const float* W,
                            const float* x0, const sh_sdmm_params* params, void* workspace, size_t bytes,
                            sh_sdmm* out, void* stream);
/* Enqueue exactly `iters` SDMM iterations of the current weighted-l1 pass (no stopping test, no
 * reweighting, no host synchronisation).  Splitting a run into several calls gives the same
 * iterates as one call.  Async. */
sh_status sh_sdmm_iterate(sh_sdmm s, int32_t iters, void* stream);
/* Current image (device P*n*n, may be NULL), block residuals ||y_i - Phi_i x|| (host R, may be
 * NULL) and relative change of the last iteration (host, P values, may be NULL).  Synchronous. */
sh_status sh_sdmm_result(sh_sdmm s, float* x_out, double* block_resid, double* rel_change, void* stream);
/* KKT residuals (as in sh_sdmm_info) and objective ||W Psi^dagger x||_1 (current weights) of the session's
 * current state, one value per problem each (host arrays of P, each may be NULL).  Needs at least one
 * iteration.  Synchronous.  These measure convergence of (3): at a solution every split image equals its
 * proximal point and the duals balance (SDMM paragraph). */
sh_status sh_sdmm_kkt(sh_sdmm s, double* kkt_primal, double* kkt_dual, double* objective, void* stream);
/* Checkpoint and resume of a session (the SDMM paragraph's iteration carried over a restart): the state one
 * iteration hands to the next — x, the split and dual vectors of the l1, data and positivity terms, the data
 * images and block residuals, the weights, the coefficients alpha (synthesis prior) and the running image and
 * iteration counter (block-subset iterations) — after a header with the session's sizes and options.
 * sh_sdmm_state_bytes gives the size; export copies the state into host memory the caller owns (at least that
 * many bytes) after the work already enqueued on `stream`; import overwrites a session's state with one
 * exported from a session created with the same op, psi, data and parameters, after which sh_sdmm_iterate
 * continues exactly as the exporting session would have (bitwise).  Both synchronise `stream`.
 * Errors: SH_EINVAL (NULL, buffer too small, or for import: size, header, sizes or options that differ). */
sh_status sh_sdmm_state_bytes(sh_sdmm s, size_t* bytes);
sh_status sh_sdmm_state_export(sh_sdmm s, void* host, size_t bytes, void* stream);
sh_status sh_sdmm_state_import(sh_sdmm s, const void* host, size_t bytes, void* stream);
/* Per-iteration metrics of a session (the quantities the stopping test of the SDMM paragraph and the
 * constraints of eq. (3) are judged by), kept on the device and read back when the caller chooses.
 * sh_sdmm_metrics_enable gives the session a ring of `rows` rows (0 switches it off and frees it; at most
 * 2^20), allocated with hipMalloc, and returns the row width 2P + R in *row_width (may be NULL).  From then on
 * every iteration, replayed graph or not, appends one row of doubles: [0, P) the relative change
 * ||x_n - x_(n-1)|| / ||x_n|| of each problem, [P, 2P) its objective ||W Psi^dagger x_n||_1 (||W alpha_n||_1
 * for the synthesis prior) with the pass's weights, [2P, 2P + R) each block's ||y_i - Phi_i x_n|| / eps_i
 * (block-subset iterations refresh their selected blocks only; the others repeat their last value, at first
 * their residual at the starting image).
 * Recording adds one weighted-l1 reduction and one small kernel per iteration.  enable synchronises the
 * device.  sh_sdmm_metrics_read copies the rows not yet read, oldest first, at most max_rows of them, into
 * `host` (caller-owned, max_rows * (2P + R) doubles, row-major) after the work enqueued on `stream`, and
 * synchronises it; *rows_out is the number copied, *first_iter (may be NULL) the session iteration count
 * after the first of them (iterations are counted from 1).  When more than `rows` iterations passed since the
 * last read the oldest were overwritten: the copy then starts at the oldest row still held, which
 * *first_iter shows.  sh_sdmm_state_import empties the ring and numbers its rows from the imported iteration
 * count.  Errors: SH_EINVAL (NULL, rows out of range, ring off for read), SH_ENOMEM. */
sh_status sh_sdmm_metrics_enable(sh_sdmm s, int32_t rows, int32_t* row_width);
sh_status sh_sdmm_metrics_read(sh_sdmm s, double* host, int32_t max_rows, int32_t* rows_out, int64_t* first_iter,
                               void* stream);
sh_status sh_sdmm_destroy(sh_sdmm s);

/* ---------------------------------------------------------------------------
 * Learned warm start: a U-Net mapping the normalised dirty image to a first
 * image estimate x0 (and, through Psi^dagger x0, first weights W) for the SDMM
 * solve above, which keeps its constraints and stopping test.  Not part of the
 * paper's method; it only changes where the iterations start.
 *
 * Architecture (levels L, base channels c, c_l = c 2^(l-1)): encoder level l =
 * two 3x3 zero-padded convolutions + ReLU (levels >= 2 after a 2x2 max-pool);
 * decoder level l = L-1..1: 2x2 stride-2 transposed convolution c_{l+1} -> c_l,
 * concat [upsampled, encoder level l], two 3x3 convolutions + ReLU; head = 1x1
 * convolution to one channel + ReLU.  Loss: mean squared error over pixels between the head's
 * output before its ReLU and the target (the ReLU applies to predictions only).
 * Parameters are one flat float32 array: for each layer in the order enc1a,
 * enc1b, ..., encLb, up(L-1)t, up(L-1)a, up(L-1)b, ..., up1b, head, the weight
 * then the bias; conv weights [cout][cin][3][3], transposed-conv weights
 * [cin][cout][2][2], head [1][c][1][1].
 * Arithmetic: bfloat16 operands (weights, activations, layer gradients) in
 * MFMA products with float32 accumulation; float32 master weights, gradients
 * and Adam state.
 * Images: device float32, B x H x W, H and W divisible by 2^(L-1).
 * A handle keeps its activations and its bfloat16 weight operands (converted again only after the
 * parameters change): calls on one handle must be ordered, on one stream or by the caller.
 * ------------------------------------------------------------------------- */
typedef struct sh_unet_s* sh_unet;
/* base: multiple of 16 in [16, 128]; levels 1..6.  Parameters start at zero.  Synchronous. */
sh_status sh_unet_create(int32_t base, int32_t levels, sh_unet* out);
sh_status sh_unet_destroy(sh_unet u);
sh_status sh_unet_num_params(sh_unet u, int64_t* n_out);
/* Copy n host float32 parameters in (resets the Adam state) or out.  Synchronous.  SH_ENONFINITE on
 * a non-finite parameter. */
sh_status sh_unet_set_params(sh_unet u, const float* host, int64_t n);
sh_status sh_unet_get_params(sh_unet u, float* host, int64_t n);
/* y = network(x), both device float32 B x H x W.  Async. */
sh_status sh_unet_forward(sh_unet u, const float* x, int32_t B, int32_t H, int32_t W, float* y, void* stream);
/* Loss mean((z(x) - target)^2), z the head output before its ReLU (host), and, if grads_host is not
 * NULL, its gradient with respect to every parameter (host, flat layout).  Synchronous. */
sh_status sh_unet_loss_grad(sh_unet u, const float* x, const float* target, int32_t B, int32_t H, int32_t W,
                            double* loss_out, float* grads_host, void* stream);
/* One Adam step (lr, beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) on the loss of the batch;
 * loss_out (host, may be NULL: then the call is async) receives the loss before the step. */
sh_status sh_unet_train_step(sh_unet u, const float* x, const float* target, int32_t B, int32_t H, int32_t W,
                             float lr, double* loss_out, void* stream);

/* Warm start of a solve with plan op (P problems, image side n): x0_out (device P x n x n) =
 * s U(d / s) per problem, with d = Phi^dagger y / (Phi^dagger Phi delta)(centre) the dirty image
 * in units of the PSF peak (delta = unit image at (n/2, n/2)) and s = RMS(d) (so the network
 * input has unit RMS).  y: device M complex64,
 * user order.  Pass x0_out to sh_sdmm_solve with w_from_x0 = 1.  Synchronous (allocates scratch). */
sh_status sh_warm_start(sh_unet u, sh_op op, const float* y, float* x0_out, void* stream);
/* The network input alone: d_out (device P x n x n) = d / s and scale_out (device P float32) = s,
 * with d and s as for sh_warm_start.  Synchronous. */
sh_status sh_dirty_normalised(sh_op op, const float* y, float* d_out, float* scale_out, void* stream);
/* x[p] *= scale[p] (invert 0) or x[p] /= scale[p] (invert 1) for P images of N pixels (device).  Async. */
sh_status sh_scale_images(float* x, const float* scale, int32_t P, int64_t N, int32_t invert, void* stream);

/* ---------------------------------------------------------------------------
 * Kernel timing (HIP events around the gridding/degridding launches).
 * ------------------------------------------------------------------------- */
/* Enable (1) or disable (0) event timing; enabling clears the counters. */
sh_status sh_profile_enable(int32_t on);
/* Launch count and total milliseconds of kernel group `name` ("degrid", "grid", "fold",
 * "fft_rows", "fft_cols", "dwt", "prox", "cg", "toeplitz") recorded since enabling.
 * Synchronises the device. */
sh_status sh_profile_read(const char* name, int64_t* count, double* total_ms);

#ifdef __cplusplus
}
#endif
#endif /* SARAHIP_H */
