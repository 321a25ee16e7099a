/*
 * mapmaker.h -- C ABI of the MI355X (gfx950) GLS map-making library.
 *
 * The library solves the generalised-least-squares map-making problem of
 * arXiv:2501.16122, Sec. II: with time-ordered data d (eq. (1)), the pointing
 * matrix P whose row t holds 1, cos 2psi_t, sin 2psi_t at the I, Q, U columns
 * of the pixel seen at sample t (eq. (2), (8)), and a noise covariance N,
 * the map is
 *
 *     x = (P^T N^-1 P)^-1 P^T N^-1 d           (eq. (5)),
 *
 * found by preconditioned conjugate gradient on A x = b with
 * A = P^T N^-1 P and b = P^T N^-1 d (eq. (6)) and the block-Jacobi
 * preconditioner M = (P^T diag(N)^-1 P)^-1 made of per-pixel 3x3 inverses
 * (eq. (7); nc x nc for the map forms with fewer values per pixel, see
 * below).  The operators are lazy (Sec. III-A): building a handle
 * precomputes the pointing elements and preconditioner once, and each apply
 * call only streams the timeline.
 *
 * Conventions shared by every call
 * --------------------------------
 * - Status: MM_OK (0) on success; MM_NOTCONVERGED (> 0) when a solve ran out
 *   of iterations (its outputs are still written); negative codes are errors
 *   and leave outputs undefined.  mm_last_error() returns a thread-local
 *   message for the last failing call of this thread.
 * - Memory ownership follows Sec. III-A: the caller allocates and frees every
 *   array.  Pointers named *_host are host memory read during the call;
 *   every other pointer is device memory on the current HIP device.  Derived
 *   state lives in a caller-provided device workspace sized by the matching
 *   *_workspace_size call; the library allocates no device memory of its own.
 *   A handle borrows the caller's device arrays (pix, psi, workspace) for its
 *   whole lifetime: keep them alive until *_destroy.
 * - Streams: `stream` is a hipStream_t (NULL = default stream).  Calls are
 *   stream-ordered and asynchronous unless marked "blocking".
 * - Layout: the timeline is detector-major (detector d owns samples
 *   [det_offsets[d], det_offsets[d+1])); pixel indices are int32 in
 *   [0, n_pix); maps over the kept pixels are interleaved I, Q, U
 *   (f64[3 * n_kept], eq. (8)); full-grid maps are f64[3 * n_pix].
 * - Map forms: a pointing handle solves for nc values per pixel, nc being
 *   its MM_STOKES_* form: I, Q, U (nc = 3, the default), Q, U only (nc = 2:
 *   the row of P keeps cos 2psi, sin 2psi) or I only (nc = 1: the row is the
 *   constant 1 and psi is not read).  Sec. III-B sizes the pixel-domain
 *   array at two or three values per pixel.  Every "3" in the vector and map
 *   sizes below is the handle's nc.
 * - Precision: `dtype` is the storage type of psi and of every timeline
 *   (MM_F64 or MM_F32).  `arith` selects the arithmetic of an operator's
 *   timeline-domain work (MM_F64 or MM_F32); pixel-domain vectors, bin sums
 *   and all PCG dot products are always FP64.
 */
#ifndef MAPMAKER_H
#define MAPMAKER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  MM_OK = 0,
  MM_NOTCONVERGED = 1,
  MM_EINVAL = -1,      /* bad argument, shape or pixel index            */
  MM_ENOSPC = -2,      /* workspace smaller than the size query asked for */
  MM_EHIP = -3,        /* a HIP runtime call failed                      */
  MM_EBREAKDOWN = -4   /* PCG breakdown: p^T A p <= 0 or non-finite       */
};

enum { MM_F64 = 0, MM_F32 = 1 };

/* Map forms (the value is the number of unknowns per pixel, nc). */
enum { MM_STOKES_I = 1, MM_STOKES_QU = 2, MM_STOKES_IQU = 3 };

typedef struct mm_pointing_s* mm_pointing_t;
typedef struct mm_noise_s* mm_noise_t;

/* Message of the last failing call on this thread ("" if none). */
const char* mm_last_error(void);

/* ABI revision of this header (bumped on incompatible change): 5. */
int mm_abi_version(void);

/* ------------------------------------------------------------------------
 * Pointing (the precomputation of Sec. III-A / "ProcessTimeSamples", and the
 * preconditioner blocks of eq. (7)).
 * ------------------------------------------------------------------------ */

/* Device workspace bytes that mm_pointing_build needs for a timeline of
 * n_samples samples over n_det detectors and a grid of n_pix pixels, with
 * angles and timelines stored in `dtype` (MM_F64 or MM_F32; any other value
 * fails with MM_EINVAL).  The same size serves every map form. */
int mm_pointing_workspace_size(int64_t n_samples, int32_t n_det, int32_t n_pix, int32_t dtype, size_t* bytes);

/* Build the pointing handle (blocking: synchronises `stream` once to read
 * the number of kept pixels and the pixel-range check).
 *   pix          int32[n_samples] device, pixel of each sample
 *   psi          f64 or f32 [n_samples] device (dtype), angle psi_t of eq. (2)
 *   det_offsets_host  int64[n_det + 1], 0 = first, n_samples = last
 *   det_weight_host   f64[n_det], diag(N)^-1 per detector (1/sigma_d^2) used
 *                     for the preconditioner blocks of eq. (7)
 *   min_hits, cond_max  a pixel is masked (dropped from the unknowns, its
 *                     samples get a zero row of P) when it has fewer than
 *                     min_hits samples or its 3x3 block has 2-norm condition
 *                     number > cond_max (+inf when singular)
 * Kept pixels are numbered in ascending pixel order.  A pixel index outside
 * [0, n_pix), or an angle that is not finite or has |2 psi| >= 4e8, fails
 * with MM_EINVAL and no handle. */
int mm_pointing_build(const int32_t* pix, const void* psi, int32_t dtype, int64_t n_samples,
                      const int64_t* det_offsets_host, int32_t n_det, const double* det_weight_host,
                      int32_t n_pix, int32_t min_hits, double cond_max,
                      void* workspace, size_t ws_bytes, void* stream, mm_pointing_t* out);

/* mm_pointing_build for a chosen map form (Sec. III-B: two or three values
 * per pixel; the intensity-only form has one).  stokes is MM_STOKES_IQU (as
 * mm_pointing_build), MM_STOKES_QU or MM_STOKES_I.  The blocks of eq. (7)
 * are nc x nc: for QU the sums of w (cos^2, cos sin, sin^2), for I the sum
 * of w; a QU block's condition number is its 2-norm one, an I block's is 1
 * (+inf when its sum is 0).  min_hits applies as given (nc is the natural
 * choice).  psi may be NULL for MM_STOKES_I, which never reads it; the same
 * workspace size as mm_pointing_build suffices.  Errors as mm_pointing_build,
 * plus MM_EINVAL for another stokes value. */
int mm_pointing_build_stokes(const int32_t* pix, const void* psi, int32_t dtype, int64_t n_samples,
                             const int64_t* det_offsets_host, int32_t n_det, const double* det_weight_host,
                             int32_t n_pix, int32_t stokes, int32_t min_hits, double cond_max,
                             void* workspace, size_t ws_bytes, void* stream, mm_pointing_t* out);

/* The handle's map form (MM_STOKES_*, i.e. nc) in *stokes (host). */
int mm_pointing_stokes(mm_pointing_t pt, int32_t* stokes);

/* Sizes of a built handle (host outputs; any pointer may be NULL). */
int mm_pointing_info(mm_pointing_t pt, int32_t* n_kept, int64_t* n_samples, int32_t* n_pix,
                     int32_t* n_det, int32_t* dtype);

/* Copy the integer products of the build (any pointer may be NULL):
 *   hits int32[n_pix], mask uint8[n_pix] (1 = masked),
 *   compact int32[n_pix] (-1 = masked), kept int32[n_kept],
 *   minv f64[nc * nc * n_kept] (row-major nc x nc inverse blocks, eq. (7)). */
int mm_pointing_export(mm_pointing_t pt, int32_t* hits, uint8_t* mask, int32_t* compact,
                       int32_t* kept, double* minv, void* stream);

/* Precompute the pointing elements of eq. (8) once (Sec. III-A) into caller
 * memory, and let the band-Toeplitz and template operators stream them
 * instead of evaluating sin/cos from psi each time they need a row:
 *   weights   dtype[n_samples] device, same dtype as psi: u_t = tan psi_t,
 *             from which the kernels rebuild the row's (cos 2psi_t, sin 2psi_t)
 *             = ((1 - u^2), 2u) / (1 + u^2) with a few multiplies (the
 *             half-angle substitution; u is finite for every finite stored
 *             angle, and a relative error e in u moves 2psi by at most e);
 *             borrowed until detached or destroyed
 * Stored weights serve arithmetic no finer than their dtype (FP32 weights are
 * not used by FP64 arithmetic).  weights = NULL detaches.  Stream-ordered.
 * The intensity-only form has no weights (MM_EINVAL). */
int mm_pointing_attach_weights(mm_pointing_t pt, void* weights, void* stream);

/* Free the host-side handle; the caller frees its own arrays and workspace. */
int mm_pointing_destroy(mm_pointing_t pt);

/* ------------------------------------------------------------------------
 * Noise models N^-1 (eq. (5)).  White: diagonal, 1/sigma_d^2 per detector.
 * Band-Toeplitz: on each stationary chunk [chunk_offsets[c],
 * chunk_offsets[c+1]) the finite section z_i = sum_{|i-j| < lambda}
 * coeff[f][|i-j|] y_j with f = chunk_filter[c]; chunks do not couple and
 * samples outside every chunk get z = 0.  Applied by overlap-save FFTs.
 * ------------------------------------------------------------------------ */

int mm_noise_white_workspace_size(int32_t n_det, size_t* bytes);
int mm_noise_white(const double* det_weight_host, int32_t n_det, void* workspace, size_t ws_bytes,
                   void* stream, mm_noise_t* out);

/* 1 <= lambda <= 4096; chunks must be ordered, non-overlapping and must not
 * cross a detector start (checked against the pointing at apply time). */
int mm_noise_toeplitz_workspace_size(int32_t lambda, int32_t n_filt, const int64_t* chunk_offsets_host,
                                     int64_t n_chunks, size_t* bytes);
int mm_noise_toeplitz(const double* coeff_host, int32_t lambda, int32_t n_filt,
                      const int64_t* chunk_offsets_host, const int32_t* chunk_filter_host,
                      int64_t n_chunks, void* workspace, size_t ws_bytes, void* stream,
                      mm_noise_t* out);
/* Circulant N^-1 per stationary chunk (the structured noise model of
 * Sec. IV, diagonal in the chunk's Fourier basis): each chunk is taken as
 * periodic and its first row holds coeff[f][0 .. lambda-1] and their mirror
 * image, i.e. z_i = sum_j coeff[f][d(i,j)] y_j over the chunk with d the
 * distance around it (d < lambda).  Arguments, tables and workspace (sized by
 * mm_noise_toeplitz_workspace_size) as for mm_noise_toeplitz; every
 * non-empty chunk must be longer than 2 (lambda - 1), else MM_EINVAL. */
int mm_noise_circulant(const double* coeff_host, int32_t lambda, int32_t n_filt,
                       const int64_t* chunk_offsets_host, const int32_t* chunk_filter_host,
                       int64_t n_chunks, void* workspace, size_t ws_bytes, void* stream,
                       mm_noise_t* out);
/* Template-filtered white weights: a general W of eq. (4) built from the
 * filtering templates of Sec. IV.  On interval i, samples
 * [interval_offsets[i], interval_offsets[i+1]) of one detector d, the
 * polynomial baselines of degree < K_i (K_i = interval_order_host[i], or
 * `order` for every interval when that pointer is NULL; 0 <= K_i <= 8) are
 * marginalised:
 *     W y = w_d (y - T (T^T T)^-1 T^T y)   on the interval,
 * T the polynomials of degree < min(K_i, length) in the sample position
 * (any basis: W does not depend on it), w_d = det_weight_host[d].  So
 * A = P^T W P and b = P^T W d give the map with every interval's baselines
 * projected out; K_i = 0 is plain white weighting.  The intervals must
 * partition the timeline: interval_offsets[0] = 0, non-decreasing, the last
 * equal to the pointing's n_samples, none crossing a detector start (checked
 * at apply time, MM_EINVAL).  A map component constant over whole intervals
 * (the I monopole with K_i >= 1) is then unconstrained; PCG started from 0
 * stays orthogonal to it.  The handle works with every operator and solve
 * entry point, mm_batch_step included (a batch may mix template-filtered,
 * white and band-Toeplitz members); the operator variants do not apply.
 * Workspace: mm_noise_templates_workspace_size; copies its tables there and
 * synchronises `stream` once. */
int mm_noise_templates_workspace_size(int32_t n_det, int64_t n_intervals, size_t* bytes);
int mm_noise_templates(const double* det_weight_host, int32_t n_det, const int64_t* interval_offsets_host,
                       const int32_t* interval_order_host, int32_t order, int64_t n_intervals,
                       void* workspace, size_t ws_bytes, void* stream, mm_noise_t* out);
int mm_noise_destroy(mm_noise_t nz);

/* ------------------------------------------------------------------------
 * Operators (eq. (3), (6), (7)).  x, q, r, z are f64[nc * n_kept]; timelines
 * are dtype[n_samples] of the pointing's dtype.  Outputs are overwritten.
 * ------------------------------------------------------------------------ */

/* tod = P x  (zero on samples of masked pixels). */
int mm_apply_P(mm_pointing_t pt, const double* x, void* tod, int32_t arith, void* stream);
/* q = P^T tod. */
int mm_apply_PT(mm_pointing_t pt, const void* tod, double* q, int32_t arith, void* stream);
/* tod_out = N^-1 tod_in (tod_out must not alias tod_in). */
int mm_apply_Ninv(mm_noise_t nz, mm_pointing_t pt, const void* tod_in, void* tod_out, int32_t arith,
                  void* stream);
/* q = P^T N^-1 P x in one fused pass: the timeline-length intermediate stays
 * on chip (registers for white noise, LDS for band-Toeplitz). */
int mm_apply_A(mm_pointing_t pt, mm_noise_t nz, const double* x, double* q, int32_t arith, void* stream);
/* mm_apply_A with an explicit band-Toeplitz operator variant (the bits of
 * mm_solve_opts.op_variant, 0 <= variant < 32; ignored for white noise).
 * Every variant computes the same sums up to the order of floating-point
 * atomics; this call lets a caller check or time one. */
int mm_apply_A_variant(mm_pointing_t pt, mm_noise_t nz, const double* x, double* q, int32_t arith, int32_t variant,
                       void* stream);
/* b = P^T N^-1 tod (the right-hand side of eq. (6)), fused likewise. */
int mm_rhs(mm_pointing_t pt, mm_noise_t nz, const void* tod, double* b, int32_t arith, void* stream);
/* Q = A X for n_rhs vectors at once (X, Q: f64[n_rhs][nc * n_kept]); the
 * right-hand sides of one tile run side by side, so the pointing is streamed
 * from memory once for all of them. */
int mm_apply_A_multi(mm_pointing_t pt, mm_noise_t nz, int32_t n_rhs, const double* x, double* q, int32_t arith,
                     void* stream);
/* z = M r with the nc x nc inverse blocks of eq. (7). */
int mm_apply_M(mm_pointing_t pt, const double* r, double* z, void* stream);
/* map_full f64[nc * n_pix] = x at kept pixels, 0 at masked ones. */
int mm_expand_map(mm_pointing_t pt, const double* x, double* map_full, void* stream);

/* ------------------------------------------------------------------------
 * Solve (eq. (5)/(6) by PCG, Sec. II).  Blocking.
 * ------------------------------------------------------------------------ */

typedef struct {
  double tol;           /* stop at ||r_k|| / ||b|| <= tol (recursive residual); default 1e-10 */
  int32_t max_iter;     /* iteration cap per PCG run; default 2000                         */
  int32_t fixed_iter;   /* > 0: run exactly this many iterations (no early stop)          */
  int32_t check_every;  /* host polls convergence every this many iterations; default 8   */
  int32_t mixed;        /* 0: FP64 operator; 1: FP32 inner solves + FP64 refinement      */
  int32_t max_outer;    /* mixed: refinement steps cap; default 10                        */
  double inner_tol;     /* mixed: inner relative tolerance; default 1e-5                 */
  int32_t timing;       /* 1: time each iteration and its A kernel with HIP events       */
  int32_t autotune;     /* 1: time the band-Toeplitz operator variants on this problem at
                           solver creation and keep the fastest (remembered by the noise
                           handle per problem size, and across the process's noise handles
                           per size class: same device, storage, arithmetic, right-hand
                           sides, values per pixel, band and noise kind, and sample count
                           rounded down to a power of two); 0: use op_variant            */
  int32_t op_variant;   /* variant when not autotuned (default 0): bit 0 = tiles in launch
                           order instead of the XCD-aware order, bit 1 = map read from
                           global memory instead of staged in LDS, bit 2 = shorter tiles in
                           runs that carry the overlapping half-window from tile to tile
                           (needs stored pointing weights; never stages), bit 3 = plain
                           tiles with two workgroups per CU, whose FFT exchanges pass real
                           and imaginary parts through half the LDS in turn (bits 1 and 2
                           do not apply), so the memory phases of one tile overlap the
                           FFT of another, bit 4 = plain tiles of the arithmetic's longer
                           plan (FP64: 16384 points, the FP32 plan's tile length; FP32:
                           32768 points), one 1024-thread workgroup per CU with half-LDS
                           exchanges (bits 1 to 3 do not apply); 0 <= op_variant < 32      */
  int32_t graph;        /* 1: the first mm_solver_step of a given length k > 0 records its k
                           iterations (operator and PCG launches) into a HIP graph and
                           every later step of that length replays it with one graph
                           launch on the solver's stream (recorded on a private stream,
                           so the caller's may be the null stream); another k records
                           anew.  Same kernels and arguments as the eager launches.
                           Ignored when timing = 1 and by mm_batch_step.  Default 0       */
  const double* x0;     /* start vector (device, f64[n_rhs][nc * n_kept]) or NULL for x0 = 0;
                           the residual starts at b - A x0 (FP64), the mixed form refines from
                           x0; the solve's outputs do not alias it                           */
  int32_t bj_start;     /* mixed form with x0 NULL: 1 (default) refines from the block-Jacobi
                           map x0 = M b (eq. (7)), whose residual b - A x0 is formed in FP64;
                           0 from x0 = 0.  The FP32 inner solves then work on corrections
                           whose I component is no longer the sky's, so FP32 rounding of
                           the I-dominated timeline leaks far less into Q and U            */
} mm_solve_opts;

typedef struct {
  int32_t iters;        /* PCG iterations (summed over inner solves)         */
  int32_t outer_iters;  /* refinement steps (1 for the FP64 solve)          */
  int32_t converged;    /* 1 if the tolerance was met                        */
  int32_t breakdown;    /* 1 if PCG broke down                               */
  double rel_resid;     /* last recursive residual ||r|| / ||b||            */
  double true_rel_resid;/* ||b - A x|| / ||b|| recomputed in FP64 at exit    */
  /* filled when opts.timing = 1 (iterations that did work only):           */
  double op_ms;         /* summed duration of the A = P^T N^-1 P kernel      */
  int32_t op_launches;  /* launches summed in op_ms                          */
  int32_t op_variant;   /* band-Toeplitz operator variant used (see opts)    */
  double iter_ms_p50;   /* median duration of one PCG iteration              */
  double iter_ms_p99;   /* 99th percentile of the same                       */
} mm_solve_info;

/* Fill opts with the defaults above. */
int mm_solve_opts_default(mm_solve_opts* opts);

int mm_solve_workspace_size(mm_pointing_t pt, mm_noise_t nz, const mm_solve_opts* opts, size_t* bytes);

/* Solve for the map from the timeline `tod` (dtype of the pointing).
 *   map_out   f64[nc * n_pix] device, full grid (0 at masked pixels), may be NULL
 *   x_out     f64[nc * n_kept] device, compact solution, may be NULL
 *   history_host  f64[history_len] host, ||r_k||/||b|| for k = 0.. (may be NULL)
 * Returns MM_OK, MM_NOTCONVERGED or an error (MM_EBREAKDOWN keeps the last
 * good iterate in the outputs). */
int mm_solve(mm_pointing_t pt, mm_noise_t nz, const void* tod, double* map_out, double* x_out,
             const mm_solve_opts* opts, mm_solve_info* info, double* history_host, int32_t history_len,
             void* workspace, size_t ws_bytes, void* stream);

/* mm_solve for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same solve, with the solver's vectors, partial sums and state in a 64 MiB
 * device array inside the library instead of a caller workspace.  The call
 * allocates no device memory, pinned memory, event or graph (no history
 * output; opts.autotune, opts.timing and opts.graph must be 0, else
 * MM_EINVAL: pass opts.op_variant).  The array holds the state of one
 * right-hand side of at most about 0.9 million unknowns (nc * n_kept, e.g.
 * a 512^2 I, Q, U map, FP64 or mixed): a larger problem fails with
 * MM_ENOSPC before any work.  Each GPU the library runs on holds its own
 * copy of the array until the process ends; every call on one GPU shares it
 * (a call clears what it needs), so calls that overlap on one GPU race.
 * Blocking; returns like mm_solve. */
int mm_solve_noalloc(mm_pointing_t pt, mm_noise_t nz, const void* tod, double* map_out, double* x_out,
                     const mm_solve_opts* opts, mm_solve_info* info, void* stream);

/* ------------------------------------------------------------------------
 * Resumable solves: one or several right-hand sides sharing a pointing and a
 * noise model (detector splits, Monte Carlo noise realisations), advanced in
 * asynchronous steps so that many solves can be in flight at once.
 * ------------------------------------------------------------------------ */

typedef struct mm_solver_s* mm_solver_t;

/* Workspace bytes of a solver of n_rhs right-hand sides for a problem with
 * at most n_kept_max kept pixels of ncomp values each (1, 2 or 3), without a
 * pointing handle: what mm_solver_workspace_size returns once the pointing
 * is built is never larger.  For sizing before the pointing exists, e.g.
 * admission by device footprint.  Host only. */
int mm_solver_workspace_bound(int32_t n_kept_max, int32_t ncomp, int32_t n_rhs, const mm_solve_opts* opts,
                              size_t* bytes);

int mm_solver_workspace_size(mm_pointing_t pt, mm_noise_t nz, int32_t n_rhs, const mm_solve_opts* opts,
                             size_t* bytes);

/* Form b = P^T N^-1 d (FP64) for each timeline of `tod` (dtype[n_rhs][n_samples])
 * and start PCG, asynchronously on `stream`, which the solver keeps using.
 * The workspace is borrowed until mm_solver_destroy. */
int mm_solver_create(mm_pointing_t pt, mm_noise_t nz, int32_t n_rhs, const void* tod, const mm_solve_opts* opts,
                     void* workspace, size_t ws_bytes, void* stream, mm_solver_t* out);

/* Enqueue up to k more PCG iterations (a pending outer refinement step first)
 * and an asynchronous copy of the solver state to host memory.  Never blocks;
 * the kernels of a right-hand side that is done return at once. */
int mm_solver_step(mm_solver_t sv, int32_t k);

/* Non-blocking: *done = 1 once every right-hand side has converged, broken
 * down or reached its caps, as of the last step whose state copy has landed;
 * *in_flight (may be NULL) = 1 while the latest step's copy has not landed;
 * info (n_rhs entries, may be NULL) reports the last landed state. */
int mm_solver_poll(mm_solver_t sv, int32_t* done, int32_t* in_flight, mm_solve_info* info);

/* Blocking: true FP64 residual, then the full-grid maps (f64[n_rhs][nc * n_pix],
 * may be NULL) and compact solutions (f64[n_rhs][nc * n_kept], may be NULL).
 * history_host receives right-hand side 0's residual history (inner, or the
 * outer FP64 one for mixed solves).  Returns like mm_solve. */
int mm_solver_finish(mm_solver_t sv, double* maps_out, double* x_out, mm_solve_info* info, double* history_host,
                     int32_t history_len);

/* Checkpoint and resume of a resumable solve (preempting it to free its
 * workspace, or resuming it elsewhere).
 * mm_solver_snapshot_size: bytes of a snapshot (a small header plus the
 * solver's share of its workspace).  mm_solver_snapshot (blocking: waits
 * for the solver's stream) copies the state after the last enqueued step
 * into dst, host or device memory, `bytes` >= the size (else MM_ENOSPC).
 * mm_solver_restore (blocking) overwrites the state of `sv` with a
 * snapshot; sv must have been created for the same problem: the same
 * pointing sizes, map form, dtype, number of right-hand sides and options
 * (MM_EINVAL otherwise).  The restored solve continues with mm_solver_step
 * and ends with mm_solver_finish as if it had never stopped, up to the
 * rounding order of floating-point atomics.  Timing statistics are not
 * part of a snapshot. */
int mm_solver_snapshot_size(mm_solver_t sv, size_t* bytes);
int mm_solver_snapshot(mm_solver_t sv, void* dst, size_t bytes);
int mm_solver_restore(mm_solver_t sv, const void* src, size_t bytes);

/* Free the host side (pinned state copy, events); the caller frees the workspace. */
int mm_solver_destroy(mm_solver_t sv);

/* Advance n resumable solvers together: the PCG iterations of Sec. II for
 * several independent map-making problems in shared launches.  Each of up to
 * k iterations is one operator launch per noise kind (white, band-Toeplitz or
 * circulant, template-filtered) over the tiles, or template intervals, of
 * every member's right-hand sides (A = P^T N^-1 P, eq. (6); A = P^T W P,
 * eq. (4), for template-filtered weights) and one
 * launch per PCG vector step over all their vectors; for mixed-precision
 * members a pending outer refinement step runs first.  Members may differ in
 * size, pointing, noise model and tolerances; they must share one device,
 * the stream they were created on, the timeline dtype, the precision mode
 * (mixed or not) and the map form, and hold at most 16 right-hand sides in
 * all (MM_EINVAL otherwise).  Asynchronous: every member records its state copy as after
 * mm_solver_step and is polled and finished on its own.  Batched steps are
 * not timed (opts.timing). */
int mm_batch_step(mm_solver_t* solvers, int32_t n, int32_t k);

/* ------------------------------------------------------------------------
 * The autotuner's choices (opts.autotune).  The process keeps one cache of
 * them keyed by problem class; a later problem of a cached class takes the
 * choice without timing.  These calls copy the cache out and add to it, so
 * that a caller can keep the choices across processes.  Host memory only;
 * no device work.  The calls are thread-safe.
 * ------------------------------------------------------------------------ */
typedef struct mm_tune_entry {
  int32_t device;       /* HIP device ordinal the choice was timed on         */
  int32_t log2_samples; /* floor(log2(n_samples))                             */
  int32_t dtype;        /* timeline storage: MM_F64 or MM_F32                  */
  int32_t arith;        /* operator arithmetic: MM_F64 or MM_F32               */
  int32_t n_rhs;        /* right-hand sides per solve, >= 1                    */
  int32_t ncomp;        /* values per pixel (map form): 1, 2 or 3              */
  int32_t lambda;       /* band of N^-1 (lags), 1 to 4096                      */
  int32_t noise_kind;   /* 1 = band-Toeplitz, 2 = circulant                    */
  int32_t op_variant;   /* the chosen operator variant, 0 <= op_variant < 32   */
} mm_tune_entry;

/* *n = the number of cached choices; the first min(cap, *n) of them are
 * copied to out (may be null when cap is 0).  MM_EINVAL for a null n, a
 * negative cap, or a null out with cap > 0. */
int mm_tune_cache_get(mm_tune_entry* out, int32_t cap, int32_t* n);

/* Add n choices from `in`; a choice whose class is cached already replaces
 * the cached one.  MM_EINVAL, with nothing added, for n < 0, a null `in`
 * with n > 0, or any entry outside the ranges above. */
int mm_tune_cache_put(const mm_tune_entry* in, int32_t n);

#ifdef __cplusplus
}
#endif

#endif /* MAPMAKER_H */
