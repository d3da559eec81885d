/*
 * sfft.h -- C ABI of the MI355X (gfx950) SFFT image-subtraction library.
 *
 * The operation is pipeline step 6 of the phrosty paper ("Pipeline steps":
 * apply SFFT subtraction to the cross-convolved science/template pair to
 * produce a difference image), a method that fits a delta-basis matching
 * kernel able to follow a spatially varying PSF ("Statement of need") by
 * solving a large linear system ("Future development").  The paper prints
 * no equations; the library computes exactly the following fit:
 *
 *   G    = 1 - [mask != 0]                       good pixels
 *   G_R  = G * [w <= y < ny-w] * [w <= x < nx-w] template side (w-wide border strip excluded)
 *   xh   = 2x/(nx-1) - 1, yh = 2y/(ny-1) - 1     frame-centred coordinates
 *   m_j  = xh^p yh^q, graded by d = p+q then q ascending (1; xh, yh; xh^2, xh yh, yh^2; ...)
 *   A_a  = m_a G_R R   (a < nK = (DK+1)(DK+2)/2),   S_m = G S
 *   (T_u X)(y,x) = X(y-u_y, x-u_x) inside the frame, else 0,   u in {-w..w}^2
 *   theta = argmin || S_m - sum_{a,u} k_{a,u} T_u A_a - sum_b c_b G m_b ||^2
 *         = Omega^{-1} beta   (normal equations, Cholesky, FP64)
 *   D = S - sum_{a,u} k_{a,u} T_u(m_a R) - sum_b c_b m_b   (unmasked R, whole frame)
 *
 * Coefficient layout (n = L^2 nK + nB, L = 2w+1):
 *   theta[a*L*L + (u_y+w)*L + (u_x+w)] = k_{a,u},   theta[nK*L*L + b] = c_b.
 *
 * Conventions for every entry point:
 *   - Every call returns an int status (SFFT_OK or a negative error code);
 *     nothing else crosses the ABI.
 *   - Image, mask, coefficient and output buffers are DEVICE pointers owned
 *     by the caller, row-major with x fastest and a row pitch `ld` (in
 *     elements, ld >= nx).  Inputs are never modified.
 *   - Work is enqueued asynchronously on the plan's HIP stream; buffers must
 *     stay alive until that stream has drained.  One plan per stream; a plan
 *     is not thread-safe.
 *   - Arguments are validated synchronously before anything is enqueued
 *     (SFFT_EINVAL).  Outcomes only known on the device (a non-positive
 *     Cholesky pivot, non-finite input) are recorded in device memory,
 *     LAPACK-style, and read with sfft_status(), which synchronises.
 */
#ifndef SFFT_H_
#define SFFT_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  SFFT_OK = 0,
  SFFT_EINVAL = -1,     /* bad descriptor or argument (w<0, DK<0, DB<0, N < 4w+2, N > 4096, NULL) */
  SFFT_ENOMEM = -2,     /* device allocation failed, or caller workspace too small            */
  SFFT_EHIP = -3,       /* a HIP runtime call failed                                          */
  SFFT_ENOTSPD = -4,    /* Omega is not positive definite (sfft_status only)                   */
  SFFT_ESTATE = -5,     /* call out of order (e.g. solve before build)                         */
  SFFT_ENONFINITE = -6, /* NaN/Inf in the science or template image (sfft_status only)          */
  SFFT_ETOOBIG = -7     /* larger than the static scratch of sfft_subtract_pair_noalloc           */
};

enum {
  SFFT_MODE_F64 = 0,    /* images double; FFTs, products and sums in FP64                          */
  SFFT_MODE_F32C = 1    /* images float; FFTs and spectral products in FP32, lag-window sums in
                           FP64, Omega stored in FP64; Cholesky, solve and refinement in FP64      */
};

typedef struct {
  int32_t ny, nx;        /* frame size, 4w+2 <= ny, nx <= 4096                                 */
  int32_t w;             /* kernel half-width, L = 2w+1                                       */
  int32_t dk, db;        /* polynomial degree of the kernel's / background's spatial variation */
  int32_t mode;          /* SFFT_MODE_F64 or SFFT_MODE_F32C                                    */
  int32_t refine_steps;  /* iterative-refinement steps after the Cholesky solve; -1 = 1        */
  int32_t flags;         /* assembly route, one of SFFT_FLAG_ASSEMBLY_* (bits 0-1), optionally
                            | SFFT_FLAG_CONST_RATIO | SFFT_FLAG_OUTPUT_MASK; other bits 0        */
} sfft_desc;

/* How the lag windows of Omega and beta are computed (sfft_desc.flags).
 * All routes give the same sums up to rounding:
 *   FFT    -- zero-padded transforms, spectral products, pruned inverses
 *             (cost ~ P^2 log P per plane; the route for large frames);
 *   DIRECT -- plain FP64 sums over the frame, sum_z X_l(z) X_r(z + d), for
 *             every lag d of every window (cost ~ lags * N^2; wins for small
 *             frames; needs nx <= 1024 and w <= 9, else SFFT_EINVAL);
 *   MFMA   -- the same FP64 sums as matrix-core products: for each source
 *             row y' of the right plane, C(dy, dx) += sum_x X_l(y' - dy, x)
 *             X_r(y', x + dx) is a (16 lags dy) x K x (16 lags dx) product
 *             on v_mfma_f64_16x16x4f64 (cost ~ lags^2 * N^2, on the FP64
 *             matrix cores; any w);
 *   AUTO   -- DIRECT when it is allowed and needs at most 1e9 multiply-adds,
 *             else FFT, until sfft_autotune_route has timed the routes on
 *             real inputs and kept the fastest. */
enum {
  SFFT_FLAG_ASSEMBLY_AUTO = 0,
  SFFT_FLAG_ASSEMBLY_FFT = 1,
  SFFT_FLAG_ASSEMBLY_DIRECT = 2,
  SFFT_FLAG_ASSEMBLY_MFMA = 3
};

/* Constant photometric ratio (sfft_desc.flags bit 4).  Left free, the sum of
 * the kernel -- the template-to-science flux ratio a point source at z sees,
 * sum_a m_a(z) s_a with s_a = sum_u k_{a,u} -- varies across the frame with
 * the kernel's shape ("Statement of need": a spatially varying kernel).  With
 * this flag the fit keeps it constant: the least-squares minimum under the
 * nK - 1 equality constraints s_a = 0 (a >= 1), computed from the same
 * factor as theta0 = Omega^{-1} beta:
 *   Z = Omega^{-1} C^T,  (C Z) lambda = C theta0,  theta = theta0 - Z lambda,
 * C (nK - 1 rows) summing the coefficients of each non-constant monomial.
 * Z's nK - 1 columns are extra right-hand sides of the same substitution and
 * refinement launches; the small system is solved by Cholesky on the device.
 * The background is not constrained.  sfft_residual still measures the free
 * normal equations, which a constrained theta does not satisfy.  No effect
 * when DK = 0. */
enum { SFFT_FLAG_CONST_RATIO = 16 };

/* Output-masked fit (sfft_desc.flags).  By default excluded pixels are
 * zero-filled: the excluded science pixels stay in the least squares as
 * equations "0 = model", which keeps every normal-matrix entry a
 * correlation.  With this flag the sum runs over the good output pixels only
 * (mask == 0), the template side unchanged (A_a = m_a G_R R):
 *   theta = argmin sum_{z: G(z)=1} (S(z) - sum k_{a,u} T_u A_a(z) - sum c_b m_b(z))^2,
 *   Omega = Omega_zf - Phi_M^T Phi_M,   beta = beta_zf,
 * Phi_M the kernel columns of the design-matrix rows at the excluded pixels
 * (their background columns and target are zero).  The correction is a
 * symmetric rank-|M| update of the (L^2 nK)^2 kernel block on the FP64
 * matrix cores, applied after the zero-filled assembly by every route; it
 * costs about (L^2 nK)^2 |M| multiply-adds (0.9 TFLOP for a 4088^2 frame
 * with 1.2 % excluded pixels at w = 9, DK = 2).  The workspace grows by
 * nK (ny + 2w)(nx + 2w) doubles and (ny nx + 2 ny + 1) int32.  A pair that
 * shares its template (sfft_batch_plan_shared) uses its owner's corrected
 * Omega; its beta needs no correction.  No effect without a mask. */
enum { SFFT_FLAG_OUTPUT_MASK = 32 };

typedef struct sfft_plan_s* sfft_handle;

/* n = (2w+1)^2 nK + nB for a valid descriptor.  Host only. */
int sfft_num_coeffs(const sfft_desc* d, int64_t* n);

/* Device bytes a plan for `d` needs (workspace for spectra, lag windows,
 * Omega and its factor).  Host only; no device is touched. */
int sfft_workspace_bytes(const sfft_desc* d, size_t* bytes);

/* Create a plan bound to `hip_stream` (a hipStream_t, NULL = default stream).
 * `workspace` NULL: the plan allocates (and frees in sfft_destroy) its own
 * device memory; otherwise it borrows `workspace_bytes` bytes of caller
 * device memory, 256-byte aligned (else SFFT_EINVAL), which must hold
 * sfft_workspace_bytes() (else SFFT_ENOMEM); its contents on entry do not
 * matter and the plan writes nothing outside it.  Both checks happen before
 * any device call.  Twiddle tables are computed in FP64 on the host and
 * uploaded; the call synchronises the stream. */
int sfft_plan(const sfft_desc* d, void* hip_stream, void* workspace, size_t workspace_bytes,
              sfft_handle* out);

/* Enqueue the assembly of Omega (n x n, FP64, both triangles) and beta (n):
 * the polynomial-weighted masked planes, their 2-D FFTs, the spectral
 * products and the pruned inverse transforms that keep only the lag windows
 * the entries need, and the gather into Omega/beta.
 * sci/tmpl: double* (F64) or float* (F32C), ny rows of pitch ld.
 * mask: uint8, nonzero = excluded pixel, pitch ld; NULL = no mask. */
int sfft_build_system(sfft_handle p, const void* sci, const void* tmpl, const uint8_t* mask,
                      int64_t ld);

/* Copy the assembled Omega (row-major n x n) and beta (n) into caller device
 * buffers (either may be NULL).  Requires a prior build. */
int sfft_get_system(sfft_handle p, double* omega, double* rhs);

/* Enqueue the FP64 Cholesky factorisation of Omega, the two triangular
 * solves and refine_steps steps of iterative refinement (residual
 * beta - Omega theta in FP64).  coeffs: device double[n] output, written
 * only if the factorisation succeeds.  info: device int32, set to 0 on
 * success or to k > 0 if the leading minor of order k is not positive
 * definite (LAPACK potrf convention).  Requires a prior build. */
int sfft_solve(sfft_handle p, double* coeffs, int32_t* info);

/* rho = ||beta - Omega coeffs||_2 / ||beta||_2 with the assembled system,
 * written to the device double `rho`.  Requires a prior build. */
int sfft_residual(sfft_handle p, const double* coeffs, double* rho);

/* Least-squares background for a given kernel: reads the kernel part
 * coeffs[0 .. nK L^2) (device double) and overwrites the background part
 * coeffs[nK L^2 .. n) with the solution c of Omega_BB c = beta_B - Omega_BK k
 * (the normal equations restricted to the background columns, FP64).  Used
 * to complete a predicted kernel before judging it with sfft_residual.  A
 * singular Omega_BB leaves NaN there.  Requires a prior build (SFFT_ESTATE). */
int sfft_fit_background(sfft_handle p, double* coeffs);

/* Enqueue D = S - sum_{a,u} k_{a,u} T_u(m_a R) - sum_b c_b m_b over the whole
 * frame with the unmasked template.  sci/tmpl/diff: double* (F64) or
 * float* (F32C), pitch ld; coeffs: device double[n]. */
int sfft_subtract(sfft_handle p, const void* sci, const void* tmpl, const double* coeffs,
                  void* diff, int64_t ld);

/* Enqueue out = K * img, the plan's kernel applied to one image:
 *   out(y, x) = sum_{a < nK} sum_{|u| <= w} k_{a,u} (m_a img)(y - u_y, x - u_x),
 * zero outside the frame, k_{a,u} = kcoef[a L^2 + (u_y+w) L + (u_x+w)] (the
 * kernel part of the coefficient layout, nK L^2 device doubles; any
 * background part is ignored).  This is the model the subtraction removes,
 * computed the same way (FFTs along x, the y-convolution in the row-spectral
 * domain, direct sums on the border columns).  With DK = 0 and a (2w+1)^2
 * stamp it is the plain linear convolution of pipeline step 5 of the paper
 * ("Pipeline steps": cross-convolve the template PSF with the science image
 * and the science PSF with the template), stamps up to 31 x 31 (w <= 15).
 * img/out: double* (F64) or float* (F32C), pitch ld, distinct buffers; the
 * arithmetic is FP64 in both modes.  Needs no build. */
int sfft_apply_kernel(sfft_handle p, const void* img, const double* kcoef, void* out, int64_t ld);

/* Enqueue the decorrelation kernel of pipeline step 7 of the paper
 * ("Pipeline steps": fit the decorrelation kernel and apply it to the
 * difference image, the science PSF and the cross-convolved science image;
 * the paper gives no formula, this is the project's reading).  With the
 * images cross-convolved as in step 5 (S' = P_R * S, R' = P_S * R) and
 * independent white noise sigma_sci, sigma_tmpl on the science and template
 * images, the difference image's noise has the spectrum
 *   N(f) = sigma_sci^2 |P_R^(f)|^2 + sigma_tmpl^2 |K_c^(f)|^2 |P_S^(f)|^2,
 * K_c the plan's matching kernel (coeffs, the fitted theta) at the frame
 * centre, K_c(u) = sum_a k_{a,u} (-2u_x/(nx-1))^p_a (-2u_y/(ny-1))^q_a.
 * The kernel with spectrum sqrt((sigma_sci^2 + sigma_tmpl^2) / N(f)) makes it
 * white; spectra are DFTs on a 64 x 64 grid of the stamps centred on tap
 * (0, 0), and psi is that kernel's (2t+1)^2 central taps:
 * psi[(u_y+t)(2t+1) + (u_x+t)], device doubles.  psf_sci (P_S) and psf_tmpl
 * (P_R): (2s+1)^2 device doubles, row-major, centred.  0 <= s, t <= 15 and
 * finite sigmas > 0, else SFFT_EINVAL.  Apply psi with sfft_apply_kernel on a
 * plan with w = t, DK = 0.  FP64; one block; needs no build. */
int sfft_decorrelation_kernel(sfft_handle p, const double* coeffs, const double* psf_sci, const double* psf_tmpl,
                              int32_t s, double sigma_sci, double sigma_tmpl, int32_t t, double* psi);

/* Synchronise the plan's stream and report device-side outcomes of the
 * last build/solve: SFFT_ENONFINITE if a non-finite science/template value
 * was seen, SFFT_ENOTSPD if the last solve hit a non-positive pivot, else
 * SFFT_OK.  `info_out` / `nonfinite_out` (host, may be NULL) receive the
 * raw flags. */
int sfft_status(sfft_handle p, int32_t* info_out, int32_t* nonfinite_out);

/* Stages timed by the optional per-plan event timer. */
enum {
  SFFT_STAGE_MOMENTS = 0,   /* background moments + non-finite scan            */
  SFFT_STAGE_ROW_FWD = 1,   /* plane generation + R2C along x                  */
  SFFT_STAGE_COL_FWD = 2,   /* FFT along y                                     */
  SFFT_STAGE_CORR = 3,      /* spectral products + pruned inverse along y      */
  SFFT_STAGE_ROW_WIN = 4,   /* lag-window inverse along x                      */
  SFFT_STAGE_GATHER = 5,    /* moments reduction + Omega/beta gather           */
  SFFT_STAGE_FACTOR = 6,    /* Cholesky factorisation                          */
  SFFT_STAGE_SOLVE = 7,     /* triangular solves + refinement                  */
  SFFT_STAGE_SUBTRACT = 8,  /* convolve-and-subtract                           */
  SFFT_STAGE_OUTMASK = 9,   /* output-mask correction of Omega                 */
  SFFT_NUM_STAGES = 10
};

/* HIP-event timing of the stages in `stage_mask` (bit s = stage s; 0 turns
 * timing off, SFFT_TIMING_ALL times every stage) enqueued on the plan's
 * stream from now on.  Events are recorded on that stream around each timed
 * stage, so the numbers are device time of that stage alone.  Enabling
 * creates SFFT_TIMING_RESERVE event pairs per timed stage (per pair of a
 * batch) up front, so that no event is created while the timed work runs
 * as long as sfft_timing_read is called at least every SFFT_TIMING_RESERVE
 * executions of a stage.  Bits past the last stage: SFFT_EINVAL. */
enum { SFFT_TIMING_ALL = (1 << SFFT_NUM_STAGES) - 1, SFFT_TIMING_RESERVE = 32 };
int sfft_timing_enable(sfft_handle p, int stage_mask);

/* Synchronise the plan's stream and return, per stage, the total milliseconds
 * and the number of timed executions since the last read (host arrays of
 * SFFT_NUM_STAGES entries, either may be NULL), then reset the counters. */
int sfft_timing_read(sfft_handle p, double* ms, int64_t* count);

/* ---- batches: S x T science/template pairs, sizes may differ per pair ----
 * The pairing of every science image with every template gives S x T
 * difference images (paper, "Pipeline steps", step 1; the paper runs them
 * serially, step 10).  A batch plan holds one single-pair plan per pair on
 * one stream and runs the assembly of every pair, then ONE blocked FP64
 * Cholesky + solve whose launches serve all pairs at once (the latency-bound
 * part), then the subtraction of every pair. */

/* Device bytes of a batch plan for `npairs` descriptors. Host only. */
int sfft_batch_workspace_bytes(const sfft_desc* descs, int32_t npairs, size_t* bytes);

/* Create a batch plan (allocates its workspace) bound to `hip_stream`.  Every
 * descriptor must ask for the same number of refinement steps (one batched
 * solve runs them for all pairs), else SFFT_EINVAL.  Single-pair calls on a
 * batch handle return SFFT_EINVAL; sfft_status, sfft_timing_* and
 * sfft_destroy accept it. */
int sfft_batch_plan(const sfft_desc* descs, int32_t npairs, void* hip_stream, sfft_handle* out);

/* A batch plan whose pairs may share a template (S science images against
 * one template and mask: the S x T pairing of "Pipeline steps", step 1).
 * tmpl_of: HOST int32[npairs]; tmpl_of[i] is the pair whose template and
 * mask pair i uses -- i itself (pair i owns them), or an earlier pair o < i
 * that owns them (tmpl_of[o] == o) and has the same descriptor, else
 * SFFT_EINVAL.
 *   Omega depends only on the template and the mask (its entries are
 * correlations of the planes m_a G_R R and G m_b), so every pair sharing a
 * template has the same Omega and the same factor: a sharing pair transforms
 * its science image alone, forms beta from it and the owner's template
 * spectra, and is solved with the owner's factor (its own substitutions and
 * refinement); its subtraction reuses the owner's row spectra of the
 * template.  The results equal those of sfft_batch_plan on the same pairs
 * (the shared quantities are computed once instead of once per pair).
 *   sfft_batch_run/capture on such a plan require tmpl[i] == tmpl[o],
 * mask[i] == mask[o] (as pointers; both NULL allowed) and ld[i] == ld[o] for
 * every sharing pair, else SFFT_EINVAL.  The info of a sharing pair is its
 * owner's factorisation outcome.  The workspace is at most
 * sfft_batch_workspace_bytes of the same descriptors. */
int sfft_batch_plan_shared(const sfft_desc* descs, const int32_t* tmpl_of, int32_t npairs, void* hip_stream,
                           sfft_handle* out);

/* Enqueue build + solve + subtract for every pair.  sci, tmpl, mask, ld,
 * coeffs, diff: HOST arrays of npairs entries holding DEVICE pointers (mask
 * array or entries may be NULL) and row pitches; info: device int32[npairs]
 * (may be NULL), LAPACK-style per pair, and a failed pair does not affect
 * the others.  A pair whose factorisation failed (info > 0) keeps its
 * coeffs untouched, and its diff is then computed from those untouched
 * coefficients: it is undefined as a result and must be discarded. */
int sfft_batch_run(sfft_handle b, const void* const* sci, const void* const* tmpl, const uint8_t* const* mask,
                   const int64_t* ld, double* const* coeffs, void* const* diff, int32_t* info);

/* Tune the plan on real inputs (sci/tmpl/mask/ld as for sfft_build_system;
 * for a batch handle, pair 0's buffers): builds the system once, then times
 * the correlation kernel for each candidate residue chunk (the number of
 * spectral residues staged in LDS per step, which sets the LDS per block and
 * so the blocks per CU) and keeps the fastest in the plan -- and in every
 * batch member with pair 0's descriptor.  Later builds use it; their results
 * equal the untuned ones up to rounding (the residue sums are regrouped).
 * Synchronises the stream.  Optional report (host arrays of capacity cap):
 * c1_out[i] chunk, ms_out[i] average kernel time; *count_out entries.  A plan
 * on the direct route has nothing to tune (count 0). */
int sfft_autotune(sfft_handle p, const void* sci, const void* tmpl, const uint8_t* mask, int64_t ld, int32_t* c1_out,
                  float* ms_out, int32_t cap, int32_t* count_out);

/* Time the assembly (sfft_build_system) of this plan on real inputs with each
 * route -- FFT, DIRECT (where allowed) and MFMA, one warm-up and three timed
 * builds each -- and, if the descriptor asks for SFFT_FLAG_ASSEMBLY_AUTO,
 * keep the fastest in the plan (and in every batch member with pair 0's
 * descriptor; for a batch handle the inputs are pair 0's).  A forced route is
 * kept.  ms_out (host, may be NULL): 3 entries, the average build time of the
 * FFT, DIRECT and MFMA routes in ms (-1 = not allowed); route_out (host, may
 * be NULL): the flag value of the route in use afterwards.  Results of the
 * routes agree up to rounding.  Synchronises the stream. */
int sfft_autotune_route(sfft_handle p, const void* sci, const void* tmpl, const uint8_t* mask, int64_t ld,
                        float* ms_out, int32_t* route_out);

/* Capture one sfft_batch_run with these buffers into a HIP graph held by the
 * batch handle (replacing an earlier capture); nothing runs yet.  The batch
 * stream must not be the null stream.  Stage timing is suspended during the
 * capture.  The captured pointers must stay valid while the graph is used. */
int sfft_batch_capture(sfft_handle b, const void* const* sci, const void* const* tmpl, const uint8_t* const* mask,
                       const int64_t* ld, double* const* coeffs, void* const* diff, int32_t* info);

/* Replay the captured batch run on the batch stream: one graph launch for all
 * pairs.  SFFT_ESTATE without a capture. */
int sfft_batch_launch(sfft_handle b);

/* ---- one pair with no allocation ----
 * For callers that cannot allocate device memory (serving loops and
 * harnesses that forbid hipMalloc, code that must not call an allocator).
 * Same result as sfft_plan (its own workspace) + sfft_build_system +
 * sfft_solve + sfft_subtract on one pair, bit for bit, with the same
 * arguments as those calls (info: device int32, may be NULL).  The
 * workspace is a static device array of SFFT_NOALLOC_SCRATCH_BYTES bytes,
 * one per GPU, that the library holds from its load until the process ends;
 * the call never allocates (no hipMalloc/hipFree, no host heap).  A pair
 * whose workspace would exceed it (sfft_workspace_bytes plus 96 KiB of
 * twiddle tables: frames up to 1024 x 1024 at w = 9, DK = DB = 2 fit in
 * both modes, 2048 x 2048 at those settings does not) returns SFFT_ETOOBIG
 * before anything is enqueued.
 *   - The first call on a GPU, and the first call after a descriptor
 *     change on that GPU, upload the plan's tables and synchronise the
 *     stream; later calls with the same descriptor only enqueue kernels.
 *   - Every call on one GPU shares that GPU's array, which keeps the last
 *     call's contents: calls that overlap on one GPU (other streams, other
 *     threads before the previous call's work has drained) race, and the
 *     caller must order them.  Host-side state is guarded per GPU.
 *   - Device outcomes go to `info` as in sfft_solve; the non-finite flag of
 *     this path is not reported (use a plan for sfft_status). */
#define SFFT_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
int sfft_subtract_pair_noalloc(const sfft_desc* d, void* hip_stream, const void* sci, const void* tmpl,
                               const uint8_t* mask, int64_t ld, double* coeffs, void* diff, int32_t* info);

/* Release the plan (and its workspace if the plan allocated it). */
void sfft_destroy(sfft_handle p);

/* Static, human-readable text for a status code. */
const char* sfft_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* SFFT_H_ */
