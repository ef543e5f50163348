/*
 * radsvd.h -- C ABI of the MI355X (gfx950) radial-SVD rotational image
 * alignment library.
 *
 * Method: A. Rangan, "Radial-recombination for rigid rotational alignment of
 * images and volumes" (arXiv 2202.07235).  Images A and targets B are given
 * by their Fourier transforms sampled on a polar quadrature grid (section 2.3:
 * radial nodes k_r with weights w_r for \int g(k) k dk, angles
 * psi_j = 2 pi j / Q).  For every image/target pair, every translation
 * delta_t of a small set, and every on-grid rotation gamma_m = 2 pi m / Q the
 * library evaluates the landscape
 *
 *   X[a][b][t][m] = sum_{h<H} sum_j conj(Ar_h[a](psi_j)) Br_h^t[b](psi_{j-m})
 *
 * where Ar_h = sum_r U[r][h] eta_r Ahat(k_r, .) and
 * Br_h^t = sum_r U[r][h] eta_r exp(-i k_r.delta_t) Bhat(k_r, .) are the
 * principal image rings (section 3.2, eta_r = sqrt(w_r dpsi)), and U holds
 * the leading H eigenvectors of the target-averaged kernel C (sections
 * 3.3-3.4).  At H = K this is the polar quadrature of
 * <Ahat, R_gamma T_delta Bhat> (section 2.2), i.e. (2 pi)^2 <A, R_gamma T_delta B>
 * with the prefactor dropped as the paper does.  It is evaluated in two steps
 * (section 2.4 / 3.3): a per-frequency contraction over h of the angular
 * Fourier coefficients, then a length-Q FFT over the frequency q.
 *
 * Conventions
 *   - Complex arrays are interleaved (re, im): complex128 when prec ==
 *     RADSVD_FP64, else complex64 (the memory layout of torch.complex128/64).
 *   - Polar samples are [n][K][Q], psi fastest.
 *   - All device buffers are owned by the caller (the library never calls
 *     hipMalloc).  Host arrays are read during the call only.
 *   - Work is enqueued on the caller's stream (a hipStream_t passed as void*;
 *     NULL = the default stream).  Calls do not synchronise the host.
 *   - Every call validates all arguments before its first launch and returns
 *     a status; it never aborts.  radsvd_last_error() describes the last
 *     failure of the calling thread.  Asynchronous device faults surface as
 *     RADSVD_ERR_DEVICE from the launch check or from a later call.
 */
#ifndef RADSVD_H
#define RADSVD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RADSVD_OK = 0,
    RADSVD_ERR_INVALID_ARG = 1,   /* a size, pointer or flag is out of range       */
    RADSVD_ERR_UNSUPPORTED = 2,   /* valid, but not implemented for this shape/mode */
    RADSVD_ERR_WORKSPACE = 3,     /* workspace missing, misaligned or too small     */
    RADSVD_ERR_DEVICE = 4         /* a HIP call or kernel launch failed             */
} radsvd_status;

/* Arithmetic of the per-frequency contraction (the rest of the path is FP32,
 * or FP64 for RADSVD_FP64; translation phases and the eigensolver are always
 * FP64). */
typedef enum {
    RADSVD_FP64 = 0,    /* complex128 in, FP64 everywhere                         */
    RADSVD_FP32 = 1,    /* FP32 products, FP32 accumulation                        */
    RADSVD_BF16 = 2,    /* operands rounded to bf16, FP32 accumulation             */
    RADSVD_BF16X3 = 3   /* operands split x = hi + mid + lo (bf16 each); 3 or 6    */
                        /* bf16 cross products summed in FP32                      */
} radsvd_precision;

/* align_pairs output selection (bit flags). */
enum {
    RADSVD_OUT_BEST = 1,   /* best score and its (m, t) per pair                       */
    RADSVD_OUT_LSE = 2,    /* log-sum-exp over (t, m) per pair, and over b per image   */
    RADSVD_OUT_FULL = 4    /* the whole landscape X[a][b][t][m]                        */
};

typedef struct {
    int K;                  /* radial rings, 2 <= K <= 128                              */
    int Q;                  /* angles: even, Q = 2^a 3^b, 8 <= Q <= 512                 */
    int H;                  /* rank (principal rings kept), 1 <= H <= min(K, 32)        */
    int T;                  /* translations, 1 <= T <= 64                               */
    const double *k;        /* host [K]: ring radii k_r (> 0)                           */
    const double *w;        /* host [K]: radial weights w_r (> 0), sum g(k_r) w_r ~ \int g k dk */
    const double *delta;    /* host [T][2]: translations (dx, dy), same length unit as 1/k */
    int prec;               /* radsvd_precision                                         */
    int hermitian;          /* 1: caller asserts Ahat(k, psi + pi) = conj(Ahat(k, psi)) */
                            /*    for images and targets (real-space images); the library */
                            /*    then uses only the frequencies q in [0, Q/2]          */
    int products;           /* RADSVD_BF16X3 only: 3 (hi*hi + hi*mid + mid*hi) or 6     */
                            /* (+ mid*mid + hi*lo + lo*hi); ignored otherwise            */
    double sigma_delta;     /* >= 0: standard deviation of an isotropic Gaussian prior on */
                            /* the images' translations, same unit as delta.  0: kernel C */
                            /* of section 3.4 (rotations only); > 0: the translation- and */
                            /* rotation-averaged kernel of section 5 (see align_prepare)  */
} radsvd_problem;

typedef struct radsvd_plan radsvd_plan;   /* opaque host-side metadata */

/* Bytes of device workspace align_prepare needs for this problem and these
 * counts (0 if the arguments are invalid; see radsvd_last_error). */
size_t align_prepare_workspace(const radsvd_problem *prob, int n_img, int n_tgt);

/*
 * Precompute (paper section 3.5, operation-count items 1-3): the kernel C
 * of the targets at delta = 0 (section 3.4, q = 0 excluded, ring weights
 * sqrt(w_r w_r')), or with sigma_delta > 0 the kernel of the objective
 * averaged over grid rotations and Gaussian translations (section 5):
 *   C = eta_r eta_r' Re[ E+(k_r,k_r') sum_q conj(bq_r) bq_r'
 *                        - E-(k_r) E-(k_r') conj(bq0_r) bq0_r' ] / N_B,
 *   E+ = exp(-sigma^2 (k_r - k_r')^2 / 2), E- = exp(-sigma^2 k_r^2 / 2)
 * (the paper's E- with Bessel I of order -1/2 and +1/2 is this exponential),
 * bq the unitary angular spectrum of a target ring and bq0 its q = 0 term,
 * its FP64 eigendecomposition (descending eigenvalues, each
 * eigenvector's largest-magnitude entry positive), and the principal rings of
 * every image and of every target at every translation, transformed to
 * angular frequency.
 *
 *   A_polar  device [n_img][K][Q] images  (complex128 for FP64, else complex64)
 *   B_polar  device [n_tgt][K][Q] targets
 *   U_in     device [K][H] FP64 row-major, or NULL.  When given, it replaces
 *            the eigenvectors of C (columns should be orthonormal) and C is
 *            not formed; the eigenvalues reported by align_get_U are then NaN.
 *            With U_in NULL, a NaN or infinite target sample makes C
 *            non-finite: U and every eigenvalue are then NaN, and every pair
 *            of the plan takes the non-finite rule of align_pairs.
 *   ws       device workspace of ws_bytes >= align_prepare_workspace(),
 *            256-byte aligned; it holds everything the plan refers to.
 *   out      receives a new plan on RADSVD_OK (free with align_plan_destroy).
 *
 * Lifetime: ws, A_polar and B_polar must stay valid and unchanged until the
 * last call enqueued with the plan has completed (the backward pass reads the
 * polar samples).  Plans are immutable once prepared, with one exception: for
 * plans the fused pair kernel serves (Hermitian, not FP64, Q in {64, 96, 128,
 * 192, 256, 384, 512}) align_prepare writes only the fused kernel's operand
 * layout, and the first align_pairs_backward or align_refine_rotation call
 * writes the generic one (its space is part of ws) on its own stream.  Apart
 * from that first call, calls on different streams may share one plan.  n_img, n_tgt in [1, 2^20].
 */
radsvd_status align_prepare(const radsvd_problem *prob, int n_img, const void *A_polar,
                            int n_tgt, const void *B_polar, const double *U_in,
                            void *ws, size_t ws_bytes, void *stream, radsvd_plan **out);

/*
 * Per-pair computation (section 3.5, items 4-5): for every pair (a, b) and
 * translation t, the contraction over the principal rings at each angular
 * frequency q followed by the FFT over q (section 3.3, steps 1 and 2), and an
 * epilogue on chip:
 *
 *   RADSVD_OUT_BEST : best_score[a][b] = max_{t,m} Re X[a][b][t][m]  (f32),
 *                     best_m[a][b], best_t[a][b] (int32) its location; the
 *                     maximum-likelihood rotation of section 2.7 is
 *                     gamma = 2 pi m / Q.  Ties go to the smallest t*Q + m; a
 *                     pair whose landscape Re X holds a value that is not
 *                     finite (NaN or infinite) gets NaN and -1, -1.
 *   RADSVD_OUT_LSE  : lse_pair[a][b] = log sum_{t,m} exp(inv_sigma2 Re X)  (f32, inv_sigma2 > 0);
 *                     if lse_img != NULL, lse_img[a] = log sum_b exp(lse_pair[a][b]).
 *                     A pair with a non-finite landscape value gets NaN, and
 *                     so does lse_img of its image.
 *   RADSVD_OUT_FULL : X_full [n_img][n_tgt][T][Q] complex (plan's I/O type).
 *                     Hermitian plans (real landscapes) write imaginary parts 0;
 *                     the values are those the BEST and LSE epilogues see.
 *
 * Pointers of the modes not selected are ignored.  All outputs are device
 * arrays, row-major.
 */
radsvd_status align_pairs(const radsvd_plan *plan, int out_flags, float inv_sigma2,
                          float *best_score, int32_t *best_m, int32_t *best_t,
                          float *lse_pair, float *lse_img, void *X_full, void *stream);

/*
 * Rotations off the grid (section 2.2: rotating a ring by any gamma multiplies
 * its Fourier-Bessel coefficients by exp(-i q gamma); section 2.4: zero-padding
 * the frequency array before the transform over q gives a finer gamma grid).
 * For every pair (a, b) whose BEST output is (best_m, best_t), the landscape at
 * translation best_t is evaluated at the rotations
 *   gamma_j = 2 pi (R best_m + j) / (R Q),  j = -R+1 .. R-1,
 * i.e. the length-R*Q zero-padded transform within one grid step of the grid
 * maximum, with the frequencies in the band |q| <= Q/2 and the q = Q/2 term
 * taken as a cosine (so j = 0 reproduces the grid landscape).  Writes
 *   fine_score [n_img][n_tgt] f32: the largest Re X(gamma_j);
 *   fine_m     [n_img][n_tgt] int32: (R best_m + j) mod (R Q) of that maximum,
 *              gamma = 2 pi fine_m / (R Q); ties go to the smallest j.
 * best_m, best_t: device [n_img][n_tgt] int32, a BEST output of align_pairs with
 * this plan; a pair with best_m < 0 (non-finite landscape), or whose landscape
 * is not finite at a candidate rotation, gets NaN and -1.  The sums run in the
 * plan's I/O precision (FP64 for RADSVD_FP64, else FP32) on the plan's
 * principal rings in the generic layout, whatever the plan's contraction
 * precision (so j = 0 may differ from best_score by that precision's error);
 * the first call with a plan the fused kernel serves writes that layout (see
 * align_prepare).  R in [1, 64].  Errors: RADSVD_ERR_INVALID_ARG (NULL or
 * misaligned arrays, R outside [1, 64]).
 */
radsvd_status align_refine_rotation(const radsvd_plan *plan, const int32_t *best_m, const int32_t *best_t, int R,
                                    float *fine_score, int32_t *fine_m, void *stream);

/*
 * align_pairs for a list of pairs (principal-mode marching, section 5: the
 * candidates that a low-rank pass selects are evaluated again at a higher
 * rank).  pairs: device [n][2] int32 (image, target) of this plan; outputs as
 * in align_pairs but indexed by list position: best_score, best_m, best_t,
 * lse_pair [n], X_full [n][T][Q].  An entry outside the plan's counts gets
 * NaN and -1.  Runs the per-pair kernel in the plan's precision on the
 * generic operand layout (written on the first such call, see align_prepare).
 * Errors: RADSVD_ERR_INVALID_ARG (n < 1, NULL or misaligned arrays, flags as
 * in align_pairs).
 */
radsvd_status align_pairs_list(const radsvd_plan *plan, int out_flags, float inv_sigma2, int n, const int32_t *pairs,
                               float *best_score, int32_t *best_m, int32_t *best_t, float *lse_pair, void *X_full,
                               void *stream);

/*
 * The k best targets of every image by a score (marching, section 5):
 * cand[a][c], c < k, the target of the c-th largest score[a][.] (device
 * [n_img][n_tgt] f32, e.g. best_score of a low-rank align_pairs), ties to the
 * smaller target; NaN scores are never taken and slots beyond the finite ones
 * get -1.  k in [1, 1024].  Errors: RADSVD_ERR_INVALID_ARG.
 */
radsvd_status align_top_targets(int n_img, int n_tgt, const float *score, int k, int32_t *cand, void *stream);

/*
 * Landscape quality (section 3.5) of an approximate landscape X_est against a
 * reference X_ref (e.g. low rank against full rank), both device
 * [n_pairs][len] complex (FP64 if fp64 = 1, else FP32; FULL outputs with
 * len = T * Q), on their real parts:
 *   f [n_pairs] f32: the fraction of the pair's X_ref values that are <= X_ref
 *       at the argmax of X_est (first maximum), NaN if a value is not finite;
 *   pair_stats [n_pairs][6] FP64: per pair sum (e - r)^2, sum r^2, sum e, sum r,
 *       sum e^2, sum e r (output, also the reduction's input);
 *   summary [3] FP64: relative Frobenius error ||X_est - X_ref|| / ||X_ref||,
 *       correlation over the whole array, mean f (sums in a fixed order).
 * Errors: RADSVD_ERR_INVALID_ARG (sizes < 1, NULL or misaligned arrays).
 */
radsvd_status align_landscape_metrics(long long n_pairs, int len, const void *X_est, const void *X_ref, int fp64,
                                      float *f, double *pair_stats, double *summary, void *stream);

/* Bytes of device scratch align_pairs_backward needs for this plan. */
size_t align_backward_workspace(const radsvd_plan *plan);

/*
 * Backward pass of the soft-alignment loss L = sum_a grad_lse_img[a] lse_img[a]
 * (lse_img as produced by align_pairs with the same inv_sigma2).  Paper
 * section 2.6 (likelihood): under the Gaussian noise model of section 2.5
 * the log-likelihood of a target at pose (gamma, delta) against an image is,
 * up to terms constant in the pose, Re X / sigma^2; lse_pair is the log of
 * its sum over poses and lse_img the log of the sum over targets (a
 * marginal likelihood with a uniform prior), so L is a weighted sum of
 * per-image log-likelihoods.  Writes
 *   grad_B_polar device [n_tgt][K][Q] complex (plan's I/O type):
 *                dL/dRe Bhat + i dL/dIm Bhat, every entry treated as free;
 *   grad_U       device [K][H] FP64: dL/dU with U a free matrix (the
 *                eigendecomposition is not differentiated).
 * Either output may be NULL.  lse_img and grad_lse_img are device [n_img] f32.
 * Every step runs in FP64 on the plan's stored principal-ring coefficients
 * (FP32 for every precision but RADSVD_FP64): the landscape is recomputed,
 * and lse_img serves only as the exponent shift; the normalisation over
 * (b, t, m) is recomputed in FP64.  Images are processed in chunks whose
 * landscape transforms take at most 4 GiB of the scratch.
 * bwd_ws: device scratch of bwd_bytes >= align_backward_workspace(plan),
 * 256-byte aligned.  The first call with a plan the fused kernel serves also
 * writes the plan's generic operand layout on `stream` (see align_prepare; so
 * does the first align_refine_rotation call);
 * later calls on other streams must be ordered after it.  Errors: RADSVD_ERR_INVALID_ARG (NULL plan or lse
 * pointers, inv_sigma2 not finite and > 0, misaligned outputs),
 * RADSVD_ERR_WORKSPACE (scratch missing, misaligned or too small).
 */
radsvd_status align_pairs_backward(const radsvd_plan *plan, float inv_sigma2,
                                   const float *lse_img, const float *grad_lse_img,
                                   void *grad_B_polar, double *grad_U,
                                   void *bwd_ws, size_t bwd_bytes, void *stream);

/* Outputs of one job of a batched launch (RADSVD_OUT_BEST). */
typedef struct {
    float *best_score;      /* device [n_img][n_tgt] */
    int32_t *best_m;        /* device [n_img][n_tgt] */
    int32_t *best_t;        /* device [n_img][n_tgt] */
} radsvd_job_out;

/* Bytes of device scratch align_pairs_batched needs (job table and queue). */
size_t align_batched_workspace(int n_jobs);

/*
 * Many independent alignment jobs (each prepared with its own plan: its own
 * grid, rank, translations and counts) in one persistent launch with
 * RADSVD_OUT_BEST outputs: section 3.5's per-pair step for every job, the
 * tiles of all jobs drawn from one work queue.  Every plan must be Hermitian,
 * FP32, BF16 or bf16x3 (all the same precision and product count), with
 * Q in {128, 192, 256, 384, 512}.  Results are bitwise equal to one
 * align_pairs call per job.  batch_ws (device, 256-byte aligned,
 * >= align_batched_workspace(n_jobs) bytes) receives the job table and the
 * queue; the sequence contains no hipMemsetAsync and no host memory is read
 * at run time, so it can be captured in a HIP graph.  The plans' workspaces
 * and the outputs must stay valid until the launch completes; calls that
 * share one batch_ws must not overlap.  Errors: RADSVD_ERR_INVALID_ARG (NULL
 * pointers, n_jobs outside [1, 4096], mixed precisions), RADSVD_ERR_UNSUPPORTED
 * (a plan off the supported set), RADSVD_ERR_WORKSPACE.
 */
radsvd_status align_pairs_batched(const radsvd_plan *const *plans, int n_jobs,
                                  const radsvd_job_out *outs, void *batch_ws, size_t batch_bytes,
                                  void *stream);

/*
 * align_pairs_batched for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same launch and the same results, bitwise, with the job
 * table and queues in a device array the library holds for the life of the
 * process, one per GPU (256 KiB), instead of a caller workspace.  The caller
 * still passes the plans and the outputs; the call allocates no device
 * memory.  The array of the current device is used; it keeps the last call's
 * contents, and the launch rewrites every field it reads (queue positions
 * start at zero) with kernels, not memset nodes.  Calls that overlap on one
 * GPU (other streams, or another thread) share the array and race: order
 * them.  Errors: as align_pairs_batched, and RADSVD_ERR_UNSUPPORTED for
 * n_jobs > RADSVD_NOALLOC_MAX_JOBS.
 */
#define RADSVD_NOALLOC_MAX_JOBS 2048
radsvd_status align_pairs_batched_noalloc(const radsvd_plan *const *plans, int n_jobs,
                                          const radsvd_job_out *outs, void *stream);

/* Copy U (device [K][K] FP64, column h = eigenvector h) and the eigenvalues
 * (device [K] FP64, descending) of C into caller buffers (either may be NULL).
 * With a caller-supplied U_in only its H columns are defined. */
radsvd_status align_get_U(const radsvd_plan *plan, double *U_dev, double *lambda_dev,
                          void *stream);

/* Tile-order selection for align_pairs / align_pairs_batched (autotuner hook).
 * The fast Hermitian path computes tiles of 8 images x 16 targets; `band`
 * is the number of image tiles each XCD walks before the target tile
 * advances (1, 2, 4, 8 or 16; 0 = the default, 8).  It changes the order in
 * which tiles run, and so the operand reuse in each XCD's L2, never the
 * results.  Applies to later calls with this plan.  Errors:
 * RADSVD_ERR_INVALID_ARG for a NULL plan or another value. */
radsvd_status align_set_tile(radsvd_plan *plan, int band);

/* Wave layout of the fast Hermitian path (autotuner hook): the waves resident
 * on one compute unit, 4 (one four-wave workgroup per CU) or 8 (two of them,
 * or, for split bf16 with 6 products at Q = 384 and 512, one eight-wave
 * workgroup); 0 = the default, which depends on Q, the precision and the rank.
 * Both are available at Q = 128, 192 and 256; elsewhere only the default.  The
 * arithmetic, and so every result, is the same in both layouts: the choice
 * changes occupancy and prefetch depth, and applies to later align_pairs and
 * align_pairs_batched calls with this plan.  Errors: RADSVD_ERR_INVALID_ARG
 * for a NULL plan or a value other than 0, 4, 8; RADSVD_ERR_UNSUPPORTED for a
 * layout this plan does not have (the plan is unchanged). */
radsvd_status align_set_waves(radsvd_plan *plan, int waves);

void align_plan_destroy(radsvd_plan *plan);

/* ======================================================================== */
/* Volume alignment with principal volumes (paper section 4)                */
/* ======================================================================== */
/*
 * Volumes are given by their spherical-harmonic coefficients on K spherical
 * shells of radius k_r in frequency space (section 4.3): complex
 * [n][K][(L+1)^2], index l^2 + l + m for degree l = 0..L and order
 * m = -l..l, orthonormal harmonics with the Condon-Shortley phase; FP64
 * plans take complex128, FP32 plans complex64.  w_r weights the shells for
 * the integral over k^2 dk.
 *
 * A rotation tau = (gamma, beta, alpha) is R_z(alpha) R_y(beta) R_z(gamma)
 * (section 4.1); its action on coefficients is
 * B_l^m1 -> sum_m2 e^{-i m1 alpha} d^l_{m1 m2}(beta) e^{-i m2 gamma} B_l^m2 with
 * d^l(beta) = exp(-i beta J_y) (section 4.2).  The landscape is
 * X[a][b][ib][m1'][m2'] = <A_a, R_tau B_b> at tau = (2 pi m2'/M, beta[ib], 2 pi m1'/M),
 * M = 2L + 1, evaluated by the steps of section 4.9:
 *   step 1   Xt_l(m1, m2)   = sum_{h < H_C} conj([u_h^T A]_l^m1) [u_h^T B]_l^m2
 *   step 1b  Y_j(m1, m2)    = sum_l V[l][j] Xt_l(m1, m2),  j < H_D
 *   step 2   Xhat(m1, m2)   = sum_j [v_j^T d]_{m1 m2}(beta) Y_j(m1, m2)
 *   step 3   X(m1', m2')    = sum_{m1, m2} e^{-2 pi i m1 m1'/M} e^{-2 pi i m2 m2'/M} Xhat(m1, m2)
 * with the principal shells [u_h^T A]_l^m = sum_r U[r][h] sqrt(w_r) A_l^m(k_r)
 * (section 4.5).  U holds the eigenvectors of the radial kernel
 * C_rr' = sqrt(w_r w_r') Re sum_{l >= 1, m} conj(B_l^m(k_r)) B_l^m(k_r') (section 4.6)
 * and V those of the degree kernel
 * D_ll' = Re sum_r w_r sum_m conj(B_l^m(k_r)) B_l'^m(k_r), l, l' >= 1 (section 4.8),
 * both averaged over the targets, by descending eigenvalue.  At H_C = K and
 * H_D = L + 1 the landscape is the full sum over shells and degrees of
 * section 4.4.
 */
typedef struct {
    int K;                  /* shells, 2..128                                            */
    int L;                  /* largest degree: 1..64 (FP32), 1..48 (FP64); M = 2L+1       */
    int H_C;                /* radial rank, 1..K                                          */
    int H_D;                /* degree rank, 1..L+1                                        */
    int n_beta;             /* interior angles, 1..256                                    */
    const double *w;        /* host [K]: shell weights for \int g(k) k^2 dk, finite, > 0 */
    const double *beta;     /* host [n_beta]: interior angles beta (radians, finite)      */
    radsvd_precision prec;  /* RADSVD_FP64 or RADSVD_FP32 (contraction and I/O type)      */
    int real_volumes;       /* 1: the caller asserts every volume and target is real in    */
                            /* space, conj(A_l^m) = (-1)^(l+m) A_l^-m; X is then real and  */
                            /* only its real part is computed, from the orders m1 >= 0     */
                            /* (FULL has zero imaginary parts); 0: general complex         */
} radsvd_vol_problem;

typedef struct radsvd_vol_plan radsvd_vol_plan;   /* opaque host metadata */

/* Workspace bytes for vol_prepare (0 on invalid arguments, see
 * radsvd_last_error).  It holds the kernels, U and V, the principal shells of
 * every volume and target, the principal-degree Wigner tables
 * [n_beta][H_D][M][M] and the per-pair intermediates of steps 1, 1b and 2
 * (sum_l (2l+1)^2 + H_D M^2 + n_beta M^2 complex values per pair) for a block
 * of pairs (at most 1 GiB together, at least one pair; vol_align walks the
 * pairs block by block). */
size_t vol_prepare_workspace(const radsvd_vol_problem *prob, int n_vol, int n_tgt);

/* Precompute (section 4.9, steps 1-7 of the operation count): C and D from
 * the targets, their eigenvectors (FP64 Jacobi on the GPU), the principal
 * shells of volumes and targets, and the tables [v_j^T d](beta) (Wigner-d by
 * its three-term recurrence in l, in FP64).
 *   A_sh  : device [n_vol][K][(L+1)^2] complex, the volumes to align;
 *   B_sh  : device [n_tgt][K][(L+1)^2] complex, the targets (they define C, D);
 *   U_in  : device [K][H_C] FP64 or NULL (NULL: from C);
 *   V_in  : device [L+1][H_D] FP64 or NULL (NULL: from D);
 *   ws    : caller-owned device workspace of vol_prepare_workspace bytes,
 *           256-byte aligned; it must outlive every call with the plan.
 * A_sh, B_sh, U_in and V_in are read by work enqueued on `stream` only and may
 * be released once that work is done.  n_vol, n_tgt in [1, 2^20] with
 * n_vol * n_tgt <= 2^31.  Errors: RADSVD_ERR_INVALID_ARG (sizes, NULL or
 * misaligned pointers: 16 bytes for coefficients, 8 for U_in, V_in),
 * RADSVD_ERR_WORKSPACE, RADSVD_ERR_DEVICE. */
radsvd_status vol_prepare(const radsvd_vol_problem *prob, int n_vol, const void *A_sh, int n_tgt,
                          const void *B_sh, const double *U_in, const double *V_in, void *ws,
                          size_t ws_bytes, void *stream, radsvd_vol_plan **out);

/* The landscape of every (volume, target) pair over (beta, alpha, gamma).
 *   RADSVD_OUT_BEST : best_score[a][b] = max Re X (f32) and
 *                     best_idx[a][b] = {ib, m1', m2'} (int32) at the first
 *                     maximum in the order (ib, m1', m2'); a pair with a NaN
 *                     anywhere in its landscape gets NaN and {-1, -1, -1};
 *   RADSVD_OUT_FULL : X_full [n_vol][n_tgt][n_beta][M][M] complex (plan's I/O type).
 * out_flags is a non-empty combination of these two.  Pairs are processed in
 * blocks; calls with one plan on several streams share its workspace and
 * race.  Errors: RADSVD_ERR_INVALID_ARG (flags, NULL or misaligned outputs:
 * 4 bytes for BEST, 8 or 16 for FULL), RADSVD_ERR_DEVICE. */
radsvd_status vol_align(const radsvd_vol_plan *plan, int out_flags, float *best_score, int32_t *best_idx,
                        void *X_full, void *stream);

/* Copy U (device [K][K]), the eigenvalues of C ([K]), V ([L+1][L+1], column
 * j = eigenvector j) and the eigenvalues of D ([L+1]), all FP64 and
 * descending, into caller buffers (any may be NULL).  With a caller-supplied
 * U_in (V_in) only its first H_C (H_D) columns are defined and the
 * eigenvalues are NaN. */
radsvd_status vol_get_UV(const radsvd_vol_plan *plan, double *U_dev, double *lamC_dev, double *V_dev,
                         double *lamD_dev, void *stream);

void vol_plan_destroy(radsvd_vol_plan *plan);

/* Description of the last error of the calling thread ("" if none). */
const char *radsvd_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* RADSVD_H */
