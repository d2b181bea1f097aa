/*
 * modal.h - C ABI of the MI355X modal bispectrum library (libmodal.so).
 *
 * Computes the data-parallel hot path of the optimal modal bispectrum
 * estimator of Fergusson & Shellard, "Optimal Polyspectra Estimation":
 *
 *   filtered maps   M_p(x)   = sum_lm q_p(l) a_lm / sqrt(C_l) Y_lm(x)
 *   cubic modes     beta_prs = sum_x w(x) M_p M_r M_s              (p <= r <= s)
 *   linear term     lin_prs  = sum_x w(x) [V_pr M_s + V_ps M_r + V_rs M_p],
 *                   V_pr(x)  = Monte-Carlo mean of M_p M_r
 *   covariance      zeta     = <beta^hat beta^hat^T> / 6,  beta^hat = beta - lin
 *   estimator       E = alpha^T zeta^-1 beta^hat / alpha^T zeta^-1 alpha,
 *                   sigma^2 = 6 / alpha^T zeta^-1 alpha
 *
 * The maps and beta follow eq. (bbispect) of Sec. III A with the separable
 * isotropic basis R_n(l1,l2,l3) = q_p(l1) q_r(l2) q_s(l3) and v_l = 1; the
 * linear term is the "3 C a" term of eq. (bispectrumest) with the pairing
 * expectation taken from Monte-Carlo maps (Sec. II); zeta is eq. (linearterm);
 * E and sigma^2 are eqs. (modalest) and (modalvariance) evaluated through the
 * Cholesky rotation of eq. (Cholrot).
 *
 * Conventions
 * -----------
 * Grid        Gauss-Legendre rings, north to south (cos theta descending),
 *             nphi equidistant pixels per ring starting at phi = 0; pixel
 *             weight w(x) = w_GL(theta_j) * 2 pi / nphi * mask(x).
 * a_lm        m-major triangle, index(l, m) = m (2 lmax + 3 - m) / 2 + (l - m),
 *             0 <= m <= l <= lmax, complex interleaved (re, im).
 *             complex128 when prec = MODAL_F64, complex64 otherwise.
 *             Y_lm carries the Condon-Shortley phase; a_{l,-m} = (-1)^m a_lm^*.
 * maps        [S][P][ntheta][nphi], float64 (MODAL_F64) or float32.
 * modes       n = lexicographic index of (p <= r <= s); nmax = P(P+1)(P+2)/6.
 * pairs       lexicographic index of (p <= r); npairs = P(P+1)/2.
 * beta, lin,  always float64, row-major [S][nmax] / [nmax][nmax].
 * zeta, alpha
 * gradients   d/d a_lm packed as complex: (d/dRe a_lm) + i (d/dIm a_lm) for
 *             m > 0 (a_{l,-m} follows from reality), d/d a_l0 (imag 0) for m = 0.
 *
 * Memory and streams
 * ------------------
 * Every pointer argument named *_dev or documented as "device" is device
 * memory owned by the caller; *_host pointers are host memory.  The library
 * allocates no device memory: a context's constant tables live in a caller
 * buffer sized by modal_ctx_bytes.  Every compute call takes a caller-owned device workspace
 * of at least modal_workspace_size() bytes (256-byte aligned) and enqueues
 * its work asynchronously on the given HIP stream (NULL = legacy default
 * stream); none of them allocates device memory.  modal_create and
 * modal_fnl synchronise (the latter returns host scalars).
 *
 * Errors
 * ------
 * No exception or abort crosses the ABI.  Every call returns a modal_status;
 * modal_last_error() gives a message for the last failing call on a context.
 * A context is not thread-safe; concurrent calls on one context must be
 * serialised by the caller.
 */
#ifndef MODAL_H
#define MODAL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct modal_ctx modal_ctx;
typedef void* modal_stream_t;   /* a hipStream_t */

typedef enum {
  MODAL_OK = 0,
  MODAL_EINVAL = 1,        /* null pointer, non-positive size, bad enum           */
  MODAL_ESHAPE = 2,        /* grid cannot represent lmax (ntheta <= lmax, nphi <= 2 lmax, odd nphi) */
  MODAL_EDEVICE = 3,       /* a HIP call failed                                    */
  MODAL_ENOTPD = 4,        /* Cholesky met a non-positive pivot (index in last_error) */
  MODAL_ENOTREADY = 5,     /* linear-term state used before FINALIZE               */
  MODAL_EUNSUPPORTED = 6,  /* precision / option not available                     */
  MODAL_ENOSPACE = 7       /* workspace or state smaller than required             */
} modal_status;

typedef enum {
  MODAL_F64 = 0,     /* FP64 everywhere                                          */
  MODAL_F32 = 1,     /* FP32 maps, FP32 MFMA contractions, FP64 recurrence/reductions */
  MODAL_BF16X3 = 2,  /* split bf16 hi+lo on the matrix cores, FP32 accumulation:
                        synthesis 4 products, cubic contraction 3 products       */
  MODAL_F16X3 = 3    /* split fp16 hi+lo (22-bit operands, 3 products) in both
                        contractions, exact power-of-two scaling of maps and
                        weights in the cubic one, FP32 accumulation; needs
                        |q_p(l) a_lm / sqrt(C_l)| < 6.5e4 (true for whitened data) */
} modal_prec;

typedef enum {
  MODAL_OP_FILTER_MAPS = 0,
  MODAL_OP_BETA = 1,
  MODAL_OP_LINEAR_ACCUMULATE = 2,
  MODAL_OP_LINEAR_APPLY = 3,
  MODAL_OP_BETA_VJP = 4,
  MODAL_OP_COVARIANCE_SAMPLE = 5,
  MODAL_OP_COVARIANCE_FISHER = 6,
  MODAL_OP_FNL = 7,
  MODAL_OP_LINEAR_FINALIZE = 8,
  MODAL_OP_NOISE_VECTORS = 9,   /* S is the number N of beta^hat vectors            */
  MODAL_OP_FNL_LOWRANK = 10,
  MODAL_OP_ALPHA_SEPARABLE = 11,   /* S is the number T of separable terms          */
  MODAL_OP_IDEAL_COVARIANCE = 12,
  MODAL_OP_POWER_BETA = 13,
  MODAL_OP_POWER_ALPHA = 14,
  MODAL_OP_POWER_COVARIANCE = 15,
  MODAL_OP_POWER_FNL = 16,
  MODAL_OP_TRISPECTRUM = 17,
  MODAL_OP_FRAME = 18,          /* S ignored                                              */
  MODAL_OP_FNL_FRAME = 19,
  MODAL_OP_COVARIANCE_CENTERED = 20,   /* S is the number N of beta^hat vectors          */
  MODAL_OP_BETA_LOO = 21
} modal_op;

typedef enum {
  MODAL_LIN_RESET = 0,       /* zero the accumulator and its count                   */
  MODAL_LIN_ACCUMULATE = 1,  /* U_pr(x) += sum over the S maps of M_p M_r            */
  MODAL_LIN_FINALIZE = 2,    /* V = U / count (in place) and its harmonic transform Z;
                                state becomes usable                                 */
  MODAL_LIN_APPLY = 3        /* lin[S][nmax] for the given a_lm                      */
} modal_lin_mode;

typedef enum {
  MODAL_COV_SAMPLE = 0,      /* zeta = (1/(6N)) sum beta^hat beta^hat^T              */
  MODAL_COV_FISHER = 1,      /* zeta = (1/(18N)) sum J C J^T, C = diag dof variance  */
  MODAL_COV_SAMPLE_CENTERED = 2   /* zeta = (1/(6(N-1))) sum (b - mean)(b - mean)^T  */
} modal_cov_method;

typedef enum {
  MODAL_STAGE_LEGENDRE = 0,   /* harmonic synthesis over l per m                    */
  MODAL_STAGE_FFT = 1,        /* ring c2r FFT                                       */
  MODAL_STAGE_CUBIC = 2,      /* pair x mode contraction over pixels                */
  MODAL_STAGE_REDUCE = 3,     /* split-K reduction and symmetrisation               */
  MODAL_STAGE_LINACC = 4,     /* linear-term accumulation                           */
  MODAL_STAGE_ADJ_PAIR = 5,   /* adjoint pair contraction                           */
  MODAL_STAGE_ADJ_FFT = 6,    /* ring r2c FFT                                       */
  MODAL_STAGE_ADJ_LEGENDRE = 7, /* adjoint Legendre contraction (incl. lambda table) */
  MODAL_STAGE_COVARIANCE = 8, /* SYRK / Fisher assembly                             */
  MODAL_STAGE_CHOLESKY = 9,   /* factorisation, triangular solves, dots             */
  MODAL_STAGE_LINEAR = 10,    /* linear term from the harmonic pair means            */
  MODAL_NSTAGES = 11
} modal_stage;

/* ------------------------------------------------------------------------ */
/* context                                                                   */
/* ------------------------------------------------------------------------ */

/* Context tables and ownership.  A context's constant tables (quadrature, pixel weights,
 * recurrence coefficients and seeds, whitened mode functions, twiddles, index tables and,
 * optionally, the lambda table) live in ONE device buffer that the caller allocates and
 * owns: the library allocates no device memory anywhere.
 *
 * MODAL_CTX_LAMBDA_TABLE (split precisions only; ignored otherwise): also keep a table of
 * the synthesis's lambda_lm(theta_j) operand words, 16 KB per (m, 64 north rings, 64 l),
 * about 1.6 GB at lmax 1000 on 1536 rings, so that the synthesis reads lambda instead of
 * running the recurrence for each block of columns (same results, bit for bit).  Without
 * it the synthesis runs the recurrence on the fly. */
#define MODAL_CTX_LAMBDA_TABLE 1u

/* Device bytes of the tables of a context with these arguments (as modal_create takes
 * them), 256-byte granular.  Host only, no device call.  Returns 0 for arguments that
 * modal_create would reject (EINVAL, ESHAPE, EUNSUPPORTED). */
size_t modal_ctx_bytes(int lmax, int ntheta, int nphi, int P, int prec, unsigned flags);

/* Create a context for one (grid, lmax, P, precision) on the current HIP device.  Host
 * inputs are copied; the caller may free them afterwards.  Synchronous.
 *   q_host    [P][lmax+1]   separable mode functions q_p(l)
 *   cl_host   [lmax+1]      filter spectrum C_l (a_lm are divided by sqrt(C_l);
 *                           C_l <= 0 zeroes that l)
 *   mask_host [ntheta][nphi] extra pixel weight multiplying the quadrature
 *                           weight (a Galactic cut is 0/1); NULL = full sky.  The
 *                           library forms w(x) = w_GL(theta_j) 2 pi / nphi mask(x)
 *                           itself, from the Gauss-Legendre rule it computes.
 *   flags     0 or MODAL_CTX_LAMBDA_TABLE
 *   tables_dev, table_bytes  caller-owned device buffer, 256-byte aligned, of at least
 *                           modal_ctx_bytes(lmax, ntheta, nphi, P, prec, flags) bytes; it
 *                           must stay allocated and untouched until modal_destroy.
 * Errors: EINVAL (null out/q/cl/tables, lmax < 0, P < 1 or > 64, bad prec or flags, a
 * misaligned buffer), ESHAPE (ntheta <= lmax, nphi <= 2 lmax or nphi odd), ENOSPACE
 * (table_bytes too small; checked before any device call), EUNSUPPORTED, EDEVICE.
 * On failure *out is NULL. */
modal_status modal_create(modal_ctx** out, int lmax, int ntheta, int nphi, int P, int prec, unsigned flags,
                          const double* q_host, const double* cl_host, const double* mask_host, void* tables_dev,
                          size_t table_bytes);
/* Destroys the host-side context (the caller then frees its table buffer). */
void modal_destroy(modal_ctx* ctx);
const char* modal_last_error(const modal_ctx* ctx);
const char* modal_version(void);

/* Shape queries (host, no device work). */
int modal_nalm(const modal_ctx* ctx);
int modal_nmax(const modal_ctx* ctx);
int modal_npairs(const modal_ctx* ctx);

/* Contraction kernel the context dispatches for the cubic reduction:
 * 0 = vector-ALU with FP64 accumulation (FP64 contexts),
 * 1 = FP32 MFMA (32x32x2 tiles over a cover of the triples, see modal_cubic_plan),
 * 2 = split bf16/fp16 MFMA (32x32x16 tiles over the same cover). */
int modal_cubic_path(const modal_ctx* ctx);
/* Multiply-adds the cubic contraction issues per pixel and map, counting tile
 * padding and every product of a split (for roofline reports; host only). */
double modal_cubic_issued_macs(const modal_ctx* ctx);
/* Work plan of the split contraction for P modes (host only, no device; Sec. II,
 * eq. (bbispect): beta_prs is the pixel sum of the triple product, so it may be read
 * from the product of any two of the three maps against the third).  Each work item
 * is 32 blocks of 2 x 2 pairs {a0, a0+1} x {b0, b0+1} against a window of 32
 * consecutive modes; it writes the cell (pair (a, b), mode t) for a <= b < P and t in
 * [zlo, zhi).  Outputs, each optional (NULL skips it):
 *   items [2 * nitems]: first slot, window base s0 (the window is [s0, s0 + 32));
 *   slots [4 * 32 * nitems]: a0, b0, zlo, zhi (unused slots have zlo = zhi = 0);
 *   cell  [nmax]: pair index * P + mode of the cell holding beta_n, triples n in the
 *         order p <= r <= s, pair index in the order a <= b;
 *   mult: waves of a workgroup that share one item (1, 2, 4 or 8).
 * max_items bounds items and slots.  Returns the item count, or -MODAL_EINVAL for P
 * outside 1..64 or max_items too small. */
int modal_cubic_plan(int P, int max_items, int* items, int* slots, int* cell, int* mult);

/* The context's quadrature: x_host[ntheta] = cos theta_j (descending),
 * w_host[ntheta] = Gauss-Legendre weights (sum 2).  Either may be NULL. */
modal_status modal_grid(const modal_ctx* ctx, double* x_host, double* w_host);

/* Bytes of workspace an operation needs for S maps (N for covariance). */
modal_status modal_workspace_size(const modal_ctx* ctx, int op, int S, size_t* bytes);
/* Bytes of the linear-term state: the pair accumulator (one pixel plane per
 * pair, [npairs][ntheta][nphi] real, at offset 0; after FINALIZE the pair means
 * V), then, 256-byte aligned, Z[npairs][nalm] complex written by FINALIZE. */
size_t modal_linear_state_size(const modal_ctx* ctx);

/* ------------------------------------------------------------------------ */
/* hot path                                                                  */
/* ------------------------------------------------------------------------ */

/* Filtered maps M_p for S maps (Sec. III A, separable form of eq. bbispect).
 *   alm_dev  [S][nalm] complex (see dtype above), device
 *   maps_dev [S][P][ntheta][nphi] real, device
 * Errors: EINVAL, ENOSPACE (ws_bytes too small), EDEVICE. */
modal_status modal_filter_maps(modal_ctx* ctx, const void* alm_dev, int S, void* maps_dev,
                               void* ws_dev, size_t ws_bytes, modal_stream_t stream);

/* Monte-Carlo linear term (Sec. II: linear term from Gaussian simulations;
 * eq. bispectrumest: the three pairings of "3 C a").
 *   RESET      state is zeroed (alm may be NULL, S ignored)
 *   ACCUMULATE U_pr += sum over S maps of M_p M_r
 *   FINALIZE   V = U / total count, then Z_ab,lm = c_m sum_x w V_ab lambda_lm
 *              e^{-i m phi} (c_m = 2 - delta_m0) for every pair; afterwards the
 *              state may be passed to modal_beta / APPLY / modal_beta_vjp.
 *              Workspace: modal_workspace_size(MODAL_OP_LINEAR_FINALIZE, 1).
 *   The linear term is evaluated from Z as sum_l qw_t(l) sum_m Re(a_lm conj Z_ab,lm),
 *   an exact rearrangement of sum_x w V_ab M_t (the maps are finite harmonic sums).
 *   APPLY      lin_dev [S][nmax] float64 = lin(a) for the S maps
 * state_dev has modal_linear_state_size() bytes; the count lives in the
 * context, so a state is tied to the context that built it.
 * Errors: EINVAL, ENOTREADY (APPLY before FINALIZE, FINALIZE with count 0),
 * ENOSPACE, EDEVICE. */
/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): modal_beta with its
 * workspace taken from a fixed device array inside the library instead of a
 * caller buffer.  The array holds MODAL_NOALLOC_SCRATCH_BYTES (64 MiB) on every
 * GPU the library runs on, until the process ends; the call allocates nothing.
 * Arguments, results and errors are those of modal_beta (same kernels, same
 * results), plus ENOSPACE when modal_workspace_size(MODAL_OP_BETA, S) exceeds
 * the array (small shapes only: for instance lmax 150 on 199 x 400 rings, P 13,
 * S 3 needs about 25 MB; full-resolution shapes need modal_beta).  Nothing in
 * the array has to start at zero.  All calls on one GPU share its array: calls
 * that overlap on one GPU (two streams, two host threads, graphs replayed
 * concurrently) race and must be serialised by the caller. */
#define MODAL_NOALLOC_SCRATCH_BYTES (64u << 20)
modal_status modal_beta_noalloc(modal_ctx* ctx, const void* alm_dev, int S, const void* state_dev,
                                double* beta_dev, modal_stream_t stream);

modal_status modal_linear_term(modal_ctx* ctx, int mode, const void* alm_dev, int S, void* state_dev,
                               double* lin_dev, void* ws_dev, size_t ws_bytes, modal_stream_t stream);

/* beta^hat_n = beta_n - lin_n for S maps (eq. bbispect); state_dev NULL gives
 * beta_n without the linear term.  beta_dev [S][nmax] float64.
 * Errors: EINVAL, ENOTREADY (state not finalised), ENOSPACE, EDEVICE. */
modal_status modal_beta(modal_ctx* ctx, const void* alm_dev, int S, const void* state_dev,
                        double* beta_dev, void* ws_dev, size_t ws_bytes, modal_stream_t stream);

/* beta^hat of skies that are themselves among the Monte-Carlo skies of the linear
 * term, with each sky's own maps left out of the pair means it is corrected with
 * (Sec. II: linear term from simulations; the self-inclusion bias is O(1/N)):
 *   V^(-i) = (N V - M^i_p M^i_r) / (N - 1),  beta^hat^(-i) = beta_i - lin(a_i; V^(-i))
 *          = ((N + 2) beta_i - N lin(a_i; V)) / (N - 1),
 * since the three pairings of M^i_p M^i_r M^i_s sum to 3 beta_i.  N is the number of
 * skies accumulated into the state.  Every one of the S skies must have been
 * accumulated exactly once, with these a_lm (the library cannot check this; for other
 * skies the result is not a leave-one-out term).  Arguments as modal_beta; state_dev
 * must be finalised.  Workspace: modal_workspace_size(MODAL_OP_BETA_LOO, S).
 * Errors: EINVAL (null state), ENOTREADY (state not finalised, or N < 2), ENOSPACE,
 * EDEVICE. */
modal_status modal_beta_loo(modal_ctx* ctx, const void* alm_dev, int S, const void* state_dev,
                            double* beta_dev, void* ws_dev, size_t ws_bytes, modal_stream_t stream);

/* Vector-Jacobian product: grad[s] = sum_n cot[s][n] d beta^hat_n / d a_lm
 * (V held fixed), packed as documented above.
 *   cot_dev [S][nmax] float64, grad_dev [S][nalm] complex (alm dtype).
 * Errors: EINVAL, ENOTREADY, ENOSPACE, EDEVICE. */
modal_status modal_beta_vjp(modal_ctx* ctx, const void* alm_dev, int S, const void* state_dev,
                            const double* cot_dev, void* grad_dev, void* ws_dev, size_t ws_bytes,
                            modal_stream_t stream);

/* Modal covariance zeta [nmax][nmax] float64 (eq. linearterm).
 *   SAMPLE: beta_dev [N][nmax] beta^hat vectors; zeta = sum b b^T / (6 N) (no mean
 *           subtracted: beta^hat has zero mean for Gaussian skies).  No workspace.
 *   SAMPLE_CENTERED: zeta = sum (b - m)(b - m)^T / (6 (N - 1)), m the mean of the N
 *           rows (the unbiased estimate when the mean is not known); N >= 2.
 *           Workspace: modal_workspace_size(MODAL_OP_COVARIANCE_CENTERED, N).
 *   FISHER: alm_dev [N][nalm] maps, state_dev finalised, cvar_host [lmax+1]
 *           the variance C_l of a_lm used as the metric (C_l for a_l0,
 *           C_l / 2 for Re and Im of a_lm, m > 0);
 *           zeta = sum_i J_i C J_i^T / (18 N), J = d beta^hat / d a.
 * Errors: EINVAL, ENOTREADY, ENOSPACE, EDEVICE. */
modal_status modal_covariance(modal_ctx* ctx, int method, const double* beta_dev, const void* alm_dev,
                              const void* state_dev, const double* cvar_host, int N, double* zeta_dev,
                              void* ws_dev, size_t ws_bytes, modal_stream_t stream);

/* Estimator (eqs. Cholrot, modalest, modalvariance): factor zeta = L L^T in
 * FP64, y = L^-1 alpha, z_s = L^-1 beta_s, E_s = y.z_s / y.y, sigma^2 = 6 / y.y.
 *   zeta_dev [nmax][nmax] (read only), alpha_dev [nmax], beta_dev [S][nmax]
 *   E_host [S], sigma2_host [1] (host); L_dev [nmax][nmax] or NULL (lower
 *   triangle of L written row-major, upper triangle zeroed).
 * Synchronises the stream.  Errors: EINVAL, ENOTPD (pivot index in
 * last_error), ENOSPACE, EDEVICE. */
modal_status modal_fnl(modal_ctx* ctx, const double* zeta_dev, const double* alpha_dev,
                       const double* beta_dev, int S, double* E_host, double* sigma2_host,
                       double* L_dev, void* ws_dev, size_t ws_bytes, modal_stream_t stream);

/* Low-rank covariance (Sec. III B, eq. ic_bivector): zeta ~= I + sum_j b_j b_j^T
 * in a frame where the ideal covariance is the identity (for instance after
 * modal_whiten with the Cholesky factor of the ideal covariance).  k = 1 is the
 * paper's noise/mask "bivector"; k > 1 the principal-component form it announces.
 *
 * modal_noise_vectors: the k leading eigenpairs (mu_j, v_j) of the sample
 * covariance sum_i beta_i beta_i^T / (6N) of the rows of beta_dev [N][nmax]
 * float64, and b_j = sqrt(max(mu_j - 1, 0)) v_j (the best rank-k fit of zeta - I),
 * each signed so that its entry of largest magnitude is positive.  Computed from
 * the N x N Gram matrix by `iters` rounds of subspace iteration on a block of
 * min(k + 4, 16, N, nmax) columns and a final Rayleigh-Ritz step; the error of the
 * subspace shrinks like (mu_{kb+1} / mu_k)^iters.
 *   bt_dev [k][nmax] float64 (written), mu_host [k] (written; the call
 *   synchronises the stream).  1 <= k <= min(16, N, nmax), iters >= 1.
 *   Workspace: modal_workspace_size(MODAL_OP_NOISE_VECTORS, N) (holds N^2 doubles).
 * Errors: EINVAL, ENOSPACE, EDEVICE. */
modal_status modal_noise_vectors(modal_ctx* ctx, const double* beta_dev, int N, int k, int iters, double* bt_dev,
                                 double* mu_host, void* ws_dev, size_t ws_bytes, modal_stream_t stream);

/* Estimator of eqs. (modalest, modalvariance) with zeta = I + sum_j b_j b_j^T for
 * the k rows of bt_dev [k][nmax] (0 <= k <= 16; k = 0 is zeta = I), through the
 * Woodbury identity (eq. ic_bivectorinv for k = 1):
 *   alpha_dev [nmax], beta_dev [S][nmax] float64; E_host [S], sigma2_host [1].
 * Synchronises the stream.  Workspace: modal_workspace_size(MODAL_OP_FNL_LOWRANK, S).
 * Errors: EINVAL (also alpha^T zeta^-1 alpha <= 0), ENOSPACE, EDEVICE. */
modal_status modal_fnl_lowrank(modal_ctx* ctx, const double* bt_dev, int k, const double* alpha_dev,
                               const double* beta_dev, int S, double* E_host, double* sigma2_host, void* ws_dev,
                               size_t ws_bytes, modal_stream_t stream);

/* Rotation into the orthonormal frame of zeta = I + b b^T (Sec. III B, eq. Cholrot):
 * y_r = lambda~^-1 x_r for the closed-form lower Cholesky factor lambda~ of
 * I + b b^T, for R rows x_dev [R][nmax] -> y_dev [R][nmax] (float64; y may equal
 * x).  In that frame E = alpha'.beta' / |alpha'|^2.  No workspace; asynchronous.
 * Errors: EINVAL, EDEVICE. */
modal_status modal_bivector_rotate(modal_ctx* ctx, const double* b_dev, const double* x_dev, int R, double* y_dev,
                                   modal_stream_t stream);

/* y_r = L^-1 x_r for R rows x_dev [R][nmax] -> y_dev [R][nmax] (float64, y may
 * equal x), L the lower Cholesky factor returned by modal_fnl (only the lower
 * triangle is read): the rotation of eq. (Cholrot), e.g. into the frame where a
 * reference covariance is the identity.  No workspace; asynchronous.
 * Errors: EINVAL, EDEVICE. */
modal_status modal_whiten(modal_ctx* ctx, const double* L_dev, const double* x_dev, int R, double* y_dev,
                          modal_stream_t stream);

/* Truncated orthonormal frame of the modes (Sec. II: an orthonormal basis truncated to
 * the modes that span the space of interest; eq. Cholrot: re-orthonormalisation by a
 * Cholesky factor).  The separable q-product modes are linearly dependent in floating
 * point once P is large (their ideal covariance zeta0 is singular to FP64 at lmax 1000,
 * P 40), so the factor is pivoted and truncated:
 *   Pi^T zeta0 Pi ~= L L^T,  L = [L11; L21] (nmax x k),
 * taking at each step the mode with the largest remaining diagonal and stopping once that
 * diagonal is <= tol * max(diag zeta0).  The k kept modes perm[0..k) span, to that
 * tolerance, what all nmax modes span; T = L11^-1 [I_k 0] Pi^T is orthonormal under zeta0.
 *
 * modal_frame: zeta0_dev [nmax][nmax] symmetric positive semi-definite (read only; e.g.
 *   modal_ideal_covariance), 0 <= tol < 1; writes *k_host, perm_dev [nmax] int (first k
 *   used) and L11_dev [nmax * nmax] double (the k x k lower triangle, row-major with
 *   leading dimension k, upper part zeroed).  FP64, one column per step (left-looking).
 *   Synchronises.  Workspace: modal_workspace_size(MODAL_OP_FRAME, 0) (holds nmax^2 doubles).
 * modal_frame_rotate: y_dev [R][k] = L11^-1 x[perm] for rows x_dev [R][nmax] (the frame
 *   coordinates, eq. Cholrot on the kept modes); asynchronous, no workspace.
 * modal_fnl_frame: E_s, sigma^2 of eqs. (modalest, modalvariance) on the k kept modes, with
 *   zeta_dev [nmax][nmax] any covariance of the modes (zeta0 itself gives E = a'.b' / |a'|^2
 *   in the frame); alpha_dev [nmax], beta_dev [S][nmax].  Synchronises.
 *   Workspace: modal_workspace_size(MODAL_OP_FNL_FRAME, S).
 * Errors: EINVAL (null pointer, tol outside [0, 1), k outside 1..nmax), ENOTPD (fnl_frame:
 *   zeta restricted to the kept modes not positive definite), ENOSPACE, EDEVICE. */
modal_status modal_frame(modal_ctx* ctx, const double* zeta0_dev, double tol, int* k_host, int* perm_dev,
                         double* L11_dev, void* ws_dev, size_t ws_bytes, modal_stream_t stream);
modal_status modal_frame_rotate(modal_ctx* ctx, int k, const int* perm_dev, const double* L11_dev,
                                const double* x_dev, int R, double* y_dev, modal_stream_t stream);
modal_status modal_fnl_frame(modal_ctx* ctx, const double* zeta_dev, int k, const int* perm_dev,
                             const double* alpha_dev, const double* beta_dev, int S, double* E_host,
                             double* sigma2_host, void* ws_dev, size_t ws_bytes, modal_stream_t stream);

/* Theory mode coefficients alpha_n (eq. abispect, v_l = 1) of a separable reduced
 * bispectrum b_{l1 l2 l3} = sum_t X_t(l1) Y_t(l2) Z_t(l3), symmetrised over the
 * order of (l1, l2, l3), whitened by the context's C_l (terms with C_l = 0 drop):
 *   alpha_prs = sum_{l1 l2 l3} h^2_{l1 l2 l3} bbar / sqrt(C_l1 C_l2 C_l3) q_p(l1) q_r(l2) q_s(l3),
 * evaluated exactly through the Legendre triple integral on a Gauss-Legendre rule in
 * mu with (3 lmax + 2) / 2 nodes.
 *   terms_host [T][3][lmax+1] (host, X_t, Y_t, Z_t), 1 <= T <= 64; alpha_dev [nmax] float64.
 * Synchronises the stream.  Workspace: modal_workspace_size(MODAL_OP_ALPHA_SEPARABLE, T).
 * Errors: EINVAL, ENOSPACE, EDEVICE. */
modal_status modal_alpha_separable(modal_ctx* ctx, const double* terms_host, int T, double* alpha_dev, void* ws_dev,
                                   size_t ws_bytes, modal_stream_t stream);

/* Ideal modal covariance: zeta0 = <beta beta^T> / 6 for full-sky isotropic Gaussian skies
 * whose whitened coefficients have <|a~_lm|^2> = c_l (eq. cbispect with a diagonal
 * covariance), i.e. the Gram matrix of the separable modes under h^2 c c c:
 *   zeta0_nn' = (1/6) sum_{l1 l2 l3} h^2 c_l1 c_l2 c_l3 sum_{sigma in S3} Q_n(l) Q_n'(sigma l),
 * Q_prs(l) = q_p(l1) q_r(l2) q_s(l3).  Its Cholesky factor orthonormalises the basis
 * (Sec. II) and gives the frame where the ideal covariance is the identity
 * (modal_fnl + modal_whiten).  c_host [lmax+1] (host) or NULL: c_l = 1 where C_l > 0.
 *   zeta_dev [nmax][nmax] float64.  Synchronises the stream.
 *   Workspace: modal_workspace_size(MODAL_OP_IDEAL_COVARIANCE, 0).
 * Errors: EINVAL, ENOSPACE, EDEVICE. */
modal_status modal_ideal_covariance(modal_ctx* ctx, const double* c_host, double* zeta_dev, void* ws_dev,
                                    size_t ws_bytes, modal_stream_t stream);

/* Modal power-spectrum estimator (Sec. IV, the quadratic analogue of the bispectrum
 * one).
 *
 * modal_power_beta: for every pair p <= r (npairs = P (P + 1) / 2, ordered as for the
 * linear-term state) beta_pr = sum_x w(x) (M_p M_r - V_pr) for S maps, with the
 * filtered maps of modal_filter_maps and V the Monte-Carlo pair means of a finalised
 * linear-term state (state_dev NULL: no subtraction).  The mean term is read from
 * the state's harmonic transform (sum_x w V_pr = sqrt(4 pi) Re Z_pr,00), not from V.
 *   beta_dev [S][npairs] float64.  Workspace: modal_workspace_size(MODAL_OP_POWER_BETA, S).
 *   Errors: EINVAL, ENOTREADY, ENOSPACE, EUNSUPPORTED, EDEVICE.
 * The estimator's modes are the paper's isotropic R_n(l) = q_0(l) q_n(l), n < P: the
 * pairs (0, n), i.e. the first P entries of each row of beta (on the full sky the other
 * pairs are linearly dependent on these and on each other).
 * modal_power_alpha: alpha_n = sum_l (2l+1) q_0(l) q_n(l) dcl(l) / C_l for a spectral
 *   deviation dcl_host [lmax+1] (host) = C~_l - C_l; alpha_dev [P].  Synchronises.
 *   Workspace: modal_workspace_size(MODAL_OP_POWER_ALPHA, 0).
 * modal_power_ideal_covariance: zeta = <beta beta^T> / 2 on those modes for full-sky
 *   Gaussian skies with whitened spectrum c_l (c_host [lmax+1] or NULL: 1 where C_l > 0):
 *   zeta_nn' = sum_l (2l+1) c_l^2 R_n(l) R_n'(l); zeta_dev [P][P].  Synchronises.
 *   Workspace: modal_workspace_size(MODAL_OP_POWER_COVARIANCE, 0).
 * modal_power_fnl: E_s = alpha^T zeta^-1 beta_s / alpha^T zeta^-1 alpha and
 *   sigma^2 = 2 / alpha^T zeta^-1 alpha by FP64 Cholesky (as modal_fnl) on the P modes;
 *   beta_dev is the [S][npairs] output of modal_power_beta (its first P columns are used).
 *   Synchronises.  Workspace: modal_workspace_size(MODAL_OP_POWER_FNL, S).
 *   Errors: EINVAL, ENOTPD, ENOSPACE, EDEVICE. */
modal_status modal_power_beta(modal_ctx* ctx, const void* alm_dev, int S, const void* state_dev, double* beta_dev,
                              void* ws_dev, size_t ws_bytes, modal_stream_t stream);
modal_status modal_power_alpha(modal_ctx* ctx, const double* dcl_host, double* alpha_dev, void* ws_dev,
                               size_t ws_bytes, modal_stream_t stream);
modal_status modal_power_ideal_covariance(modal_ctx* ctx, const double* c_host, double* zeta_dev, void* ws_dev,
                                          size_t ws_bytes, modal_stream_t stream);
modal_status modal_power_fnl(modal_ctx* ctx, const double* zeta_dev, const double* alpha_dev, const double* beta_dev,
                             int S, double* E_host, double* sigma2_host, void* ws_dev, size_t ws_bytes,
                             modal_stream_t stream);

/* Modal trispectrum estimator (Sec. IV, the diagonal-free trispectrum): for the
 * separable modes q_p q_r q_s q_u, p <= r <= s <= u (nquad = P(P+1)(P+2)(P+3)/24,
 * lexicographic; modal_nquad),
 *   tau_prsu = sum_x w [M_p M_r M_s M_u - (6 pairs) V_ab M_c M_d + (3 pairings) V_ab V_cd]
 * with V the Monte-Carlo pair means of a finalised linear-term state (state_dev NULL:
 * V = 0, the plain quartic sums).  Computed as the pairs x pairs symmetric update
 * K = sum_x w A A^T - 6 sum_x w V V^T, A_ab = M_a M_b - 3 V_ab, tau = the mean of K over the
 * three pairings; split-bf16 matrix cores for MODAL_BF16X3 and MODAL_F16X3 contexts,
 * FP64 for MODAL_F64 (a reference path without pixel chunking).  MODAL_F32 contexts get
 * EUNSUPPORTED: there is no FP32 update, and a split one would not keep the FP32 bound.
 *   tau_dev [S][nquad] float64.  Workspace: modal_workspace_size(MODAL_OP_TRISPECTRUM, S);
 * for float contexts it includes pixel-block-major copies of the pair means (npairs x
 * npix floats, rounded up to 32-pixel blocks; with a state) and of the S skies' maps,
 * made at each call.
 * Errors: EINVAL, ENOTREADY, ENOSPACE, EUNSUPPORTED (MODAL_F32), EDEVICE. */
modal_status modal_trispectrum(modal_ctx* ctx, const void* alm_dev, int S, const void* state_dev, double* tau_dev,
                               void* ws_dev, size_t ws_bytes, modal_stream_t stream);
int modal_nquad(const modal_ctx* ctx);

/* Autotuner: times modal_beta on the caller's inputs (same arguments and
 * workspace as modal_beta; one warm-up and two timed calls per candidate) for
 * each candidate launch configuration - pixels per split-K chunk of the
 * matrix-core contraction (8K, 16K, 32K or 64K for the split precisions, 2K or
 * 4K for FP32; rounded to whole staged steps and to a multiple of 8 chunks) and,
 * for the LDS ping-pong ring FFT only, rings per FFT workgroup (4, 2, 1 as LDS
 * allows; the register-pass FFT of float maps has one shape) - and keeps the
 * fastest in the context (reported through chunk_px / fft_rings when not NULL).
 * A workspace sized by modal_workspace_size stays valid for every candidate.
 * Synchronises the stream.  Errors: as modal_beta. */
modal_status modal_autotune(modal_ctx* ctx, const void* alm_dev, int S, const void* state_dev, double* beta_dev,
                            void* ws_dev, size_t ws_bytes, modal_stream_t stream, int* chunk_px, int* fft_rings);

/* ------------------------------------------------------------------------ */
/* captured launches                                                         */
/* ------------------------------------------------------------------------ */

typedef struct modal_graph modal_graph;

/* Capture a sequence of modal_beta calls into one HIP graph (batching: many
 * Monte-Carlo maps, possibly of different l_max, replayed with one launch).  Call i uses ctxs[i], alms[i] ([S[i]][nalm_i] device),
 * states[i] (finalised or NULL), betas[i] ([S[i]][nmax_i] device) and its own
 * workspace ws[i] of ws_bytes[i] bytes; contexts must live on one device.
 * Arguments are validated exactly as modal_beta does; the pointers are baked
 * into the graph and must stay valid while it is used.  Capture runs on a
 * private stream (nothing executes); replay with modal_graph_launch on any
 * stream of that device.  Profiling is suspended during capture.
 * Errors: EINVAL, ENOTREADY, ENOSPACE, EDEVICE (capture/instantiate failed); the failing
 * call's context records the error, prefixed with "graph call <i>: ". */
modal_status modal_beta_graph_create(int n, modal_ctx* const* ctxs, const void* const* alms, const int* S,
                                     const void* const* states, double* const* betas, void* const* ws,
                                     const size_t* ws_bytes, modal_graph** out);
modal_status modal_graph_launch(modal_graph* g, modal_stream_t stream);
void modal_graph_destroy(modal_graph* g);

/* ------------------------------------------------------------------------ */
/* instrumentation                                                           */
/* ------------------------------------------------------------------------ */

/* Per-stage GPU timing: when enabled, every stage of every call is bracketed
 * by HIP events recorded on the call's stream (a few microseconds per stage).
 * modal_profile_read synchronises on the recorded events and returns, per
 * stage, the summed elapsed milliseconds and the number of launches timed;
 * reset != 0 clears the totals.  Arrays have MODAL_NSTAGES entries; either
 * may be NULL.  Errors: EINVAL, EDEVICE. */
modal_status modal_profile_enable(modal_ctx* ctx, int enable);
modal_status modal_profile_read(modal_ctx* ctx, double* ms_host, long long* count_host, int reset);

#ifdef __cplusplus
}
#endif
#endif /* MODAL_H */
