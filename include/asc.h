/*
 * asc.h -- C ABI of the MI355X (gfx950) hot path of accelerated spectral
 * clustering by graph filtering of random signals (Tremblay, Puy, Borgnat,
 * Gribonval & Vandergheynst, ICASSP 2016).
 *
 * Problem statement followed (algorithm of Sec. 4.1): given an undirected
 * weighted graph W (Sec. 2.1) and a number of clusters k,
 *   1. estimate lambda_N, the largest eigenvalue of L = S - W;
 *   2. estimate lambda_k by counting eigenvalues below trial cut-offs with
 *      filtered random signals and bisecting on [0, lambda_N] (Sec. 3.2);
 *   3. build the order-p polynomial approximation of the ideal low-pass
 *      h_{lambda_k} (Eq. ideal, Sec. 2.4);
 *   4-5. filter eta = r random signals, row i of the result is node i's feature
 *      vector (Sec. 3.1);
 *   6. run k-means on the features.
 * The polynomial is a Chebyshev expansion on [0, lambda_max] with Jackson
 * damping: p(x) = sum_{j=0..p} a_j T_j(x), x = 2 lambda / lambda_max - 1,
 * a_j = g_j c_j, where c_j are the exact Chebyshev coefficients of the step
 * 1[x <= x_c] with c_0 NOT halved, and g_j the Jackson factors.  Filtering
 * evaluates Y = sum_j a_j T_j(Lt) R, Lt = (2/lambda_max) L - I, by the
 * three-term recurrence T_{j+1} = 2 Lt T_j - T_{j-1}.
 *
 * Conventions (every entry point):
 *  - Pointers are DEVICE pointers unless the name ends in _host.  All buffers
 *    are owned by the caller; the library never allocates device memory.
 *    Work that needs scratch takes (ws, ws_bytes) sized by the matching
 *    *_workspace() query; ws must be 256-byte aligned.
 *  - `stream` is a hipStream_t (NULL = the default stream).  All work is
 *    enqueued on it in order; only arguments ending in _host synchronise the
 *    stream.  Without _host outputs a call never synchronises and may be
 *    captured into a HIP graph (no memset nodes are recorded).
 *  - Signal blocks are row-major n x r with leading dimension ld (elements):
 *    row i, column c at base[i*ld + c].  float32 blocks need ld % 4 == 0 and
 *    16-byte aligned base; bfloat16 blocks ld % 8 == 0 and 16-byte alignment.
 *    r may be any value >= 1 (ragged column tails are masked).
 *  - Arguments are validated before any launch; a violation returns
 *    ASC_ERR_INVALID and launches nothing.  A HIP launch error returns
 *    ASC_ERR_HIP.  Outputs are unspecified after an error, but no write ever
 *    leaves the buffers described here.  asc_last_error() describes the most
 *    recent failure of the calling thread.
 *  - The only process-wide state is the tuning table (asc_tune_*).
 */
#ifndef ASC_H
#define ASC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ASC_ABI_VERSION 1

typedef enum {
    ASC_OK = 0,
    ASC_ERR_INVALID = 1,        /* bad argument, shape, alignment or graph       */
    ASC_ERR_WORKSPACE = 2,      /* ws NULL, misaligned or smaller than required  */
    ASC_ERR_HIP = 3,            /* a HIP runtime call or launch failed           */
    ASC_ERR_NONFINITE = 4,      /* NaN/Inf met in a checked result               */
    ASC_ERR_LMAX_TOO_SMALL = 5  /* lambda_max below lambda_N: recurrence grows   */
} asc_status;

typedef enum { ASC_F32 = 0, ASC_BF16 = 1 } asc_dtype;

/* Device-side health flags (bit set), readable with asc_read_flags. */
#define ASC_FLAG_NONFINITE 1u
#define ASC_FLAG_GROWTH 2u      /* |T_j R|_F > 1.5 |R|_F: lambda_max too small */
#define ASC_FLAG_BAD_GRAPH 4u
#define ASC_FLAG_BAD_INPUT 8u   /* a cluster label outside [0, k) was skipped */

/* Undirected weighted graph W (Sec. 2.1) in CSR, both (i,j) and (j,i) stored.
 * row_ptr[n+1] (row_ptr[0] = 0, row_ptr[n] = nnz < 2^31), col_idx[nnz]
 * strictly increasing inside a row, no self-loops; w[nnz] finite, >= 0 and
 * symmetric (W_ij = W_ji), or NULL for unit weights.  strength[n] holds
 * s_i = sum_j W_ij in float64 and is filled by asc_graph_prepare; every
 * other call reads it.  L = S - W is never formed. */
typedef struct {
    int64_t n;
    int64_t nnz;
    const int32_t *row_ptr;
    const int32_t *col_idx;
    const float *w;
    const double *strength;
} asc_graph;

int asc_abi_version(void);
/* Text of the calling thread's last error ("" if none); never NULL. */
const char *asc_last_error(void);

/* Node strengths s_i = sum_{j != i} W_ij of Sec. 2.1 (float64, summed in
 * row order).  strength[n] is written.  validate != 0 additionally checks the
 * CSR invariants above, the weights and the symmetry of W on the device
 * (needs ws of asc_graph_prepare_workspace bytes, else ws may be NULL),
 * synchronises, and returns ASC_ERR_INVALID if any check fails. */
size_t asc_graph_prepare_workspace(int64_t n, int validate);
asc_status asc_graph_prepare(const asc_graph *g, double *strength, int validate, void *ws, size_t ws_bytes,
                             void *stream);

/* Normalised Laplacian (footnote of Sec. 2.1): L_n = I - S^{-1/2} W S^{-1/2}.
 * From a prepared graph g (strengths filled) writes w_out[nnz] = w_e /
 * sqrt(s_i s_k) (float64 arithmetic, 0 where s_i or s_k is 0; unit weights
 * when g->w is NULL) and strength_out[n] = 1.  The graph {n, nnz, row_ptr,
 * col_idx, w_out, strength_out} then makes every entry point apply L_n in
 * place of L; its largest eigenvalue is at most 2, so lmax = 2 may be passed
 * without an estimate.  Gradients computed on it are with respect to w_out.
 * Outputs must not alias g's arrays. */
asc_status asc_graph_normalize(const asc_graph *g, float *w_out, double *strength_out, void *stream);

/* Step 1 of the algorithm (Sec. 4.1): an upper estimate of lambda_N.
 * Lanczos in float64 from the start vector v0[n] (not normalised; any
 * non-zero vector) for `iters` steps (stops early on breakdown), then
 * lmax = min(1.01 * largest Ritz value, 2 max_i s_i) (Gershgorin bound).
 * Writes lmax[1] (device); lmax_host (may be NULL) synchronises and copies it.
 * iters in [1, 4096]. */
size_t asc_lmax_workspace(int64_t n, int iters);
asc_status asc_lmax_estimate(const asc_graph *g, const double *v0, int iters, double *lmax,
                             double *lmax_host, void *ws, size_t ws_bytes, void *stream);

/* Step 3 (Sec. 2.4, Sec. 4.1): coefficients of the ideal low-pass h_{lambda_c}
 * (Eq. ideal) for n_cut cut-offs lambda_c[n_cut] on [0, lmax[0]]:
 * x_c = clip(2 lambda_c/lmax - 1, -1, 1), theta = acos x_c,
 * c_0 = 1 - theta/pi, c_j = -2 sin(j theta)/(j pi); jackson != 0 multiplies by
 * g_j = [(p+2-j) cos(j a) + sin(j a) cot a]/(p+2), a = pi/(p+2).
 * Writes coeffs[n_cut][p+1] (float64, computed on the device). p in [0, 100000]. */
asc_status asc_cheb_coeffs(const double *lambda_c, int n_cut, const double *lmax, int p, int jackson,
                           double *coeffs, void *stream);

/* Steps 4-5 (Sec. 3.1, Sec. 2.4): Y = sum_{j=0..p} a_j T_j(Lt) R.
 * R: n x r block of dtype sig (float32 or bfloat16), leading dim ldr.
 * Y: n x r float32, leading dim ldy, must not overlap R.  coeffs[p+1] float64
 * (device), lmax[1] float64 (device).  Signal states are stored in `sig`,
 * arithmetic and the accumulation of Y are float32.
 * ckpt (may be NULL) receives what asc_cheb_filter_bwd needs, sized by
 * asc_ckpt_bytes (256-byte aligned):
 *   ckpt_stride >= 2: the pairs (T_sc R, T_sc+1 R), sc = 0, c, 2c, ... < p;
 *   ckpt_stride == 1: every state T_0 R .. T_p R (the recurrence writes its
 *     states into this store instead of reusing two buffers; no recompute in
 *     the backward).  Its size and panel layout use the default slice width
 *     of (r, sig), independent of the tuning table, so a store sized by
 *     asc_ckpt_bytes stays valid across asc_tune_set / asc_autotune_filter.
 * The call also computes |T_0|_F and |T_p|_F and raises ASC_FLAG_GROWTH /
 * ASC_FLAG_NONFINITE in the workspace flags (asc_read_flags). */
size_t asc_filter_workspace(int64_t n, int64_t r, asc_dtype sig, int p);
size_t asc_ckpt_bytes(const asc_graph *g, int64_t r, asc_dtype sig, int p, int ckpt_stride);
asc_status asc_cheb_filter(const asc_graph *g, const double *lmax, const double *coeffs, int p,
                           const void *R, asc_dtype sig, int64_t r, int64_t ldr, float *Y, int64_t ldy,
                           void *ckpt, int ckpt_stride, void *ws, size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * asc_cheb_filter with the same arguments, checks, kernels and results, except
 * that the workspace is a static device array of ASC_NOALLOC_SCRATCH_BYTES
 * (64 MiB) inside the library instead of (ws, ws_bytes).  The array is
 * created with the library's code object on every device the library runs
 * on and held until the process ends; its device address is looked up once
 * per device, on the first call with that device current.  Nothing is
 * allocated by the call (R, Y and ckpt are still the caller's).
 * Limit: asc_filter_workspace(n, r, sig, p) <= ASC_NOALLOC_SCRATCH_BYTES,
 * e.g. n <= 130000 at r = 32 or n <= 86000 at r = 96 (float32); larger
 * sizes return ASC_ERR_WORKSPACE and launch nothing.
 * Every call on one device uses that device's one array, which keeps the
 * last call's contents (everything a call reads from it, it first writes
 * itself, the health flags included): calls ordered on one stream are safe,
 * calls that overlap in time on one device (other streams, other threads)
 * race and give wrong results.  The health flags live in the array and are
 * not readable through asc_read_flags. */
#define ASC_NOALLOC_SCRATCH_BYTES (64u << 20)
asc_status asc_cheb_filter_noalloc(const asc_graph *g, const double *lmax, const double *coeffs, int p,
                                   const void *R, asc_dtype sig, int64_t r, int64_t ldr, float *Y, int64_t ldy,
                                   void *ckpt, int ckpt_stride, void *stream);

/* Sec. 3.2: Chebyshev moments mu_j = <R, T_j(Lt) R>_F, j = 0..p (float64,
 * deterministic fixed-order reductions), from ceil(p/2) recurrence steps
 * using mu_{2j} = 2 |T_j R|^2 - mu_0 and mu_{2j+1} = 2 <T_{j+1} R, T_j R> - mu_1
 * (valid because Lt is symmetric).  The eigenvalue count below lambda_c is
 * then sum_j a_j(lambda_c) mu_j.  Writes mu[p+1]. */
size_t asc_moments_workspace(int64_t n, int64_t r, asc_dtype sig, int p);
asc_status asc_cheb_moments(const asc_graph *g, const double *lmax, int p, const void *R, asc_dtype sig,
                            int64_t r, int64_t ldr, double *mu, void *ws, size_t ws_bytes, void *stream);

/* Sec. 3.2 dichotomy on [0, lmax]: lo = 0, hi = lmax; `steps` times
 * mid = (lo+hi)/2, count = sum_j a_j(mid) mu_j, hi = mid if count >= k - 1/2
 * else lo = mid.  Writes lambda_k[1] = hi and traj[steps][2] = (mid, count).
 * Runs on the device in float64. */
asc_status asc_eigcount_dichotomy(const double *mu, int p, const double *lmax, int k, int steps, int jackson,
                                  double *lambda_k, double *traj, void *stream);

/* Step 2 of Sec. 4.1: lambda_k estimate from random signals R.  literal == 0:
 * one moment pass (asc_cheb_moments) then the dichotomy; literal != 0: one
 * filter pass per trial cut-off with count = <R, Y_mid>_F.  Same outputs as
 * asc_eigcount_dichotomy. */
size_t asc_eigcount_workspace(int64_t n, int64_t r, asc_dtype sig, int p, int steps, int literal);
asc_status asc_eigcount_lambda_k(const asc_graph *g, const double *lmax, int k, int p, int steps, int literal,
                                 const void *R, asc_dtype sig, int64_t r, int64_t ldr, double *lambda_k,
                                 double *traj, void *ws, size_t ws_bytes, void *stream);

/* Steps 2-5 of Sec. 4.1 in ONE recurrence pass: runs T_0 R .. T_p R into the
 * state store `states` (asc_ckpt_bytes(g, r, sig, p, 1) bytes), takes the
 * Chebyshev moments from the first ceil(p/2) steps (as asc_cheb_moments),
 * runs the dichotomy (as asc_eigcount_dichotomy; lambda_k[1], traj[steps][2]),
 * computes the Jackson coefficients at lambda_k (coeffs_out[p+1], may be NULL)
 * and forms Y = sum_j a_j T_j R from the stored states.  Equivalent to
 * asc_eigcount_lambda_k + asc_cheb_coeffs + asc_cheb_filter without the
 * second recurrence; `states` can feed asc_cheb_filter_bwd with
 * ckpt_stride = 1 and these coefficients.  1 <= p. */
size_t asc_lambda_k_filter_workspace(int64_t n, int64_t r, asc_dtype sig, int p);
asc_status asc_lambda_k_filter(const asc_graph *g, const double *lmax, int k, int p, int steps, const void *R,
                               asc_dtype sig, int64_t r, int64_t ldr, float *Y, int64_t ldy, double *lambda_k,
                               double *traj, double *coeffs_out, void *states, void *ws, size_t ws_bytes,
                               void *stream);

/* Row normalisation of the features (footnote of Sec. 2.1): y_i <- y_i/|y_i|,
 * zero rows stay zero.  In place on Y (n x r float32, ldy); norms[n] (may be
 * NULL) receives |y_i| (float32, accumulated in float64). */
asc_status asc_normalize_features(float *Y, int64_t n, int64_t r, int64_t ldy, float *norms, void *stream);

/* Step 6 (Sec. 4.1), k-means with Euclidean distance.
 * init_rows: C[c] = F[rows[c]] for c < k (rows[k] int32 on the device).
 * assign: labels_i = argmin_c sum_col (F_ic - C_cc)^2 evaluated in float64
 *   column by column in order (no fused multiply-add), lowest c on ties;
 *   dist2[n] (may be NULL) gets the minimum as float32.  k in [1, 1024],
 *   r <= 4096.  For 2 <= k <= 64 (and r small enough for LDS) the candidates
 *   come from float32 matrix-core distances with a rigorous error bound and
 *   only the centroids that could be nearest are evaluated by the float64
 *   definition (with dist2 NULL, not even the winner when it is the only
 *   such centroid); the results are the definition's either way.
 * update: C[c] = mean of the members of c (float64 sums in a fixed order,
 *   rounded to float32); an empty cluster keeps its previous centroid;
 *   counts[k] (int64, may be NULL) gets the member counts.
 * F: n x r float32 (ldf); C: k x r float32 contiguous. */
asc_status asc_kmeans_init_rows(const float *F, int64_t n, int64_t r, int64_t ldf, const int32_t *rows, int k,
                                float *C, void *stream);
asc_status asc_kmeans_assign(const float *F, int64_t n, int64_t r, int64_t ldf, const float *C, int k,
                             int32_t *labels, float *dist2, void *stream);
size_t asc_kmeans_update_workspace(int64_t n, int64_t r, int k);

/* k-means++ seeding (Sec. 5 uses Matlab's k-means, whose default start draws
 * each new centre with probability proportional to its squared distance to
 * the nearest centre so far).  The draw is exact integer arithmetic: with
 * D_i the least squared distance (float64, columns in order, no fused
 * multiply-add) from row i to the rows chosen so far and the weights
 * q_i = floor(2^30 (D_i / max_j D_j)), draw c >= 1 takes the least row i whose
 * prefix sum q_0 + ... + q_i exceeds floor(U_c T / 2^53), T = sum_i q_i (if
 * T = 0: row floor(U_c n / 2^53)); draw 0 takes row floor(U_0 n / 2^53).
 * U[k] (device, uint64) are the caller's random integers, taken modulo 2^53;
 * rows[k] (device, int32) receives the chosen rows, ready for
 * asc_kmeans_init_rows.  F: n x r float32 (ldf), finite.  1 <= k <= min(n,
 * 1024).  ws: asc_kmeanspp_workspace(n) bytes.  Launches 4 kernels per draw. */
size_t asc_kmeanspp_workspace(int64_t n);
asc_status asc_kmeanspp(const float *F, int64_t n, int64_t r, int64_t ldf, int k, const uint64_t *U, int32_t *rows,
                        void *ws, size_t ws_bytes, void *stream);
asc_status asc_kmeans_update(const float *F, int64_t n, int64_t r, int64_t ldf, const int32_t *labels, int k,
                             float *C, int64_t *counts, void *ws, size_t ws_bytes, void *stream);

/* k-means with replicates (Sec. 5 clusters with Matlab's k-means and 20
 * replicates): reps independent runs of Lloyd's method over the same F, run q
 * starting from C = F[rows[q*k + c]] (rows[reps*k], int32 on the device; an
 * out-of-range row reads row 0), each taking iters steps of
 * asc_kmeans_assign then asc_kmeans_update and a last assignment.  The
 * arithmetic is theirs; the centroid sums are split over as many partial
 * blocks as in asc_kmeans_update (so the results are equal bit for bit)
 * unless reps * ceil(n / 256) exceeds 16384, where fewer blocks per run take
 * the rows (the float64 sums may then round differently before the float32
 * means).  A run's inertia is sum_i min_c d(i, c), the
 * float64 distances of that assignment summed in a fixed order; the run of
 * least inertia (the lowest q on ties) gives labels[n] (int32) and, when C is
 * not NULL, its centroids C[k*r] (float32).  inertia[reps] (float64, may be
 * NULL) receives every run's inertia.  A run whose assignment changes no
 * label has reached a fixed point: its remaining steps are skipped, which
 * changes no result.  F: n x r float32 (ldf); 1 <= k <= 1024, 1 <= reps <=
 * 65535, 0 <= iters <= 10000.  ws: asc_kmeans_replicates_workspace(n, r, k,
 * reps) bytes (0 for invalid sizes). */
size_t asc_kmeans_replicates_workspace(int64_t n, int64_t r, int k, int reps);
asc_status asc_kmeans_replicates(const float *F, int64_t n, int64_t r, int64_t ldf, int k, int reps, int iters,
                                 const int32_t *rows, int32_t *labels, float *C, double *inertia, void *ws,
                                 size_t ws_bytes, void *stream);

/* ---- differentiation (extension beyond the paper) ----
 * Conventions: lambda_max is a constant; every stored CSR entry e = (i,k) is
 * its own parameter w_e, entering L as L_ik = -w_e and L_ii = sum_e w_e, so
 * the gradient of an undirected edge is the sum of its two entries.
 *
 * Gaussian-kernel similarity (Sec. 2.2 step 1): w_e = exp(-d2_e / sigma^2),
 * evaluated in float64 and stored in float32; sigma > 0.
 * asc_gauss_weights_bwd: dsigma[1] = sum_e dW_e w_e 2 d2_e / sigma^3
 * (float64, fixed-order reduction). */
asc_status asc_gauss_weights(const float *d2, int64_t nnz, double sigma, float *w, void *stream);
size_t asc_gauss_weights_bwd_workspace(int64_t nnz);
asc_status asc_gauss_weights_bwd(const float *d2, const float *w, const float *dW, int64_t nnz, double sigma,
                                 double *dsigma, void *ws, size_t ws_bytes, void *stream);

/* Loss on the row-normalised features: loss[1] = sum_i |y_i/|y_i| - t_i|^2
 * (float64) and G = dloss/dY = (g_i - f_i (f_i . g_i)) / |y_i| with
 * f_i = y_i/|y_i|, g_i = 2 (f_i - t_i); rows with |y_i| = 0 get G_i = 0.
 * Y, target, G: n x r float32 with leading dims ldy, ldt, ldg. */
size_t asc_rownorm_loss_bwd_workspace(int64_t n);
asc_status asc_rownorm_loss_bwd(const float *Y, int64_t ldy, const float *target, int64_t ldt, int64_t n, int64_t r,
                                double *loss, float *G, int64_t ldg, void *ws, size_t ws_bytes, void *stream);

/* Adjoint of asc_cheb_filter: given G = dloss/dY (n x r float32, ldg) and the
 * checkpoints that asc_cheb_filter wrote with the same ckpt_stride (and the
 * same R, coeffs and lmax; the checkpoint layouts do not depend on tuning;
 * ckpt_stride = 1: the full state store, also
 * the one of asc_lambda_k_filter), computes
 *   dW[nnz]     = dloss/dw_e per stored entry (float32; NULL to skip),
 *   dcoeffs[p+1] = <G, T_j R>_F (float64; NULL to skip)
 * by the reverse recurrence A_p = a_p G, A_j = a_j G + 2 Lt A_{j+1} - A_{j+2},
 * dw_(i,k) = (2/lmax)(M_ii - M_ik), M = A_1 T_0^T + sum_{j>=1} 2 A_{j+1} T_j^T.
 * Recurrence states are recomputed segment by segment from the checkpoints
 * (read directly from the store when ckpt_stride == 1).
 * The sparsity pattern must be symmetric (entries without a stored transpose
 * raise ASC_FLAG_BAD_GRAPH and keep dW = 0). */
size_t asc_filter_bwd_workspace(int64_t n, int64_t nnz, int64_t r, asc_dtype sig, int p, int ckpt_stride);
asc_status asc_cheb_filter_bwd(const asc_graph *g, const double *lmax, const double *coeffs, int p, const void *R,
                               asc_dtype sig, int64_t r, int64_t ldr, const void *ckpt, int ckpt_stride,
                               const float *G, int64_t ldg, float *dW, double *dcoeffs, void *ws, size_t ws_bytes,
                               void *stream);

/* ---- batches of graphs (steps 2-5 of Sec. 4.1 for many graphs at once) ----
 * The batch is one block-diagonal graph `g` (strength filled): graph q owns
 * rows node_off_host[q] .. node_off_host[q+1]-1 and its columns stay in that
 * range (node_off_host[0] = 0, node_off_host[n_graphs] = g->n; host arrays).
 * For every graph q, asc_batch_run computes the Chebyshev moments of its rows
 * of R (ceil(p/2) recurrence levels), runs the dichotomy for k_host[q] on
 * [0, lmax[q]] for `steps` steps (lambda_k[q], traj[q][steps][2] = (mid,
 * count)), then filters its rows of R at lambda_k[q] with the Jackson-damped
 * order-p polynomial into Y.  All graphs advance in lockstep (one launch per
 * recurrence level covers every graph); nothing returns to the host.
 * tile_rows (0 = default) sets the rows of a work tile; tiles never straddle
 * graphs.  With use_graph != 0 the whole sequence is captured into a HIP
 * graph on the first call (and again whenever a pointer argument changes) and
 * replayed as one launch.  The plan is host memory owned by the library
 * (free with asc_batch_destroy); the device workspace comes from the caller
 * (asc_batch_workspace bytes) and must not be shared by concurrent runs.  The
 * first run with a given ws pointer uploads the plan's tile list into it and
 * later runs (and the captured graph) read it from there: keep the contents of
 * ws between runs, or pass a different pointer.
 * 1 <= p <= 4000. */
asc_status asc_batch_create(const asc_graph *g, int n_graphs, const int64_t *node_off_host, const int32_t *k_host,
                            int64_t r, asc_dtype sig, int p, int steps, int tile_rows, void **plan);
size_t asc_batch_workspace(const void *plan);
asc_status asc_batch_info(const void *plan, int *slice_cols, int *tile_rows, int *ntiles);
asc_status asc_batch_run(void *plan, const double *lmax, const void *R, int64_t ldr, float *Y, int64_t ldy,
                         double *lambda_k, double *traj, void *ws, size_t ws_bytes, int use_graph, void *stream);
asc_status asc_batch_destroy(void *plan);

/* Autotuner of a batch plan: times asc_batch_run (eager, probe_runs runs per
 * candidate after one warm-up run) for every slice width the recurrence
 * supports up to the one covering r, crossed with tiles of 1, 2, 4, 8, 16 and
 * 32 passes of the step kernel, on the caller's batch, lmax and R, and
 * re-plans `plan` with the fastest (ties keep the earlier candidate).
 * Y, lambda_k and traj are scratch during tuning and hold the result of the
 * last candidate afterwards; rerun asc_batch_run for the tuned plan's result.
 * ws needs asc_batch_tune_workspace(plan) bytes (the largest candidate);
 * asc_batch_workspace(plan) afterwards reports the tuned plan's need, and any
 * captured graph or uploaded tile list is dropped, also on failure.  The
 * float64 moment partials are summed per tile, so lambda_k can differ in the
 * last bits between plans.  Synchronises the stream. 1 <= probe_runs <= 100.
 * Returns the chosen slice width, tile rows and mean run time in ms. */
size_t asc_batch_tune_workspace(const void *plan);
asc_status asc_batch_autotune(void *plan, const double *lmax, const void *R, int64_t ldr, float *Y, int64_t ldy,
                              double *lambda_k, double *traj, int probe_runs, void *ws, size_t ws_bytes,
                              int *best_slice_cols, int *best_tile_rows, float *best_ms, void *stream);

/* K-nearest-neighbour similarity graph (Sec. 5: a K-nearest-neighbours graph
 * with K ~ log N) from n points X (float32, row i at X[i*ldx], d coordinates,
 * 1 <= d <= 64), built in two calls that share ws (asc_knn_workspace bytes,
 * unchanged between them):
 *  asc_knn: nbr[n][k] (int32) and d2[n][k] (float64) = the k points j != i of
 *    least |x_i - x_j|^2, computed in float64 from the float32 coordinates
 *    (added in order), ascending, ties to the lower index; and row_ptr[n+1] of
 *    the union-symmetrised graph ({i, j} kept when either is a neighbour of the
 *    other).  fallback_rows (optional, device uint32): how many rows the
 *    float32 matrix-core proposals could not certify and a float64 scan over all
 *    points redid.  A point with non-finite coordinates gets nbr = -1 entries.
 *  asc_knn_graph_fill: after the caller reads nnz = row_ptr[n] and allocates,
 *    col_idx[nnz] (increasing in each row) and d2[nnz] (float32 of the float64
 *    distance) of that graph; with asc_gauss_weights it gives the similarity
 *    weights w = exp(-d2 / sigma^2) of Sec. 2.2.
 * 1 <= k <= min(32, n - 1), 2 n k < 2^31. */
size_t asc_knn_workspace(int64_t n, int d, int k);
asc_status asc_knn(const float *X, int64_t n, int d, int64_t ldx, int k, int32_t *nbr, double *d2, int32_t *row_ptr,
                   uint32_t *fallback_rows, void *ws, size_t ws_bytes, void *stream);
asc_status asc_knn_graph_fill(const float *X, int64_t n, int d, int64_t ldx, int k, const int32_t *nbr,
                              const int32_t *row_ptr, int32_t *col_idx, float *d2, void *ws, size_t ws_bytes,
                              void *stream);

/* Order of the polynomial (note on the choice of m, Sec. 2.4): for every
 * rho[q] = lambda_c / lambda_N (device, n_rho values in (0, 1)) the errors
 *   err[q][m-1] = max |h(x_i) - p_m(x_i)| over the grid x_i = cos(pi i/(G-1)),
 *                 i = 0..G-1 (G = grid), restricted to |x_i - x_c| >= 2 band,
 * m = 1..m_max, where x_c = 2 rho - 1, h = 1[x <= x_c] and p_m the order-m
 * approximation of asc_cheb_coeffs (Jackson-damped when jackson != 0), and
 *   m_star[q][d] = the least m with err[q][m-1] <= delta[d], m_max + 1 if none.
 * The printed criterion takes the sup over the whole spectrum, which the jump
 * of h makes unreachable below 1/2; band (a fraction of lambda_N, >= 0) is the
 * transition width left out.  err may be NULL (then ws holds it, sized by
 * asc_order_table_workspace).  1 <= m_max <= 8000, 2 <= grid <= 2^22. */
size_t asc_order_table_workspace(int n_rho, int m_max);
asc_status asc_order_table(const double *rho, int n_rho, const double *delta, int n_delta, double band, int m_max,
                           int grid, int jackson, double *err, int32_t *m_star, void *ws, size_t ws_bytes,
                           void *stream);

/* Stability measure for the number of clusters (Sec. 4.3, Eq. stab): for every
 * k = k_min..k_max the algorithm of Sec. 4.1 (steps 2-6) runs on J independent
 * realisations of its random signals, and
 *   gamma(k) = mean over the J(J-1)/2 pairs i < j of ARI(C_k^i, C_k^j),
 * ARI being the adjusted Rand index of Hubert & Arabie (J. Classification
 * 1985).  k* = argmax gamma is the estimated number of clusters.
 * Realisation j for k uses the first eta_host[k - k_min] columns of its pool,
 * columns [j*eta_max, (j+1)*eta_max) of R (n x J*eta_max, dtype sig, leading
 * dim ldr, i.i.d. unit-variance entries; the method's variance 1/eta_k is
 * applied inside).  Per (k, j): lambda_k by the dichotomy (`steps` steps) on
 * the eigenvalue counts of its own signals, the order-p filter at that
 * cut-off, row normalisation, and k-means (Lloyd, kmeans_iters iterations,
 * then a final assignment) from each of `reps` replicates, whose initial
 * centroids are the rows init_rows[k - k_min][j][rep][0..k-1] of the features
 * (int32 [nk][J][reps][k_max], rows in [0, n)); the replicate of least inertia
 * sum_i |f_i - mu_{label_i}|^2 (float64; lowest replicate on ties) gives C_k^j.
 * One recurrence pass keeps every state of all J*eta_max columns (the state
 * store is part of ws); the k-dependent work reads the store only.
 * Outputs (device): gamma[nk]; optional (NULL to skip): ari[nk][J(J-1)/2]
 * (pair order (0,1), (0,2), ..., (1,2), ...), labels[nk][J][n],
 * lambda_k[nk][J], traj[nk][J][steps][2] (mid, count), inertia[nk][J][reps].
 * Limits: 1 <= k_min <= k_max <= min(n, 128), at most 256 values of k;
 * 2 <= J <= 1024; J*reps <= 65535; 1 <= eta <= eta_max, J*eta_max <= 65536;
 * 1 <= p <= 8192.  asc_stability_workspace returns 0 for invalid arguments.
 * ws flags (asc_read_flags): those of the recurrence pass. */
size_t asc_stability_workspace(const asc_graph *g, int k_min, int k_max, const int *eta_host, int J, int reps, int p,
                               int steps, asc_dtype sig, int64_t eta_max);
asc_status asc_stability(const asc_graph *g, const double *lmax, int k_min, int k_max, const int *eta_host, int J,
                         int reps, int p, int steps, int kmeans_iters, const void *R, asc_dtype sig, int64_t eta_max,
                         int64_t ldr, const int32_t *init_rows, double *gamma, double *ari, int32_t *labels,
                         double *lambda_k, double *traj, double *inertia, void *ws, size_t ws_bytes, void *stream);

/* Adjusted Rand index of every pair a < b of J labellings (Sec. 4.3, after
 * Hubert & Arabie 1985): labels int32, row a at labels[a*ldl], n entries in
 * [0, k) (an entry outside is skipped and raises ASC_FLAG_BAD_INPUT in ws),
 * k <= 128, 2 <= J <= 1024.  ari[J(J-1)/2] in the order (0,1), (0,2), ...;
 * mean (optional) = their mean.  The contingency counts and the pair sums are
 * exact integers; ARI = 2(index C(n,2) - sa sb) / ((sa+sb) C(n,2) - 2 sa sb),
 * 1 where that is 0/0 (both labellings one cluster, or both all singletons). */
size_t asc_ari_workspace(void);
asc_status asc_ari_pairs(const int32_t *labels, int64_t n, int64_t ldl, int J, int k, double *ari, double *mean,
                         void *ws, size_t ws_bytes, void *stream);

/* Kernel configuration of the recurrence step, kept in a process-wide table
 * keyed by (n, nnz, r, sig); calls on a graph without an entry use the
 * default (slice width = the smallest of 8/16/32 float32 or 16/32/64 bfloat16
 * columns that covers r, variant 0).
 *   slice_cols: columns processed per pass (float32: 8, 16, 32, 64;
 *               bfloat16: 16, 32, 64, 128); 0 in asc_tune_set removes the
 *               entry.
 *   variant:    bit 0: non-temporal hints on the streamed arrays (CSR,
 *               T_{j-1}, Y) so that the gathered block stays cached; bit 1:
 *               the lanes of a row load the next 8 column indices / weights
 *               with one coalesced request and broadcast them in the row
 *               group (fewer vector-memory requests per neighbour); bit 2:
 *               each XCD processes one contiguous band of rows (L2 locality
 *               for graphs whose neighbours are close in index order); bit 3
 *               (slice widths of 8 lanes per row, i.e. 32 float32 or 64
 *               bfloat16 columns, and 2 to 4 slices): one launch per step
 *               covers every slice, reading the row's column indices and
 *               weights once (it gathers all slices' panels at once, so it
 *               pays where they fit the Infinity Cache together); with bit 3
 *               only bit 2 of the others applies.  0 <= variant <= 15.
 * Every filter step writes T_{j+1}; with float32 states Y is read and updated
 * on every other step (a_j T_j + a_{j+1} T_{j+1} together) and on the last
 * one; with bfloat16 states on every step, from T_{j+1} before its rounding.
 * asc_autotune_filter times every candidate on the caller's graph and signals
 * for probe_steps recurrence steps (Y and ws are scratch; needs ws of
 * asc_filter_workspace(n, r, sig, 1) bytes), records the fastest and returns
 * it.  It synchronises the stream.  asc_tune_save / asc_tune_load write and
 * read the table as JSON (one entry per line).  The table is guarded by a
 * mutex. */
asc_status asc_tune_set(int64_t n, int64_t nnz, int64_t r, asc_dtype sig, int slice_cols, int variant);
asc_status asc_tune_get(int64_t n, int64_t nnz, int64_t r, asc_dtype sig, int *slice_cols, int *variant);
asc_status asc_tune_save(const char *path);
asc_status asc_tune_load(const char *path);
asc_status asc_autotune_filter(const asc_graph *g, const double *lmax, const void *R, asc_dtype sig, int64_t r,
                               int64_t ldr, float *Y, int64_t ldy, int probe_steps, void *ws, size_t ws_bytes,
                               int *best_slice_cols, int *best_variant, float *best_ms_per_step, void *stream);

/* Plain device-to-device streaming copy of `bytes` (multiple of 16, 16-byte
 * aligned pointers): the reference kernel for measured copy bandwidth and for
 * calibrating memory counters. */
asc_status asc_stream_copy(const void *src, void *dst, size_t bytes, void *stream);

/* Random-row gather reference: reads row idx[e] (clamped into [0, rows)) of
 * a table of `rows` rows of 32 float32 (128 bytes, 16-byte aligned) for every
 * e < nidx, with the recurrence's access shape (8 lanes of 16 bytes per row,
 * 8 rows in flight per lane group).  Driven by a graph's column indices, its
 * time is the floor that the neighbour gathers of one 32-column recurrence
 * step set on this device.  sink[0] (device) is written only if a lane's sum
 * equals 1.2345678e7. */
asc_status asc_gather_probe(const float *table, int64_t rows, const int32_t *idx, int64_t nidx, float *sink,
                            void *stream);

/* Health flags raised by the last filter / moment pass that used ws.
 * Synchronises the stream; flags_host gets ASC_FLAG_* bits.  Returns
 * ASC_ERR_LMAX_TOO_SMALL or ASC_ERR_NONFINITE if the matching flag is set. */
asc_status asc_read_flags(const void *ws, uint32_t *flags_host, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* ASC_H */
