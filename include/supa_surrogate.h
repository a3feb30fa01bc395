/*
 * supa_surrogate.h -- C ABI of the learned surrogate's kernels (gfx950).
 *
 * The surrogate extends the paper's method: a conditional MLP maps a shower's
 * initial condition (energy, polar angle, azimuth; the conditioning variables
 * of the paper's section "Extensions") plus Gaussian noise to the mean and
 * log-variance of its coarse per-layer deposit images (the image
 * representation of the appendix "Downsampling").  It is trained with the
 * Gaussian negative log-likelihood on images made by supa_simulate, and at
 * inference showers whose predicted uncertainty is above a threshold are
 * simulated instead (fallback); per-layer energy distributions of the result
 * are compared with the simulator's by the 1-D Wasserstein distance, the
 * metric of the paper's section "Performance Analysis of Generative Models".
 *
 * Conventions (all entry points):
 *   - pointers are device pointers owned by the caller; bf16 arrays are
 *     uint16_t holding bfloat16 bit patterns; matrices are row-major with the
 *     given leading dimension (elements);
 *   - work is enqueued on `hip_stream` (hipStream_t, NULL = default stream)
 *     and nothing is synchronised; errors of a kernel launch are returned;
 *   - return SUPA_OK, SUPA_ERR_INVALID_ARG (bad sizes or NULL pointers,
 *     nothing launched) or SUPA_ERR_DEVICE; supa_surrogate_last_error() gives
 *     the message of the calling thread's last error.
 */
#ifndef SUPA_SURROGATE_H
#define SUPA_SURROGATE_H

#include <stdint.h>

#include "supa.h"

#ifdef __cplusplus
extern "C" {
#endif

enum { SUPA_EPI_F32 = 0, SUPA_EPI_BIAS_F32 = 1, SUPA_EPI_BIAS_GELU = 2, SUPA_EPI_GELU_GRAD = 3 };

/*
 * C = op(A) op(B), bf16 inputs, float32 accumulation on the matrix cores.
 *   trans_a = 0: A is M x K ([M][lda]);  1: A is stored K x M ([K][lda]).
 *   trans_b = 0: B is K x N ([K][ldb]);  1: B is stored N x K ([N][ldb]).
 * Supported (trans_a, trans_b, epilogue): (0,0,F32), (0,0,BIAS_F32),
 * (0,0,BIAS_GELU), (0,1,F32), (0,1,GELU_GRAD), (1,0,F32).  Epilogues:
 *   F32        C float [M][ldc] = acc
 *   BIAS_F32   C float = acc + bias[n]
 *   BIAS_GELU  pre bf16 [M][ldc] = acc + bias[n]; C bf16 = GELU(pre),
 *              GELU(a) = a Phi(a) (exact, erf form); pre may be NULL
 *              (inference: the pre-activation is not stored)
 *   GELU_GRAD  C bf16 = acc * GELU'(pre[m][n]) (pre read, bf16 [M][ldc])
 * M, N, K >= 1 and multiples of 8; leading dimensions multiples of 8.
 */
supa_status supa_gemm_bf16(void *hip_stream, int trans_a, int trans_b, int epilogue, int M, int N,
                           int K, const uint16_t *A, int lda, const uint16_t *B, int ldb,
                           const float *bias, void *C, int ldc, uint16_t *pre);

/*
 * C = op(A) op(B) (float [M][N], ldc = N, no epilogue) with K split into
 * `parts` ranges computed by separate workgroups (for products with few
 * output tiles and a long K, such as weight gradients over a batch), then
 * summed in order: deterministic.  scratch: caller-owned float workspace of
 * parts * M * N entries (unused when parts == 1).  Layouts as in
 * supa_gemm_bf16 (NN, NT, TN).  supa_gemm_splitk_parts gives a part count
 * that fills the device (about 1024 workgroups).
 */
supa_status supa_gemm_bf16_splitk(void *hip_stream, int trans_a, int trans_b, int M, int N, int K,
                                  const uint16_t *A, int lda, const uint16_t *B, int ldb, float *C, int parts,
                                  float *scratch);
int32_t supa_gemm_splitk_parts(int M, int N, int K);

/*
 * Gaussian NLL of targets y[b][j] = img[b][j] * y_scale / e0[b] under
 * out[b] = [mu | s_raw] (float [B][2D]), s = clamp(s_raw, -s_clamp, s_clamp):
 * adds sum over b, j of 1/2 (s + (y - mu)^2 exp(-s)) to *loss (float, device)
 * and writes dout = d mean / d out as bf16 [B][2D] (zero for clamped s).
 * s_clamp >= 0; 0 holds s at 0: a squared-error fit of the means alone.
 * mse_mean = 1: the mean half of dout is the gradient of the mean of
 * 1/2 (y - mu)^2 instead (means fitted by squared error, variances by the
 * NLL at those means); 0: the NLL gradient throughout.
 */
supa_status supa_nll_grad(void *hip_stream, int B, int D, const float *out, const float *img,
                          const float *e0, float y_scale, float s_clamp, int32_t mse_mean,
                          uint16_t *dout, float *loss);

/*
 * out[n] = sum over m < M of X[m][n] for n < N (X bf16 [M][ld]).  scratch:
 * caller-owned float workspace of supa_colsum_scratch_floats(M, N) entries
 * (row slices are summed in parallel, then per column in slice order:
 * deterministic); NULL sums each column in one thread (slow, no workspace).
 */
supa_status supa_colsum_bf16(void *hip_stream, int M, int N, const uint16_t *X, int ld, float *out,
                             float *scratch);

/* Workspace entries (float) supa_colsum_bf16 needs for M x N; 0 for empty sizes. */
int64_t supa_colsum_scratch_floats(int M, int N);

/* Adam (Kingma & Ba, 2015) step `step` (>= 1) on n float32 parameters p with
 * gradients g and moments m, v; p_bf16 (may be NULL) receives bf16(p). */
supa_status supa_adam(void *hip_stream, int64_t n, float *p, const float *g, float *m, float *v,
                      uint16_t *p_bf16, float lr, float beta1, float beta2, float eps, int step);

/* y[i] = bf16(x[i]) (round to nearest even) for i < n. */
supa_status supa_to_bf16(void *hip_stream, int64_t n, const float *x, uint16_t *y);

/*
 * Input rows x bf16 [B][ld]: e0*e_scale, polar*polar_scale, azimuth*az_scale,
 * then n_noise standard normals, zeros up to ld.  Normal pairs come from the
 * Box-Muller transform of the words of Philox4x32-10 blocks keyed by `seed`
 * and counted by (row_base + row, stream_id, 0x5eed, q) for q = 0, 4, 8, ...
 * 3 + n_noise <= ld, ld multiple of 8.
 */
supa_status supa_surrogate_features(void *hip_stream, int B, int ld, int n_noise, const float *e0,
                                    const float *polar, const float *azimuth, float e_scale,
                                    float polar_scale, float az_scale, uint32_t row_base,
                                    uint32_t stream_id, uint64_t seed, uint16_t *x);

/*
 * From out (float [B][2D], D = L * bins) per shower b: layer_e[b][l] =
 * e0[b] / y_scale * sum of mu over the bins of layer l; unc[b] =
 * sqrt(sum exp(s)) / max(sum mu, 1e-6); img (may be NULL) [B][D] =
 * e0[b] / y_scale * mu.  With 0 <= rho <= 1 the per-layer energies are
 * samples: e0/y_scale * (sum mu + sd z), sd^2 = rho (sum sigma)^2 +
 * (1 - rho) sum sigma^2 (bins of a layer correlated with coefficient rho),
 * z = Box-Muller normal from the Philox4x32-10 block keyed by `seed` and
 * counted by (row_base + b, l, 0x9a7e, 0); rho < 0: no sampling.
 */
supa_status supa_surrogate_gate(void *hip_stream, int B, int D, int L, const float *out,
                                const float *e0, float y_scale, float s_clamp, float *layer_e,
                                float *unc, float *img, float rho, uint32_t row_base, uint64_t seed);

/*
 * The final layer and the gate in one pass, without the [B][2D] output: the
 * same layer_e and unc as supa_surrogate_gate on out = h W + bias (up to the
 * order of float additions), for W given transposed.  h bf16 [B][ldh] (the
 * last hidden activations, K columns), w_t bf16 [2D][ldw] (row n = column n
 * of W, K entries), bias float [2D].  Each 128-column tile of a row (half
 * of a layer's bins, means or log-variances) is reduced in the product's
 * epilogue into partial (float scratch, caller-owned, B * (2D / 128) * 2
 * floats); a second kernel combines them per shower.  layer_cnt (float
 * [B][L], may be NULL): per layer, the number of bins whose predicted energy
 * mu * e0 / y_scale exceeds cnt_thr >= 0 (the predicted occupied cells).
 * For K = 256 the product runs transposed, each workgroup holding 256 rows
 * of h in registers and streaming W^T through LDS (one launch for the mean
 * tiles, one for the log-variance tiles); other K take 128 x 128 tiles.
 * Requirements: K a multiple of 8, L <= 64, D / L a multiple of 128, h and
 * w_t 16-byte aligned.
 */
supa_status supa_surrogate_gate_fused(void *hip_stream, int B, int K, int D, int L, const uint16_t *h, int ldh,
                                      const uint16_t *w_t, int ldw, const float *bias, const float *e0,
                                      float y_scale, float s_clamp, float *partial, float *layer_e, float *unc,
                                      float rho, uint32_t row_base, uint64_t seed, float cnt_thr,
                                      float *layer_cnt);

/*
 * Timing of supa_surrogate_gate_fused, for measurement: with on != 0, every
 * later call made while the device current at this call is current records
 * HIP events on its stream around its kernels (off: no events).  Not thread
 * safe: the events are the process's.  supa_surrogate_last_times waits for
 * the last timed call and writes up to three durations (ms): the product's
 * mean tiles, its log-variance tiles (0 when K != 256: one launch covers
 * both), the per-row gate.  SUPA_ERR_STATE if no call was timed since
 * timing was switched on.
 */
supa_status supa_surrogate_timing(int on);
supa_status supa_surrogate_last_times(float *ms, int32_t count);

/*
 * The network's forward pass in one kernel (inference): n_hidden (1..8)
 * layers of 256 units, bias + GELU, on k_in inputs (x bf16
 * [B][ldx], k_in a multiple of 16 up to 256), then with n_out > 0 a linear
 * layer of n_out outputs (a multiple of 4, at most 64) into out (float
 * [B][ldo]), else the last hidden activations into h (bf16 [B][ldh]).  The
 * activations stay in registers: a workgroup takes 256 rows through every
 * layer, each layer's weights streaming through LDS.  The same values as
 * supa_gemm_bf16 layer by layer (BIAS_GELU, then BIAS_F32) up to the order
 * of the float sums (the bias first here) and the GELU, evaluated through a
 * polynomial of Phi within 5.9e-5 |a| of the exact one (erf form) at every
 * a.  wt and bias: host arrays of device pointers, one per
 * layer (hidden layers, then the output layer): wt[l] bf16 [out][in] as
 * written by supa_mlp_fused_weights (layer 0 with permute = 0, the others
 * with permute = 1), bias[l] float [out].  x, weights and the output
 * 16-byte aligned; ldo and ldh multiples of 4.
 */
supa_status supa_mlp_forward_fused(void *hip_stream, int B, int k_in, int n_hidden, const uint16_t *x, int ldx,
                                   const uint16_t *const *wt, const float *const *bias, int n_out, float *out,
                                   int ldo, uint16_t *h, int ldh);

/*
 * A layer's weights for supa_mlp_forward_fused: wt[n][k'] = bf16(W[k][n])
 * (W float [in][out], round to nearest even), with k' = k, or with permute
 * the index the fused pass keeps the previous layer's outputs at: bits 2 and
 * 3 of k swapped (in a multiple of 32).
 */
supa_status supa_mlp_fused_weights(void *hip_stream, int in, int out, const float *W, int permute, uint16_t *wt);

/* y[c][r] = bf16(x[r][c]): float [rows][cols] to bf16 [cols][rows] (round to nearest even). */
supa_status supa_transpose_to_bf16(void *hip_stream, int rows, int cols, const float *x, uint16_t *y);

/*
 * idx[0..*count) = the indices i < n with v[i] > tau, increasing.  idx holds
 * n int32; count is one device int32; block_scratch holds ceil(n/1024) int32.
 */
supa_status supa_select_above(void *hip_stream, int n, const float *v, float tau, int32_t *idx,
                              int32_t *count, int32_t *block_scratch);

/* out_k[j] = in_k[idx[j]] for j < m, three float arrays. */
supa_status supa_gather3(void *hip_stream, int m, const int32_t *idx, const float *a,
                         const float *b, const float *c, float *oa, float *ob, float *oc);

/* dst[idx[j]][0..w) = src[j][0..w) for j < m (float rows). */
supa_status supa_scatter_rows(void *hip_stream, int m, int w, const int32_t *idx, const float *src,
                              float *dst);

/* out[r][l] = sum over q < g of x[r][l*g + q] (float), r < rows, l < L. */
supa_status supa_group_sums(void *hip_stream, int rows, int L, int g, const float *x, float *out);

/*
 * The judge of the surrogate (section "Performance Analysis of Generative
 * Models": 1-D Wasserstein distances between distributions of the same
 * quantity from two generators).
 *
 * supa_w1_equal: exact W1 between the columns of two samples of equal size,
 * w1[c] = (1/n) sum_i |a_(i)c - b_(i)c| with a_(i)c the i-th smallest value
 * of column c (the area between the two empirical distribution functions).
 * a float [n][lda], b float [n][ldb], 1 <= n <= 2^30, 1 <= cols <= 4096
 * <= lda, ldb; w1 double [cols] (device); work: device workspace of
 * supa_w1_equal_workspace_bytes(n, cols) bytes.  Each column is sorted by a
 * stable radix sort of its float bit patterns (NaNs sort past +inf, -0 before
 * +0); the sums are in double, in an order fixed by n alone (deterministic).
 */
int64_t supa_w1_equal_workspace_bytes(int64_t n, int32_t cols);
supa_status supa_w1_equal(void *hip_stream, int64_t n, int32_t cols, const float *a, int64_t lda,
                          const float *b, int64_t ldb, double *w1, void *work, int64_t work_bytes);

/* The sort of supa_w1_equal on its own: out float [cols][n] holds column c of
 * x (float [n][ld]) in increasing order; work: device workspace of
 * supa_sort_columns_workspace_bytes(n, cols) bytes. */
int64_t supa_sort_columns_workspace_bytes(int64_t n, int32_t cols);
supa_status supa_sort_columns(void *hip_stream, int64_t n, int32_t cols, const float *x, int64_t ld,
                              float *out, void *work, int64_t work_bytes);

/* Occupied cells of per-layer images: cnt[r][l] = the number of q < g with
 * img[r][l * g + q] > thr (img float [rows][L * g], cnt float [rows][L]). */
supa_status supa_occupied_counts(void *hip_stream, int64_t rows, int32_t L, int32_t g, const float *img,
                                 float thr, float *cnt);

/* Message of the calling thread's last surrogate-kernel error. */
const char *supa_surrogate_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
