// supa_surrogate_api.hip -- C ABI of include/supa_surrogate.h: argument
// checks on the host, then the kernels of supa_mlp.hip on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "../../include/supa_surrogate.h"
#include "supa_device.hpp"
#include "supa_mlp.hpp"

namespace supa {
hipError_t launch_gemm(int ta, int tb, int epi, const GemmArgs &g, hipStream_t s);
hipError_t launch_nll(int B, int D, const float *out, const float *img, const float *e0,
                      float y_scale, float s_clamp, int mse_mean, uint16_t *dout, float *loss,
                      hipStream_t s);
hipError_t launch_colsum(int M, int N, const uint16_t *X, int ld, float *out, float *scratch, hipStream_t s);
int64_t colsum_scratch_floats(int M, int N);
hipError_t launch_sum_parts(int64_t n, int parts, const float *part, float *out, hipStream_t s);
hipError_t launch_adam(int64_t n, float *p, const float *g, float *m, float *v, uint16_t *pb,
                       float lr, float b1, float b2, float eps, int step, hipStream_t s);
hipError_t launch_to_bf16(int64_t n, const float *x, uint16_t *y, hipStream_t s);
hipError_t launch_features(int B, int ld, int n_noise, const float *e0, const float *polar,
                           const float *az, float e_scale, float polar_scale, float az_scale,
                           uint32_t row_base, uint32_t stream, uint64_t seed, uint16_t *x,
                           hipStream_t s);
hipError_t launch_gate(int B, int D, int L, const float *out, const float *e0, float y_scale,
                       float s_clamp, float *layer_e, float *unc, float *img, float rho,
                       uint32_t row_base, uint64_t seed, hipStream_t s);
hipError_t launch_select(int n, const float *v, float tau, int32_t *idx, int32_t *count,
                         int32_t *block_scratch, hipStream_t s);
hipError_t launch_gather3(int m, const int32_t *idx, const float *a, const float *b, const float *c,
                          float *oa, float *ob, float *oc, hipStream_t s);
hipError_t launch_scatter_rows(int m, int w, const int32_t *idx, const float *src, float *dst,
                               hipStream_t s);
hipError_t launch_group_sums(int rows, int L, int g, const float *x, float *out, hipStream_t s);
hipError_t launch_gate_fused(int B, int K, int D, int L, const uint16_t *h, int ldh, const uint16_t *wt, int ldw,
                             const float *bias, const float *e0, float y_scale, float s_clamp, float *partial,
                             float *layer_e, float *unc, float rho, uint32_t row_base, uint64_t seed,
                             float cnt_thr, float *layer_cnt, const hipEvent_t *ev, hipStream_t s);
hipError_t launch_transpose_bf16(int rows, int cols, const float *x, uint16_t *y, hipStream_t s);
hipError_t launch_mlp_fused(const MlpFusedArgs &a, hipStream_t s);
hipError_t launch_mlp_weights(int in, int out, const float *W, int permute, uint16_t *wt, hipStream_t s);
size_t sort_work_bytes(int64_t n, int cols);
hipError_t launch_sort_columns(const float *x, int64_t ld, int64_t n, int cols, void *work, uint32_t **sorted,
                               hipStream_t s);
hipError_t launch_w1_sorted(const uint32_t *ka, const uint32_t *kb, int64_t n, int cols, double *part, double *w1,
                            hipStream_t s);
int64_t w1_sorted_partial_words(int64_t n, int cols);
hipError_t launch_keys_to_floats(const uint32_t *k, int64_t total, float *out, hipStream_t s);
hipError_t launch_occupied_counts(int64_t rows, int L, int g, const float *img, float thr, float *cnt,
                                  hipStream_t s);
}  // namespace supa

static thread_local std::string t_err;

static supa_status bad(const char *msg) {
    t_err = msg;
    return SUPA_ERR_INVALID_ARG;
}

static supa_status dev(hipError_t e, const char *what) {
    if (e == hipSuccess) return SUPA_OK;
    t_err = std::string(what) + ": " + hipGetErrorString(e);
    return SUPA_ERR_DEVICE;
}

extern "C" const char *supa_surrogate_last_error(void) { return t_err.c_str(); }

// Timing of supa_surrogate_gate_fused: four events on the device that was
// current when timing was switched on.
static struct {
    bool on = false, recorded = false;
    int device = -1;
    hipEvent_t ev[4] = {};
} g_gate_timing;

extern "C" supa_status supa_surrogate_timing(int on) {
    if (on && !g_gate_timing.ev[0]) {
        if (hipError_t e = hipGetDevice(&g_gate_timing.device); e != hipSuccess) return dev(e, "timing");
        for (hipEvent_t &e : g_gate_timing.ev)
            if (hipError_t r = hipEventCreate(&e); r != hipSuccess) return dev(r, "timing");
    }
    g_gate_timing.on = on != 0;
    g_gate_timing.recorded = false;
    return SUPA_OK;
}

extern "C" supa_status supa_surrogate_last_times(float *ms, int32_t count) {
    if (!ms || count < 1 || count > 3) return bad("ms must hold 1 to 3 floats");
    if (!g_gate_timing.recorded) {
        t_err = "no timed gate_fused call since timing was switched on";
        return SUPA_ERR_STATE;
    }
    if (hipError_t e = hipEventSynchronize(g_gate_timing.ev[3]); e != hipSuccess) return dev(e, "timing");
    for (int i = 0; i < count; ++i)
        if (hipError_t e = hipEventElapsedTime(&ms[i], g_gate_timing.ev[i], g_gate_timing.ev[i + 1]); e != hipSuccess)
            return dev(e, "timing");
    return SUPA_OK;
}

extern "C" supa_status supa_gemm_bf16(void *stream, int trans_a, int trans_b, int epilogue, int M,
                                      int N, int K, const uint16_t *A, int lda, const uint16_t *B,
                                      int ldb, const float *bias, void *C, int ldc, uint16_t *pre) {
    if (M < 1 || N < 1 || K < 1 || (M | N | K) % 8 != 0) return bad("M, N, K must be positive multiples of 8");
    if (lda % 8 || ldb % 8 || ldc < N || lda < 1 || ldb < 1) return bad("bad leading dimensions");
    if (lda < (trans_a ? M : K) || ldb < (trans_b ? K : N)) return bad("leading dimension too small");
    if (!A || !B || !C) return bad("NULL matrix");
    const bool ok = (trans_a == 0 && trans_b == 0 &&
                     (epilogue == SUPA_EPI_F32 || epilogue == SUPA_EPI_BIAS_F32 || epilogue == SUPA_EPI_BIAS_GELU)) ||
                    (trans_a == 0 && trans_b == 1 && (epilogue == SUPA_EPI_F32 || epilogue == SUPA_EPI_GELU_GRAD)) ||
                    (trans_a == 1 && trans_b == 0 && epilogue == SUPA_EPI_F32);
    if (!ok) return bad("unsupported layout / epilogue combination");
    if ((epilogue == SUPA_EPI_BIAS_F32 || epilogue == SUPA_EPI_BIAS_GELU) && !bias) return bad("bias is NULL");
    if (epilogue == SUPA_EPI_GELU_GRAD && !pre) return bad("pre is NULL");
    supa::GemmArgs g{M, N, K, A, B, lda, ldb, bias, C, ldc, pre};
    return dev(supa::launch_gemm(trans_a, trans_b, epilogue, g, (hipStream_t)stream), "gemm");
}

extern "C" int32_t supa_gemm_splitk_parts(int M, int N, int K) {
    if (M < 1 || N < 1 || K < 1) return 1;
    // about 1024 workgroups in all, each with at least 8 K steps of 32
    const int64_t tiles = (int64_t)((M + 127) / 128) * ((N + 127) / 128);
    const int64_t want = (1024 + tiles - 1) / tiles;
    const int64_t most = std::max<int64_t>(1, K / 256);
    return (int32_t)std::max<int64_t>(1, std::min(want, most));
}

extern "C" supa_status supa_gemm_bf16_splitk(void *stream, int trans_a, int trans_b, int M, int N, int K,
                                             const uint16_t *A, int lda, const uint16_t *B, int ldb, float *C,
                                             int parts, float *scratch) {
    if (M < 1 || N < 1 || K < 1 || (M | N | K) % 8 != 0) return bad("M, N, K must be positive multiples of 8");
    if (lda % 8 || ldb % 8 || lda < 1 || ldb < 1) return bad("bad leading dimensions");
    if (lda < (trans_a ? M : K) || ldb < (trans_b ? K : N)) return bad("leading dimension too small");
    if (!A || !B || !C) return bad("NULL matrix");
    if (parts < 1 || parts > 256 || (parts > 1 && !scratch)) return bad("parts in [1, 256]; scratch needed for > 1");
    const bool ok = (trans_a == 0 && trans_b == 0) || (trans_a == 0 && trans_b == 1) || (trans_a == 1 && trans_b == 0);
    if (!ok) return bad("unsupported layout");
    // K range per part: a multiple of the 32-wide K step
    const int chunk = ((K + parts - 1) / parts + 31) / 32 * 32;
    const int used = (K + chunk - 1) / chunk;
    supa::GemmArgs g{};
    g.M = M;
    g.N = N;
    g.K = K;
    g.A = A;
    g.B = B;
    g.lda = lda;
    g.ldb = ldb;
    g.C = used > 1 ? (void *)scratch : (void *)C;
    g.ldc = N;
    g.k_chunk = used > 1 ? chunk : 0;
    supa_status st = dev(supa::launch_gemm(trans_a, trans_b, SUPA_EPI_F32, g, (hipStream_t)stream), "gemm");
    if (st != SUPA_OK || used == 1) return st;
    return dev(supa::launch_sum_parts((int64_t)M * N, used, scratch, C, (hipStream_t)stream), "gemm parts");
}

extern "C" supa_status supa_nll_grad(void *stream, int B, int D, const float *out, const float *img,
                                     const float *e0, float y_scale, float s_clamp, int32_t mse_mean,
                                     uint16_t *dout,
                                     float *loss) {
    if (B < 1 || D < 1) return bad("B and D must be positive");
    if (!out || !img || !e0 || !dout || !loss) return bad("NULL pointer");
    if (!(s_clamp >= 0) || !std::isfinite(s_clamp)) return bad("s_clamp must be finite and >= 0");
    if (mse_mean != 0 && mse_mean != 1) return bad("mse_mean must be 0 or 1");
    return dev(supa::launch_nll(B, D, out, img, e0, y_scale, s_clamp, mse_mean, dout, loss,
                                (hipStream_t)stream), "nll");
}

extern "C" supa_status supa_colsum_bf16(void *stream, int M, int N, const uint16_t *X, int ld, float *out,
                                        float *scratch) {
    if (M < 1 || N < 1 || ld < N || !X || !out) return bad("bad colsum arguments");
    return dev(supa::launch_colsum(M, N, X, ld, out, scratch, (hipStream_t)stream), "colsum");
}

extern "C" int64_t supa_colsum_scratch_floats(int M, int N) {
    return (M < 1 || N < 1) ? 0 : supa::colsum_scratch_floats(M, N);
}

extern "C" supa_status supa_adam(void *stream, int64_t n, float *p, const float *g, float *m, float *v,
                                 uint16_t *p_bf16, float lr, float beta1, float beta2, float eps, int step) {
    if (n < 0 || step < 1 || !p || !g || !m || !v) return bad("bad adam arguments");
    if (n == 0) return SUPA_OK;
    return dev(supa::launch_adam(n, p, g, m, v, p_bf16, lr, beta1, beta2, eps, step, (hipStream_t)stream), "adam");
}

extern "C" supa_status supa_to_bf16(void *stream, int64_t n, const float *x, uint16_t *y) {
    if (n < 0 || (n > 0 && (!x || !y))) return bad("bad to_bf16 arguments");
    if (n == 0) return SUPA_OK;
    return dev(supa::launch_to_bf16(n, x, y, (hipStream_t)stream), "to_bf16");
}

extern "C" supa_status supa_surrogate_features(void *stream, int B, int ld, int n_noise, const float *e0,
                                               const float *polar, const float *azimuth, float e_scale,
                                               float polar_scale, float az_scale, uint32_t row_base,
                                               uint32_t stream_id, uint64_t seed, uint16_t *x) {
    if (B < 0 || n_noise < 0 || ld % 8 || 3 + n_noise > ld) return bad("bad feature sizes");
    if (B == 0) return SUPA_OK;
    if (!e0 || !polar || !azimuth || !x) return bad("NULL pointer");
    return dev(supa::launch_features(B, ld, n_noise, e0, polar, azimuth, e_scale, polar_scale, az_scale,
                                     row_base, stream_id, seed, x, (hipStream_t)stream), "features");
}

extern "C" supa_status supa_surrogate_gate(void *stream, int B, int D, int L, const float *out,
                                           const float *e0, float y_scale, float s_clamp, float *layer_e,
                                           float *unc, float *img, float rho, uint32_t row_base,
                                           uint64_t seed) {
    if (B < 0 || L < 1 || D < L || D % L) return bad("bad gate sizes");
    if (rho > 1.0f) return bad("rho must be <= 1 (negative: no sampling)");
    if (B == 0) return SUPA_OK;
    if (!out || !e0 || !layer_e || !unc) return bad("NULL pointer");
    return dev(supa::launch_gate(B, D, L, out, e0, y_scale, s_clamp, layer_e, unc, img, rho, row_base,
                                 seed, (hipStream_t)stream), "gate");
}

extern "C" supa_status supa_surrogate_gate_fused(void *stream, int B, int K, int D, int L, const uint16_t *h,
                                                 int ldh, const uint16_t *w_t, int ldw, const float *bias,
                                                 const float *e0, float y_scale, float s_clamp, float *partial,
                                                 float *layer_e, float *unc, float rho, uint32_t row_base,
                                                 uint64_t seed, float cnt_thr, float *layer_cnt) {
    if (B < 0 || K < 8 || K % 8 || L < 1 || L > 64 || D < L || D % L || (D / L) % 128)
        return bad("bad fused gate sizes (K multiple of 8, L <= 64, bins per layer multiple of 128)");
    if (ldh < K || ldw < K || ldh % 8 || ldw % 8) return bad("bad leading dimensions");
    if (!(s_clamp >= 0) || !std::isfinite(s_clamp)) return bad("s_clamp must be finite and >= 0");
    if (rho > 1.0f) return bad("rho must be <= 1 (negative: no sampling)");
    if (B == 0) return SUPA_OK;
    if (!h || !w_t || !bias || !e0 || !partial || !layer_e || !unc) return bad("NULL pointer");
    if (((uintptr_t)h | (uintptr_t)w_t) & 15) return bad("h and w_t must be 16-byte aligned");
    if (layer_cnt && !(cnt_thr >= 0)) return bad("cnt_thr must be >= 0");
    const hipEvent_t *ev = nullptr;
    if (g_gate_timing.on) {
        int d = -1;
        if (hipGetDevice(&d) == hipSuccess && d == g_gate_timing.device) ev = g_gate_timing.ev;
    }
    const supa_status st = dev(supa::launch_gate_fused(B, K, D, L, h, ldh, w_t, ldw, bias, e0, y_scale, s_clamp,
                                                       partial, layer_e, unc, rho, row_base, seed, cnt_thr, layer_cnt,
                                                       ev, (hipStream_t)stream),
                               "gate_fused");
    if (ev && st == SUPA_OK) g_gate_timing.recorded = true;
    return st;
}

extern "C" supa_status supa_mlp_forward_fused(void *stream, int B, int k_in, int n_hidden, const uint16_t *x,
                                             int ldx, const uint16_t *const *wt, const float *const *bias, int n_out,
                                             float *out, int ldo, uint16_t *h, int ldh) {
    if (B < 0 || k_in < 16 || k_in > 256 || k_in % 16 || n_hidden < 1 || n_hidden > supa::MLP_FUSED_MAX_HIDDEN)
        return bad("fused forward: k_in a multiple of 16 in [16, 256], 1 to 8 hidden layers");
    if (n_out < 0 || n_out > 64 || n_out % 4) return bad("fused forward: n_out a multiple of 4 in [0, 64]");
    if (ldx < k_in || ldx % 8) return bad("fused forward: ldx >= k_in, a multiple of 8");
    if (n_out > 0 && (ldo < n_out || ldo % 4)) return bad("fused forward: ldo >= n_out, a multiple of 4");
    if (n_out == 0 && (ldh < 256 || ldh % 4)) return bad("fused forward: ldh >= 256, a multiple of 4");
    if (!wt || !bias) return bad("fused forward: NULL weight or bias list");
    if (B == 0) return SUPA_OK;
    if (!x || (n_out > 0 ? !out : !h)) return bad("fused forward: NULL input or output");
    supa::MlpFusedArgs a{};
    a.B = B;
    a.k_in = k_in;
    a.n_hidden = n_hidden;
    a.n_out = n_out;
    a.x = x;
    a.ldx = ldx;
    const int layers = n_hidden + (n_out > 0 ? 1 : 0);
    uintptr_t align = (uintptr_t)x | (n_out > 0 ? (uintptr_t)out : (uintptr_t)h);
    for (int l = 0; l < layers; ++l) {
        if (!wt[l] || !bias[l]) return bad("fused forward: NULL weights or bias of a layer");
        a.wt[l] = wt[l];
        a.bias[l] = bias[l];
        align |= (uintptr_t)wt[l];
    }
    if (align & 15) return bad("fused forward: x, weights and the output must be 16-byte aligned");
    a.out = out;
    a.ldo = ldo;
    a.h = h;
    a.ldh = ldh;
    return dev(supa::launch_mlp_fused(a, (hipStream_t)stream), "mlp_forward_fused");
}

extern "C" supa_status supa_mlp_fused_weights(void *stream, int in, int out, const float *W, int permute,
                                              uint16_t *wt) {
    if (in < 1 || out < 1 || (permute && in % 32)) return bad("fused weights: bad sizes");
    if (!W || !wt) return bad("fused weights: NULL pointer");
    return dev(supa::launch_mlp_weights(in, out, W, permute ? 1 : 0, wt, (hipStream_t)stream), "mlp_fused_weights");
}

extern "C" supa_status supa_transpose_to_bf16(void *stream, int rows, int cols, const float *x, uint16_t *y) {
    if (rows < 0 || cols < 0 || ((int64_t)rows * cols > 0 && (!x || !y))) return bad("bad transpose arguments");
    if ((int64_t)rows * cols == 0) return SUPA_OK;
    return dev(supa::launch_transpose_bf16(rows, cols, x, y, (hipStream_t)stream), "transpose_to_bf16");
}

extern "C" supa_status supa_select_above(void *stream, int n, const float *v, float tau, int32_t *idx,
                                         int32_t *count, int32_t *block_scratch) {
    if (n < 0 || !count || !block_scratch || (n > 0 && (!v || !idx))) return bad("bad select arguments");
    return dev(supa::launch_select(n, v, tau, idx, count, block_scratch, (hipStream_t)stream), "select");
}

extern "C" supa_status supa_gather3(void *stream, int m, const int32_t *idx, const float *a, const float *b,
                                    const float *c, float *oa, float *ob, float *oc) {
    if (m < 0 || (m > 0 && (!idx || !a || !b || !c || !oa || !ob || !oc))) return bad("bad gather arguments");
    return dev(supa::launch_gather3(m, idx, a, b, c, oa, ob, oc, (hipStream_t)stream), "gather3");
}

extern "C" supa_status supa_scatter_rows(void *stream, int m, int w, const int32_t *idx, const float *src,
                                         float *dst) {
    if (m < 0 || w < 0 || (m > 0 && w > 0 && (!idx || !src || !dst))) return bad("bad scatter arguments");
    return dev(supa::launch_scatter_rows(m, w, idx, src, dst, (hipStream_t)stream), "scatter_rows");
}

extern "C" supa_status supa_group_sums(void *stream, int rows, int L, int g, const float *x, float *out) {
    if (rows < 0 || L < 1 || g < 1 || (rows > 0 && (!x || !out))) return bad("bad group_sums arguments");
    return dev(supa::launch_group_sums(rows, L, g, x, out, (hipStream_t)stream), "group_sums");
}

// ---------------------------------------------------------------------------
// the judge: exact W1 of equal-size samples, sorted columns, occupied cells
// ---------------------------------------------------------------------------
static constexpr int64_t kMaxSortRows = 1LL << 30;

static size_t al256s(size_t b) { return (b + 255) & ~(size_t)255; }

extern "C" int64_t supa_sort_columns_workspace_bytes(int64_t n, int32_t cols) {
    if (n < 0 || n > kMaxSortRows || cols < 0 || cols > 4096) return -1;
    return (int64_t)supa::sort_work_bytes(n, cols);
}

extern "C" supa_status supa_sort_columns(void *stream, int64_t n, int32_t cols, const float *x, int64_t ld,
                                         float *out, void *work, int64_t work_bytes) {
    if (n < 0 || n > kMaxSortRows || cols < 0 || cols > 4096) return bad("sort: n or cols out of range");
    if (n == 0 || cols == 0) return SUPA_OK;
    if (!x || !out || !work || ld < cols) return bad("sort: NULL array or ld < cols");
    if (work_bytes < (int64_t)supa::sort_work_bytes(n, cols)) return bad("sort: workspace too small");
    uint32_t *sorted = nullptr;
    supa_status st = dev(supa::launch_sort_columns(x, ld, n, cols, work, &sorted, (hipStream_t)stream), "sort");
    if (st != SUPA_OK) return st;
    return dev(supa::launch_keys_to_floats(sorted, n * cols, out, (hipStream_t)stream), "sorted values");
}

extern "C" int64_t supa_w1_equal_workspace_bytes(int64_t n, int32_t cols) {
    if (n < 0 || n > kMaxSortRows || cols < 0 || cols > 4096) return -1;
    return (int64_t)(2 * al256s(supa::sort_work_bytes(n, cols)) +
                     al256s((size_t)supa::w1_sorted_partial_words(n, cols) * 8));
}

extern "C" supa_status supa_w1_equal(void *stream, int64_t n, int32_t cols, const float *a, int64_t lda,
                                     const float *b, int64_t ldb, double *w1, void *work, int64_t work_bytes) {
    if (n < 1 || n > kMaxSortRows || cols < 1 || cols > 4096) return bad("w1: n or cols out of range");
    if (!a || !b || !w1 || !work || lda < cols || ldb < cols) return bad("w1: NULL array or leading dimension < cols");
    if (work_bytes < supa_w1_equal_workspace_bytes(n, cols)) return bad("w1: workspace too small");
    const size_t sw = al256s(supa::sort_work_bytes(n, cols));
    uint32_t *ka = nullptr, *kb = nullptr;
    const hipStream_t s = (hipStream_t)stream;
    supa_status st = dev(supa::launch_sort_columns(a, lda, n, cols, work, &ka, s), "w1 sort a");
    if (st == SUPA_OK) st = dev(supa::launch_sort_columns(b, ldb, n, cols, (char *)work + sw, &kb, s), "w1 sort b");
    if (st == SUPA_OK)
        st = dev(supa::launch_w1_sorted(ka, kb, n, cols, (double *)((char *)work + 2 * sw), w1, s), "w1 sums");
    return st;
}

extern "C" supa_status supa_occupied_counts(void *stream, int64_t rows, int32_t L, int32_t g, const float *img,
                                            float thr, float *cnt) {
    if (rows < 0 || L < 1 || g < 1) return bad("occupied counts: bad sizes");
    if (rows == 0) return SUPA_OK;
    if (!img || !cnt) return bad("occupied counts: NULL array");
    return dev(supa::launch_occupied_counts(rows, L, g, img, thr, cnt, (hipStream_t)stream), "occupied counts");
}
