// supa_mlp.hip -- kernels of the learned surrogate for gfx950.
//
// The surrogate is a conditional MLP: initial condition (energy, polar angle,
// azimuth; the conditioning variables of the paper's section "Extensions")
// plus Gaussian noise -> hidden layers with GELU -> mean and log-variance of
// the coarse per-layer deposit images (appendix "Downsampling").  Weights and
// activations are bfloat16, every product is accumulated in float32 by the
// matrix cores (v_mfma_f32_16x16x32_bf16).
//
//   gemm      C = op(A) op(B) with A, B bf16 and three layouts: NN (forward),
//             NT (gradient of the input), TN (gradient of the weights); fused
//             epilogues: bias, bias + GELU (keeping the pre-activation),
//             multiplication by GELU' of a stored pre-activation.  128x128
//             tiles per 256-thread workgroup, 64x64 per wave (4x4 MFMA
//             tiles), K in steps of 32 through LDS.
//   nll       Gaussian negative log-likelihood of the targets (image / E0)
//             and its gradient with respect to the outputs.
//   colsum    bias gradients.
//   adam      Adam step on float32 master weights, refreshing the bf16 copy.
//   features  input rows: scaled initial condition and Philox/Box-Muller noise.
//   gate      per shower: predicted per-layer energies, uncertainty score.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "supa_device.hpp"
#include "supa_mlp.hpp"

namespace supa {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float floatx4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// float -> bfloat16, round to nearest even (NaN kept quiet)
__device__ __forceinline__ uint16_t f2bf(float f) {
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

// Phi(a) = erfc(-a / sqrt 2) / 2: no cancellation for negative a
__device__ __forceinline__ float gelu_f(float a) {
    return 0.5f * a * erfcf(-a * 0.707106781f);
}

__device__ __forceinline__ float gelu_grad_f(float a) {
    return 0.5f * erfcf(-a * 0.707106781f) + a * 0.398942280f * __expf(-0.5f * a * a);
}

enum { EPI_F32 = 0, EPI_BIAS_F32 = 1, EPI_BIAS_GELU = 2, EPI_GELU_GRAD = 3, EPI_GATE = 4 };

constexpr int GT = 128;         // tile edge
constexpr int GK = 32;          // K step
constexpr int GPAD = GK + 8;    // LDS row length (bf16), staggers banks

// One K step of the two operand tiles, held in registers between the global
// loads and the LDS stores (so the next step's loads are in flight while
// the current one is multiplied): 512 chunks of 8 bf16 per operand tile,
// two per thread; rows or columns beyond the matrix read as zeros.
struct TileRegs {
    uint4 a[2], b[2];
};

template <int TA, int TB>
__device__ __forceinline__ void tile_load(const GemmArgs &g, int m0, int n0, int k0, TileRegs &R) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const int c = tid + r * 256;
        R.a[r] = make_uint4(0u, 0u, 0u, 0u);
        R.b[r] = make_uint4(0u, 0u, 0u, 0u);
        if (TA == 0) {
            const int m = c >> 2, kc = (c & 3) * 8;
            if (m0 + m < g.M && k0 + kc < g.K) R.a[r] = *(const uint4 *)(g.A + (int64_t)(m0 + m) * g.lda + k0 + kc);
        } else {
            const int k = c >> 4, mc = (c & 15) * 8;
            if (k0 + k < g.K && m0 + mc < g.M) R.a[r] = *(const uint4 *)(g.A + (int64_t)(k0 + k) * g.lda + m0 + mc);
        }
        if (TB == 1) {
            const int n = c >> 2, kc = (c & 3) * 8;
            if (n0 + n < g.N && k0 + kc < g.K) R.b[r] = *(const uint4 *)(g.B + (int64_t)(n0 + n) * g.ldb + k0 + kc);
        } else {
            const int k = c >> 4, nc = (c & 15) * 8;
            if (k0 + k < g.K && n0 + nc < g.N) R.b[r] = *(const uint4 *)(g.B + (int64_t)(k0 + k) * g.ldb + n0 + nc);
        }
    }
}

// The registers of a K step into LDS, both operands K-contiguous per row
// ([row][k]), the layout the matrix-core operands are read in.
template <int TA, int TB>
__device__ __forceinline__ void tile_store(const TileRegs &R, uint16_t (*As)[GPAD], uint16_t (*Bs)[GPAD]) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const int c = tid + r * 256;
        if (TA == 0) {
            *(uint4 *)&As[c >> 2][(c & 3) * 8] = R.a[r];
        } else {
            const int k = c >> 4, mc = (c & 15) * 8;
            const uint16_t *e = (const uint16_t *)&R.a[r];
#pragma unroll
            for (int q = 0; q < 8; ++q) As[mc + q][k] = e[q];
        }
        if (TB == 1) {
            *(uint4 *)&Bs[c >> 2][(c & 3) * 8] = R.b[r];
        } else {
            const int k = c >> 4, nc = (c & 15) * 8;
            const uint16_t *e = (const uint16_t *)&R.b[r];
#pragma unroll
            for (int q = 0; q < 8; ++q) Bs[nc + q][k] = e[q];
        }
    }
}

template <int TA, int TB, int EPI>
__global__ void __launch_bounds__(256) gemm_bf16(GemmArgs g) {
    // two LDS buffers: the matrix cores read one while the next K step is
    // stored into the other (one barrier per step)
    __shared__ __attribute__((aligned(16))) uint16_t As[2][GT][GPAD];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[2][GT][GPAD];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
    const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
    const int lr = lane & 15, lk = (lane >> 4) * 8;

    floatx4_t acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = floatx4_t{0.f, 0.f, 0.f, 0.f};

    const int kb = g.k_chunk > 0 ? blockIdx.z * g.k_chunk : 0;
    const int ke = g.k_chunk > 0 ? min(g.K, kb + g.k_chunk) : g.K;
    TileRegs R;
    if (kb < ke) {
        tile_load<TA, TB>(g, m0, n0, kb, R);
        tile_store<TA, TB>(R, As[0], Bs[0]);
    }
    __syncthreads();
    int cur = 0;
    for (int k0 = kb; k0 < ke; k0 += GK) {
        const bool more = k0 + GK < ke;
        if (more) tile_load<TA, TB>(g, m0, n0, k0 + GK, R);      // in flight during the products
        bf16x8_t a[4], b[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) a[i] = *(const bf16x8_t *)&As[cur][wm + i * 16 + lr][lk];
#pragma unroll
        for (int j = 0; j < 4; ++j) b[j] = *(const bf16x8_t *)&Bs[cur][wn + j * 16 + lr][lk];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        // the other buffer was last read before the previous barrier
        if (more) tile_store<TA, TB>(R, As[cur ^ 1], Bs[cur ^ 1]);
        __syncthreads();
        cur ^= 1;
    }

    if constexpr (EPI == EPI_GATE) {
        // Final layer without its output: per row, the tile's 128 columns
        // (all means, or all log-variances, of half a layer) reduce to
        // sum mu and the number of means above the row's occupancy
        // threshold, or to sum exp(s) and sum exp(s/2) with s clamped;
        // written as C[m][tile][2] (float).  N is a multiple of GT.
        __shared__ float red[2][GT][2];
        const bool var = n0 >= g.split;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float p0 = 0.f, p1 = 0.f;
                const int mrow = m0 + wm + i * 16 + (lane >> 4) * 4 + r;
                const float thr = (!var && g.e0 && mrow < g.M) ? g.cnt_scale / g.e0[mrow] : __builtin_inff();
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const float v = acc[i][j][r] + g.bias[n0 + wn + j * 16 + lr];
                    if (!var) {
                        p0 += v;
                        p1 += v > thr ? 1.0f : 0.0f;
                    } else {
                        const float sv = fminf(fmaxf(v, -g.s_clamp), g.s_clamp);
                        p0 += __expf(sv);
                        p1 += __expf(0.5f * sv);
                    }
                }
#pragma unroll
                for (int off = 1; off < 16; off <<= 1) {
                    p0 += __shfl_xor(p0, off, 64);
                    p1 += __shfl_xor(p1, off, 64);
                }
                if (lr == 0) {
                    const int row = wm + i * 16 + (lane >> 4) * 4 + r;
                    red[wave & 1][row][0] = p0;
                    red[wave & 1][row][1] = p1;
                }
            }
        __syncthreads();
        if (tid < GT && m0 + tid < g.M) {
            float *P = (float *)g.C + ((int64_t)(m0 + tid) * gridDim.x + blockIdx.x) * 2;
            P[0] = red[0][tid][0] + red[1][tid][0];
            P[1] = red[0][tid][1] + red[1][tid][1];
        }
        return;
    }

    // accumulator element r of tile (i, j): row 4*(lane/16) + r, column lane%16
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm + i * 16 + (lane >> 4) * 4 + r;
                const int n = n0 + wn + j * 16 + lr;
                if (m >= g.M || n >= g.N) continue;
                const int64_t o = (int64_t)m * g.ldc + n;
                float v = acc[i][j][r];
                if (EPI == EPI_F32) {
                    ((float *)g.C)[o + (int64_t)blockIdx.z * g.M * g.ldc] = v;
                } else if (EPI == EPI_BIAS_F32) {
                    ((float *)g.C)[o] = v + g.bias[n];
                } else if (EPI == EPI_BIAS_GELU) {
                    v += g.bias[n];
                    if (g.pre) g.pre[o] = f2bf(v);
                    ((uint16_t *)g.C)[o] = f2bf(gelu_f(v));
                } else {   // EPI_GELU_GRAD
                    ((uint16_t *)g.C)[o] = f2bf(v * gelu_grad_f(bf2f(g.pre[o])));
                }
            }
}

// out[i] = sum over z < parts of part[z][i], in order (split-K reduction)
__global__ void sum_parts_kernel(int64_t n, int parts, const float *part, float *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float s = 0.0f;
    for (int z = 0; z < parts; ++z) s += part[(int64_t)z * n + i];
    out[i] = s;
}

hipError_t launch_sum_parts(int64_t n, int parts, const float *part, float *out, hipStream_t s) {
    hipLaunchKernelGGL(sum_parts_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, parts, part, out);
    return hipGetLastError();
}

hipError_t launch_gemm(int ta, int tb, int epi, const GemmArgs &g, hipStream_t s) {
    const int parts = g.k_chunk > 0 ? (g.K + g.k_chunk - 1) / g.k_chunk : 1;
    const dim3 grid((g.N + GT - 1) / GT, (g.M + GT - 1) / GT, parts), block(256);
#define SUPA_GEMM_CASE(TA, TB, EPI)                                              \
    if (ta == TA && tb == TB && epi == EPI) {                                     \
        hipLaunchKernelGGL((gemm_bf16<TA, TB, EPI>), grid, block, 0, s, g);     \
        return hipGetLastError();                                                 \
    }
    SUPA_GEMM_CASE(0, 0, EPI_F32)
    SUPA_GEMM_CASE(0, 0, EPI_BIAS_F32)
    SUPA_GEMM_CASE(0, 0, EPI_BIAS_GELU)
    SUPA_GEMM_CASE(0, 1, EPI_F32)
    SUPA_GEMM_CASE(0, 1, EPI_GELU_GRAD)
    SUPA_GEMM_CASE(1, 0, EPI_F32)
    SUPA_GEMM_CASE(0, 1, EPI_GATE)
#undef SUPA_GEMM_CASE
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Gaussian NLL over rows b < B and bins j < D: out = [mu | s_raw] (float
// [B][2D]), target y = img[b][j] * y_scale / e0[b].  Writes d(loss)/d(out)
// as bf16 (the backward GEMMs' input) and adds the loss sum into *loss.
// ---------------------------------------------------------------------------
__global__ void nll_kernel(int B, int D, const float *out, const float *img, const float *e0,
                           float y_scale, float s_clamp, int mse_mean, uint16_t *dout, float *loss) {
    __shared__ float part[256];
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)B * D;
    const float inv_n = 1.0f / (float)total;
    float l = 0.0f;
    for (int64_t q = t; q < total; q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = q / D, j = q - b * D;
        const float mu = out[b * 2 * D + j];
        const float sr = out[b * 2 * D + D + j];
        const float s = fminf(fmaxf(sr, -s_clamp), s_clamp);
        const float y = img[b * D + j] * y_scale / e0[b];
        const float r = y - mu;
        const float ie = __expf(-s);
        l += 0.5f * (s + r * r * ie);
        dout[b * 2 * D + j] = f2bf(-r * (mse_mean ? 1.0f : ie) * inv_n);
        dout[b * 2 * D + D + j] = f2bf(fabsf(sr) <= s_clamp ? 0.5f * (1.0f - r * r * ie) * inv_n : 0.0f);
    }
    part[threadIdx.x] = l;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(loss, part[0]);
}

// column sums of a bf16 matrix [M][ld] (first N columns) -> float [N]
__global__ void colsum_kernel(int M, int N, const uint16_t *X, int ld, float *out) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    float s = 0.0f;
    for (int m = 0; m < M; ++m) s += bf2f(X[(int64_t)m * ld + n]);
    out[n] = s;
}

// Column sums in two deterministic passes: block (column tile of 64, slice
// of CS_ROWS rows) -> part[slice][n] (four waves take interleaved rows, lane
// = column, then the four partial sums meet in LDS); then per column the
// slices in order.
constexpr int CS_ROWS = 256;
__global__ void __launch_bounds__(256) colsum_part_kernel(int M, int N, const uint16_t *X, int ld, float *part) {
    __shared__ float red[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int n = blockIdx.x * 64 + lane;
    const int m0 = blockIdx.y * CS_ROWS, m1 = min(M, m0 + CS_ROWS);
    float s = 0.0f;
    if (n < N)
        for (int m = m0 + w; m < m1; m += 4) s += bf2f(X[(int64_t)m * ld + n]);
    red[w][lane] = s;
    __syncthreads();
    if (w == 0 && n < N) part[(int64_t)blockIdx.y * N + n] = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
}

__global__ void colsum_final_kernel(int slices, int N, const float *part, float *out) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    float s = 0.0f;
    for (int q = 0; q < slices; ++q) s += part[(int64_t)q * N + n];
    out[n] = s;
}

// Adam step (Kingma & Ba 2015) on float32 parameters, bf16 copy refreshed.
__global__ void adam_kernel(int64_t n, float *p, const float *grad, float *m, float *v,
                            uint16_t *p_bf16, float lr, float b1, float b2, float eps,
                            float c1, float c2) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const float g = grad[t];
    const float mm = b1 * m[t] + (1.0f - b1) * g;
    const float vv = b2 * v[t] + (1.0f - b2) * g * g;
    m[t] = mm;
    v[t] = vv;
    const float w = p[t] - lr * (mm / c1) / (sqrtf(vv / c2) + eps);
    p[t] = w;
    if (p_bf16) p_bf16[t] = f2bf(w);
}

__global__ void to_bf16_kernel(int64_t n, const float *x, uint16_t *y) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) y[t] = f2bf(x[t]);
}

// Input rows [B][ld]: e0 * e_scale, polar * polar_scale, azimuth * az_scale,
// then n_noise standard normals (Box-Muller on Philox words keyed by
// (seed; row id, stream, 0x5eed, 0)), then zeros up to ld.
__global__ void features_kernel(int B, int ld, int n_noise, const float *e0, const float *polar,
                                const float *az, float e_scale, float polar_scale, float az_scale,
                                uint32_t row_base, uint32_t stream, uint32_t k0, uint32_t k1,
                                uint16_t *x) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    uint16_t *row = x + (int64_t)b * ld;
    row[0] = f2bf(e0[b] * e_scale);
    row[1] = f2bf(polar[b] * polar_scale);
    row[2] = f2bf(az[b] * az_scale);
    for (int q = 0; q < n_noise; q += 4) {
        const uint4 w = philox4x32_10(row_base + (uint32_t)b, stream, 0x5eedu, (uint32_t)q, k0, k1);
        const float u1 = ((float)w.x + 0.5f) * 0x1p-32f, u2 = ((float)w.y + 0.5f) * 0x1p-32f;
        const float u3 = ((float)w.z + 0.5f) * 0x1p-32f, u4 = ((float)w.w + 0.5f) * 0x1p-32f;
        const float r1 = sqrtf(-2.0f * logf(u1)), r2 = sqrtf(-2.0f * logf(u3));
        float s1, c1, s2, c2;
        sincospif(2.0f * u2, &s1, &c1);
        sincospif(2.0f * u4, &s2, &c2);
        const float z[4] = {r1 * c1, r1 * s1, r2 * c2, r2 * s2};
        for (int e = 0; e < 4 && q + e < n_noise; ++e) row[3 + q + e] = f2bf(z[e]);
    }
    for (int c = 3 + n_noise; c < ld; ++c) row[c] = 0;
}

// The same rows for the network's own layout (32 inputs: 3 scaled initial
// conditions, NOISE normals, zeros), built in registers and written as four
// 16-byte stores per row instead of one 2-byte store per input: the same
// values, a quarter of the per-row store instructions' traffic in flight.
template <int NOISE>
__global__ void features32_kernel(int B, const float *e0, const float *polar, const float *az, float e_scale,
                                  float polar_scale, float az_scale, uint32_t row_base, uint32_t stream,
                                  uint32_t k0, uint32_t k1, uint16_t *x) {
    static_assert(3 + NOISE <= 32, "32 inputs per row");
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    float v[32];
#pragma unroll
    for (int c = 0; c < 32; ++c) v[c] = 0.0f;
    v[0] = e0[b] * e_scale;
    v[1] = polar[b] * polar_scale;
    v[2] = az[b] * az_scale;
#pragma unroll
    for (int q = 0; q < NOISE; q += 4) {
        const uint4 w = philox4x32_10(row_base + (uint32_t)b, stream, 0x5eedu, (uint32_t)q, k0, k1);
        const float u1 = ((float)w.x + 0.5f) * 0x1p-32f, u2 = ((float)w.y + 0.5f) * 0x1p-32f;
        const float u3 = ((float)w.z + 0.5f) * 0x1p-32f, u4 = ((float)w.w + 0.5f) * 0x1p-32f;
        const float r1 = sqrtf(-2.0f * logf(u1)), r2 = sqrtf(-2.0f * logf(u3));
        float s1, c1, s2, c2;
        sincospif(2.0f * u2, &s1, &c1);
        sincospif(2.0f * u4, &s2, &c2);
        const float z[4] = {r1 * c1, r1 * s1, r2 * c2, r2 * s2};
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (q + e < NOISE) v[3 + q + e] = z[e];
    }
    uint32_t p[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) p[c] = (uint32_t)f2bf(v[2 * c]) | ((uint32_t)f2bf(v[2 * c + 1]) << 16);
    uint4 *row = (uint4 *)(x + (int64_t)b * 32);
#pragma unroll
    for (int c = 0; c < 4; ++c) row[c] = make_uint4(p[4 * c], p[4 * c + 1], p[4 * c + 2], p[4 * c + 3]);
}

// Per shower b: predicted per-layer energies E0 * sum_bins mu (float [B][L]),
// uncertainty sqrt(sum sigma^2) / max(sum mu, tiny), and optionally the
// predicted image E0 * mu (float [B][D]).  With rho >= 0 the per-layer
// energies are samples instead: E0 * (sum mu + sd * z), z standard normal
// (Box-Muller on Philox words keyed by seed and counted by (row, layer, 0x9a7e, 0)),
// sd^2 = rho (sum sigma)^2 + (1 - rho) sum sigma^2: bins of a layer with
// correlation rho.
__global__ void gate_kernel(int B, int D, int L, const float *out, const float *e0,
                            float y_scale, float s_clamp, float *layer_e, float *unc,
                            float *img, float rho, uint32_t row_base, uint32_t k0, uint32_t k1) {
    const int b = blockIdx.x;
    const int bins = D / L;
    __shared__ float sm[256], sv[256];
    __shared__ float ss[256];
    const float *row = out + (int64_t)b * 2 * D;
    const float scale = e0[b] / y_scale;
    float tm = 0.f, tv = 0.f;
    for (int l = 0; l < L; ++l) {
        float pm = 0.f, pv = 0.f, ps = 0.f;
        for (int j = threadIdx.x; j < bins; j += blockDim.x) {
            const float mu = row[l * bins + j];
            const float s = fminf(fmaxf(row[D + l * bins + j], -s_clamp), s_clamp);
            pm += mu;
            pv += __expf(s);
            ps += __expf(0.5f * s);
            if (img) img[(int64_t)b * D + l * bins + j] = mu * scale;
        }
        sm[threadIdx.x] = pm;
        sv[threadIdx.x] = pv;
        ss[threadIdx.x] = ps;
        __syncthreads();
        for (int w = blockDim.x / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) {
                sm[threadIdx.x] += sm[threadIdx.x + w];
                sv[threadIdx.x] += sv[threadIdx.x + w];
                ss[threadIdx.x] += ss[threadIdx.x + w];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            float v = sm[0];
            if (rho >= 0.0f) {
                const uint4 w = philox4x32_10(row_base + (uint32_t)b, (uint32_t)l, 0x9a7eu, 0u, k0, k1);
                const float u1 = ((float)w.x + 0.5f) * 0x1p-32f, u2 = ((float)w.y + 0.5f) * 0x1p-32f;
                float sn, cs;
                sincospif(2.0f * u2, &sn, &cs);
                const float z = sqrtf(-2.0f * logf(u1)) * cs;
                const float sd = sqrtf(rho * ss[0] * ss[0] + (1.0f - rho) * sv[0]);
                v += sd * z;
            }
            layer_e[(int64_t)b * L + l] = v * scale;
            tm += sm[0];
            tv += sv[0];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) unc[b] = sqrtf(tv) / fmaxf(tm, 1e-6f);
}

// Per shower b (one wave; lane l < L takes layer l): the per-tile sums of
// the fused final layer (P[b][tile][2], tiles of GT columns) combined into
// what gate_kernel computes from the full output: per-layer energies (or
// samples, same Philox counters) and the uncertainty score.
__global__ void __launch_bounds__(256) gate_tiles_kernel(int B, int D, int L, const float *P, const float *e0,
                                                         float y_scale, float *layer_e, float *unc, float rho,
                                                         uint32_t row_base, uint32_t k0, uint32_t k1,
                                                         float *layer_cnt) {
    const int b = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (b >= B) return;                                   // whole waves leave together
    const int tiles = 2 * D / GT, tpl = D / L / GT;
    const float *row = P + (int64_t)b * tiles * 2;
    float sm = 0.f, sv = 0.f, ss = 0.f, sc = 0.f;
    if (lane < L) {
        for (int t = 0; t < tpl; ++t) {
            sm += row[2 * (lane * tpl + t)];
            sc += row[2 * (lane * tpl + t) + 1];
            sv += row[2 * (D / GT + lane * tpl + t)];
            ss += row[2 * (D / GT + lane * tpl + t) + 1];
        }
        if (layer_cnt) layer_cnt[(int64_t)b * L + lane] = sc;
        float v = sm;
        if (rho >= 0.0f) {
            const uint4 w = philox4x32_10(row_base + (uint32_t)b, (uint32_t)lane, 0x9a7eu, 0u, k0, k1);
            const float u1 = ((float)w.x + 0.5f) * 0x1p-32f, u2 = ((float)w.y + 0.5f) * 0x1p-32f;
            float sn, cs;
            sincospif(2.0f * u2, &sn, &cs);
            const float z = sqrtf(-2.0f * logf(u1)) * cs;
            v += sqrtf(rho * ss * ss + (1.0f - rho) * sv) * z;
        }
        layer_e[(int64_t)b * L + lane] = v * (e0[b] / y_scale);
    }
    float tm = sm, tv = sv;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        tm += __shfl_xor(tm, off, 64);
        tv += __shfl_xor(tv, off, 64);
    }
    if (lane == 0) unc[b] = sqrtf(tv) / fmaxf(tm, 1e-6f);
}

// y[c][r] = bf16(x[r][c]) (float [rows][cols] -> bf16 [cols][rows])
__global__ void transpose_bf16_kernel(int rows, int cols, const float *x, uint16_t *y) {
    __shared__ float t[32][33];
    const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
    for (int q = threadIdx.y; q < 32; q += 8) {
        const int r = r0 + q, c = c0 + threadIdx.x;
        t[q][threadIdx.x] = (r < rows && c < cols) ? x[(int64_t)r * cols + c] : 0.0f;
    }
    __syncthreads();
    for (int q = threadIdx.y; q < 32; q += 8) {
        const int c = c0 + q, r = r0 + threadIdx.x;
        if (c < cols && r < rows) y[(int64_t)c * rows + r] = f2bf(t[threadIdx.x][q]);
    }
}

// ---------------------------------------------------------------------------
// The final layer fused into the gate for the hidden width K = 256, taken
// transposed: C^T[n][m] = sum_k Wt[n][k] h[m][k] (n an output column, m a
// row), so that a row's sum over a tile's columns is mostly a sum within
// each lane.  A workgroup of four waves (one per SIMD) covers 256 rows and
// holds them in registers for the whole launch: wave w keeps rows
// 64 w .. + 64 as matrix-core B operands and takes all 128 columns of every
// tile, in two halves of 64.  W^T streams through LDS a tile (128 columns
// by all of K) at a time, two buffers, copied straight from memory into LDS
// (no registers on the way) while the matrix cores work on the previous
// tile.  Every W^T element fetched serves 256 rows and h is read once (the
// 128 x 128 tiles of gemm_bf16 fetch both operands per tile, more than the
// L2 can feed at the matrix cores' rate when K is this short).  Two
// accumulator sets, one per half: the reduction of one half (exponentials,
// sums, counts) is issued between the matrix products of the next.  One
// launch covers tiles of one kind (means, or log-variances); writes the
// same (row, tile) pairs as the EPI_GATE epilogue.
// ---------------------------------------------------------------------------
constexpr int GF_K = 256, GF_NT = 128, GF_ROWS = 256;
constexpr int GF_JW = 1;                     // blocks of 32 rows per wave (see GfState)
constexpr float GF_HALF_LOG2E = 0.72134752044448170f;     // exp(s / 2) = 2^(s * this)
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
typedef float floatx16_t __attribute__((ext_vector_type(16)));
typedef uint16_t GfTile[GF_NT][GF_K];
template <int JW> using GfAcc = floatx16_t[2][JW];      // [32-column block i][32-row block j]

// JW: blocks of 32 rows per wave (2: four waves of 64 rows, one per SIMD;
// 1: eight waves of 32 rows, two per SIMD)
template <int JW>
struct GfState {
    static constexpr int NW = 8 / JW;        // waves per workgroup
    const GemmArgs *g;
    int tid, wave, lane, lc, lh, mw, tiles;
    bf16x8_t hb[JW][16];
    float thr[JW];
    float c0[JW], c1[JW];                    // the first half's sums of the tile in flight
};

// LDS image of a W^T tile, in 16-byte chunks (8 bf16): chunk c of row n
// sits at byte 8192 (c >> 2) + 64 n + 16 ((c & 3) ^ ((n >> 2) & 3)).  Sixteen
// consecutive rows read at the same c fall on sixteen distinct bank groups,
// a K step's address is one of two per-lane bases plus a constant, and a
// copy instruction takes 64 contiguous bytes from each of 16 rows.
template <int JW>
__device__ __forceinline__ void gf_issue(const GfState<JW> &S, int t, GfTile &W, float *Bt) {
    // the eight chunk groups (chunks 4 g .. + 4 of every row) split evenly
    // over the waves; copy q of a group covers rows 16 q .. + 16, lane l
    // landing at byte 16 l of its 1 KB; waves 0 and 1 also copy 64 floats of
    // the bias
    constexpr int G = 8 / GfState<JW>::NW;
#pragma unroll
    for (int gs = 0; gs < G; ++gs)
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int grp = G * S.wave + gs;
            const int row = 16 * q + (S.lane >> 2);
            const int c = 4 * grp + ((S.lane & 3) ^ ((row >> 2) & 3));
            const uint16_t *src = S.g->B + (int64_t)(t * GF_NT + row) * S.g->ldb + c * 8;
            __builtin_amdgcn_global_load_lds(
                src, (__attribute__((address_space(3))) void *)((char *)&W[0][0] + 8192 * grp + 1024 * q), 16, 0, 0);
        }
    if (S.wave < 2)
        __builtin_amdgcn_global_load_lds(S.g->bias + t * GF_NT + 64 * S.wave + S.lane,
                                         (__attribute__((address_space(3))) void *)(Bt + 64 * S.wave), 4, 0, 0);
}

// One half-tile step: the matrix products of half PH of the tile in W into
// acc (if PROD), and in the same straight-line block the reduction of the
// previous half (prev, half RH of the tile with bias Bp; RED 1 means,
// 2 means with counts, 3 log-variances), so that its vector instructions
// issue while the matrix cores are busy.  prev[i][j][r] = column
// 64 RH + 32 i + 8 (r >> 2) + 4 lh + (r & 3) of row mw + 32 j + lc.  Per
// row, means reduce to sum mu and the number above the row's occupancy
// threshold, log-variances (clamped) to sum exp(s) and sum exp(s/2).  After
// half 0 the sums wait in S.c0 / S.c1; after half 1 the row's pair for
// tile tp is written.
template <bool PROD, int PH, int RED, int RH, int JW>
__device__ __forceinline__ void gf_half(GfState<JW> &S, const GfTile &W, GfAcc<JW> &acc, const GfAcc<JW> &prev,
                                        const float *Bp, int tp) {
    float p0[JW] = {}, p1[JW] = {};
    int cnt[JW] = {};
    const float lim = S.g->s_clamp * GF_HALF_LOG2E;
    const char *base[2][2];
    if constexpr (PROD) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int row = 64 * PH + 32 * i + S.lc;
#pragma unroll
            for (int odd = 0; odd < 2; ++odd)
                base[i][odd] = (const char *)&W[0][0] + 64 * row + 16 * ((2 * odd + S.lh) ^ ((row >> 2) & 3));
        }
    }
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
        if constexpr (PROD) {
            bf16x8_t a[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) a[i] = *(const bf16x8_t *)(base[i][kk & 1] + 8192 * (kk >> 1));
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < JW; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                        a[i], S.hb[j][kk], kk == 0 ? floatx16_t{} : acc[i][j], 0, 0, 0);
        }
        if constexpr (RED != 0) {
            if (kk < 8) {
                // step kk reduces column group (i, q) = (kk >> 2, kk & 3)
                const int i = kk >> 2, q = kk & 3;
                floatx4_t bv = *(const floatx4_t *)&Bp[64 * RH + 32 * i + 8 * q + 4 * S.lh];
                if constexpr (RED == 3) bv *= GF_HALF_LOG2E;
#pragma unroll
                for (int j = 0; j < JW; ++j)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const float a = prev[i][j][4 * q + r];
                        if constexpr (RED == 3) {
                            const float x = __builtin_amdgcn_fmed3f(fmaf(a, GF_HALF_LOG2E, bv[r]), -lim, lim);
                            const float e = __builtin_amdgcn_exp2f(x);
                            p0[j] = fmaf(e, e, p0[j]);
                            p1[j] += e;
                        } else {
                            const float v = a + bv[r];
                            p0[j] += v;
                            if constexpr (RED == 2) cnt[j] += v > S.thr[j] ? 1 : 0;
                        }
                    }
            }
        }
    }
    if constexpr (RED != 0) {
#pragma unroll
        for (int j = 0; j < JW; ++j) {
            if constexpr (RED == 2) p1[j] = (float)cnt[j];
            p0[j] += __shfl_xor(p0[j], 32, 64);
            p1[j] += __shfl_xor(p1[j], 32, 64);
            if constexpr (RH == 0) {
                S.c0[j] = p0[j];
                S.c1[j] = p1[j];
            } else {
                const int m = S.mw + 32 * j + S.lc;
                if (S.lh == 0 && m < S.g->M) {
                    float *P = (float *)S.g->C + ((int64_t)m * S.tiles + tp) * 2;
                    P[0] = S.c0[j] + p0[j];
                    P[1] = S.c1[j] + p1[j];
                }
            }
        }
    }
}

// Tile t's interval: the next tile copied into Wn / Bn while the halves of
// tile t (from Wc) are multiplied beside the reductions of tile t - 1's
// second half (bias Bp) and tile t's first half (bias Bc).  Wn, Bn were
// last read before the previous barrier; all buffers are distinct LDS
// variables chosen at compile time, so the compiler sees that reads of Wc,
// Bc and Bp need not wait for the copies.
template <int RED, bool FIRST, int JW>
__device__ __forceinline__ void gf_interval(GfState<JW> &S, int t, int t1, const GfTile &Wc, GfTile &Wn, float *Bn,
                                            const float *Bc, const float *Bp, GfAcc<JW> &acc0, GfAcc<JW> &acc1) {
    if (t + 1 < t1) gf_issue(S, t + 1, Wn, Bn);
    if constexpr (FIRST) gf_half<true, 0, 0, 1, JW>(S, Wc, acc0, acc1, Bp, t - 1);
    else gf_half<true, 0, RED, 1, JW>(S, Wc, acc0, acc1, Bp, t - 1);
    gf_half<true, 1, RED, 0, JW>(S, Wc, acc1, acc0, Bc, t);
    __builtin_amdgcn_s_waitcnt(0);                  // this wave's copies into LDS have landed
    __syncthreads();
}

// Tiles [t0, t1) of the product, all of one kind: RED 1 (means), 2 (means
// with counts) or 3 (log-variances).
template <int RED, int JW>
__global__ void __launch_bounds__(512 / JW, 1) gate_fused_k256_kernel(GemmArgs g, int t0, int t1) {
    __shared__ __attribute__((aligned(1024))) GfTile W0, W1;
    __shared__ __attribute__((aligned(16))) float B0[GF_NT], B1[GF_NT], B2[GF_NT], B3[GF_NT];
    GfState<JW> S;
    S.g = &g;
    S.tid = threadIdx.x;
    S.wave = __builtin_amdgcn_readfirstlane(S.tid >> 6);     // wave-uniform: scalar registers
    S.lane = S.tid & 63;
    S.lc = S.lane & 31;
    S.lh = S.lane >> 5;
    S.mw = blockIdx.x * GF_ROWS + S.wave * 32 * JW;
    S.tiles = g.N / GF_NT;
#pragma unroll
    for (int j = 0; j < JW; ++j) S.c0[j] = S.c1[j] = 0.f;

    // hb[j][kk]: row mw + 32 j + lc, k = 16 kk + 8 lh .. + 8 (zeros beyond M)
#pragma unroll
    for (int j = 0; j < JW; ++j) {
        const int m = S.mw + 32 * j + S.lc;
        S.thr[j] = (RED == 2 && m < g.M) ? g.cnt_scale / g.e0[m] : __builtin_inff();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            u32x4_t v = {0u, 0u, 0u, 0u};
            if (m < g.M) v = *(const u32x4_t *)(g.A + (int64_t)m * g.lda + 16 * kk + 8 * S.lh);
            S.hb[j][kk] = __builtin_bit_cast(bf16x8_t, v);
        }
    }

    // tile t0 + u: W(u & 1), bias slot u & 3
    GfAcc<JW> acc0, acc1;
    gf_issue(S, t0, W0, B0);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    gf_interval<RED, true, JW>(S, t0, t1, W0, W1, B1, B0, B3, acc0, acc1);
    int t = t0 + 1;
    for (; t + 4 <= t1; t += 4) {
        gf_interval<RED, false, JW>(S, t, t1, W1, W0, B2, B1, B0, acc0, acc1);
        gf_interval<RED, false, JW>(S, t + 1, t1, W0, W1, B3, B2, B1, acc0, acc1);
        gf_interval<RED, false, JW>(S, t + 2, t1, W1, W0, B0, B3, B2, acc0, acc1);
        gf_interval<RED, false, JW>(S, t + 3, t1, W0, W1, B1, B0, B3, acc0, acc1);
    }
    // the remaining tiles (fewer than four), then the last tile's second half
    const int left = t1 - t;
    if (left >= 1) gf_interval<RED, false, JW>(S, t, t1, W1, W0, B2, B1, B0, acc0, acc1);
    if (left >= 2) gf_interval<RED, false, JW>(S, t + 1, t1, W0, W1, B3, B2, B1, acc0, acc1);
    if (left >= 3) gf_interval<RED, false, JW>(S, t + 2, t1, W1, W0, B0, B3, B2, acc0, acc1);
    switch (left) {
    case 0: gf_half<false, 0, RED, 1, JW>(S, W0, acc0, acc1, B0, t1 - 1); break;
    case 1: gf_half<false, 0, RED, 1, JW>(S, W0, acc0, acc1, B1, t1 - 1); break;
    case 2: gf_half<false, 0, RED, 1, JW>(S, W0, acc0, acc1, B2, t1 - 1); break;
    default: gf_half<false, 0, RED, 1, JW>(S, W0, acc0, acc1, B3, t1 - 1); break;
    }
}

// ---------------------------------------------------------------------------
// The forward pass of the whole MLP in one kernel (inference): a workgroup
// of eight waves (two per SIMD) takes 256 rows through every layer with the
// activations in registers, never in memory.  Wave w holds its 32 rows as
// `v_mfma_f32_32x32x16_bf16` B operands (all 256 inputs: 64 registers); a
// layer's products (transposed, as in gate_fused_k256_kernel: W^T from LDS
// is the A operand) leave each lane the outputs 32 i + 8 g + 4 lh + q of its
// row, which bias + GELU + bf16 turn straight into the next layer's B
// operands: element 4 (g & 1) + q of K step 2 i + (g >> 1).  The next layer
// therefore sees its inputs in an order that swaps bits 2 and 3 of the index
// within each block of 32; its weights are stored with the input index
// permuted the same way (mlp_permute_k), so nothing moves between lanes.
// Each layer's W^T streams through LDS in tiles of 128 outputs by all its
// inputs, two buffers copied straight into LDS while the previous tile is
// multiplied (the tile layout of gate_fused_k256_kernel), the tile's bias
// beside it.  Out: the last hidden activations (bf16, natural order) or,
// with FINAL, a linear layer of n_out <= 64 outputs (float).
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int mlp_permute_k(int k) {
    return (k & ~12) | ((k & 4) << 1) | ((k & 8) >> 1);
}

// GELU(a) = a Phi(a) with Phi(a) - 1/2 = c P(c^2), c = a clamped to
// [-3.7, 3.7] and P a polynomial of degree 6: a weighted least-squares fit
// driven to equal ripple (Lawson's iteration, Chebyshev basis on the clamped
// range, then powers of c^2; gelu_poly_fit.py prints the coefficients).  In
// float32 its Phi is within 5.9e-5 of the exact one for every a (the clamp
// included: Phi(-3.7) ~ 1.1e-4 is split between both ends), so GELU is off by
// at most 5.9e-5 |a|: a fiftieth of the bf16 rounding of the result.  Seven
// multiply-adds and no transcendental: the erfc forms cost two
// quarter-rate instructions and ten more per element (gelu_f, exact, is kept
// for training).
__device__ __forceinline__ float gelu_poly(float a) {
    const float c = __builtin_amdgcn_fmed3f(a, -3.7f, 3.7f);
    const float s = c * c;
    float p = 4.174848555749122e-08f;
    p = fmaf(p, s, -2.483809566911077e-06f);
    p = fmaf(p, s, 6.402656435966492e-05f);
    p = fmaf(p, s, -0.0009566032676957548f);
    p = fmaf(p, s, 0.009406556375324726f);
    p = fmaf(p, s, -0.06585532426834106f);
    p = fmaf(p, s, 0.398733526468277f);       // ~ 1 / sqrt(2 pi) = Phi'(0)
    return a * fmaf(c, p, 0.5f);
}

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));

// two floats to a pair of bf16 (round to nearest even: v_cvt_pk_bf16_f32)
__device__ __forceinline__ uint32_t pack_bf16x2(float lo, float hi) {
    const bf16x2_t v = {(__bf16)lo, (__bf16)hi};
    return __builtin_bit_cast(uint32_t, v);
}

struct MfState {
    const MlpFusedArgs *a;
    int tid, wave, lane, lc, lh, row, tiles;
    u32x4_t hb[16], hn[16];          // 8 bf16 each: B operands of K steps
};

// tile u: hidden layer u / 2, outputs 128 (u % 2) .. + 128; with FINAL the
// last tile is the output layer
__device__ __forceinline__ void mf_issue(const MfState &S, int u, GfTile &W, float *Bt) {
    const MlpFusedArgs &a = *S.a;
    const bool fin = u >= 2 * a.n_hidden;
    const int l = fin ? a.n_hidden : u >> 1;
    const int K = l == 0 ? a.k_in : GF_K;
    const int r0 = fin ? 0 : 128 * (u & 1), rows = fin ? a.n_out : 128;
    const uint16_t *src = a.wt[l] + (int64_t)r0 * K;
    // wave w copies rows 16 w .. + 16 of every chunk group (4 chunks of 8)
    const int r = 16 * S.wave + (S.lane >> 2);
    for (int g = 0; g < K / 32; ++g)
        if (r < rows) {
            const int c = 4 * g + ((S.lane & 3) ^ ((r >> 2) & 3));
            __builtin_amdgcn_global_load_lds(
                src + (int64_t)r * K + c * 8,
                (__attribute__((address_space(3))) void *)((char *)&W[0][0] + 8192 * g + 1024 * S.wave), 16, 0, 0);
        }
    const int bi = 64 * S.wave + S.lane;
    if (S.wave < 2 && bi < rows)
        __builtin_amdgcn_global_load_lds(a.bias[l] + r0 + bi,
                                         (__attribute__((address_space(3))) void *)(Bt + 64 * S.wave), 4, 0, 0);
}

// acc[i] += the products of tile rows 32 i + .. (i < NI) with this wave's rows
template <int NI>
__device__ __forceinline__ void mf_products(const MfState &S, const GfTile &W, int ks, floatx16_t (&acc)[4]) {
    const char *base[NI][2];
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const int r = 32 * i + S.lc;
#pragma unroll
        for (int odd = 0; odd < 2; ++odd)
            base[i][odd] = (const char *)&W[0][0] + 64 * r + 16 * ((2 * odd + S.lh) ^ ((r >> 2) & 3));
    }
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
        if (kk < ks) {
            bf16x8_t w[NI];
#pragma unroll
            for (int i = 0; i < NI; ++i) w[i] = *(const bf16x8_t *)(base[i][kk & 1] + 8192 * (kk >> 1));
#pragma unroll
            for (int i = 0; i < NI; ++i)
                acc[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w[i], __builtin_bit_cast(bf16x8_t, S.hb[kk]),
                                                                  acc[i], 0, 0, 0);
        }
    }
}

// tile u from Wc / Bc, the next tile copied into Wn / Bn meanwhile (distinct
// LDS variables chosen at compile time: reads of Wc need not wait for it)
template <bool FINAL>
__device__ __forceinline__ void mf_tile(MfState &S, int u, const GfTile &Wc, const float *Bc, GfTile &Wn,
                                        float *Bn) {
    const MlpFusedArgs &a = *S.a;
    if (u + 1 < S.tiles) mf_issue(S, u + 1, Wn, Bn);
    // the accumulators start from the bias of their outputs (output 32 i +
    // 8 g + 4 lh + q in element 4 g + q of acc[i]): no add per element after
    // the products.  Bias words past a final layer's n_out are whatever the
    // buffer held; their outputs are not stored.
    floatx16_t acc[4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const floatx4_t bv = *(const floatx4_t *)&Bc[32 * i + 8 * g + 4 * S.lh];
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[i][4 * g + q] = bv[q];
        }
    if (FINAL && u == 2 * a.n_hidden) {
        mf_products<2>(S, Wc, 16, acc);
        // outputs 32 i + 8 g + 4 lh + q of this lane's row
        if (S.row < a.B) {
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const int f = 32 * i + 8 * g + 4 * S.lh;
                    if (f < a.n_out) {
                        floatx4_t v;
#pragma unroll
                        for (int q = 0; q < 4; ++q) v[q] = acc[i][4 * g + q];
                        *(floatx4_t *)(a.out + (int64_t)S.row * a.ldo + f) = v;
                    }
                }
        }
    } else {
        const int l = u >> 1, hf = u & 1;
        mf_products<4>(S, Wc, l == 0 ? a.k_in / 16 : 16, acc);
        const bool out_h = !FINAL && l == a.n_hidden - 1;
        // GELU + bf16: outputs 128 hf + 32 i + 8 g + 4 lh + q become
        // element 4 (g & 1) + q of the next layer's K step 8 hf + 2 i + (g >> 1)
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                float y[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) y[q] = gelu_poly(acc[i][4 * g + q]);
                const uint32_t lo = pack_bf16x2(y[0], y[1]), hi = pack_bf16x2(y[2], y[3]);
                u32x4_t &t = S.hn[8 * hf + 2 * i + (g >> 1)];
                t[2 * (g & 1)] = lo;
                t[2 * (g & 1) + 1] = hi;
                if (out_h && S.row < a.B)
                    *(uint2 *)(a.h + (int64_t)S.row * a.ldh + 128 * hf + 32 * i + 8 * g + 4 * S.lh) = make_uint2(lo, hi);
            }
        if (hf == 1) {
#pragma unroll
            for (int kk = 0; kk < 16; ++kk) S.hb[kk] = S.hn[kk];
        }
    }
    __builtin_amdgcn_s_waitcnt(0);                  // this wave's copies into LDS have landed
    __syncthreads();
}

template <bool FINAL>
__global__ void __launch_bounds__(512, 1) mlp_fused_kernel(MlpFusedArgs a) {
    __shared__ __attribute__((aligned(1024))) GfTile W0, W1;
    __shared__ __attribute__((aligned(16))) float B0[GF_NT], B1[GF_NT];
    MfState S;
    S.a = &a;
    S.tid = threadIdx.x;
    S.wave = __builtin_amdgcn_readfirstlane(S.tid >> 6);     // wave-uniform: scalar registers
    S.lane = S.tid & 63;
    S.lc = S.lane & 31;
    S.lh = S.lane >> 5;
    S.row = blockIdx.x * GF_ROWS + S.wave * 32 + S.lc;
    S.tiles = 2 * a.n_hidden + (FINAL ? 1 : 0);
    // the first layer's inputs: k = 16 kk + 8 lh .. + 8 of this lane's row
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
        u32x4_t v = {0u, 0u, 0u, 0u};
        if (S.row < a.B && 16 * kk < a.k_in) v = *(const u32x4_t *)(a.x + (int64_t)S.row * a.ldx + 16 * kk + 8 * S.lh);
        S.hb[kk] = v;
    }
    mf_issue(S, 0, W0, B0);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    for (int u = 0; u < S.tiles; u += 2) {
        mf_tile<FINAL>(S, u, W0, B0, W1, B1);
        if (u + 1 < S.tiles) mf_tile<FINAL>(S, u + 1, W1, B1, W0, B0);
    }
}

hipError_t launch_mlp_fused(const MlpFusedArgs &a, hipStream_t s) {
    const dim3 grid((unsigned)((a.B + GF_ROWS - 1) / GF_ROWS)), block(512);
    if (a.n_out > 0) hipLaunchKernelGGL(mlp_fused_kernel<true>, grid, block, 0, s, a);
    else hipLaunchKernelGGL(mlp_fused_kernel<false>, grid, block, 0, s, a);
    return hipGetLastError();
}

// wt[n][k'] = bf16(W[k][n]) for k' = permute ? mlp_permute_k(k) : k: the
// transposed weights of a layer of the fused forward pass (W float [in][out])
__global__ void mlp_weights_kernel(int in, int out, const float *W, int permute, uint16_t *wt) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)in * out) return;
    const int n = (int)(t / in), kp = (int)(t - (int64_t)n * in);
    const int k = permute ? mlp_permute_k(kp) : kp;
    wt[t] = f2bf(W[(int64_t)k * out + n]);
}

hipError_t launch_mlp_weights(int in, int out, const float *W, int permute, uint16_t *wt, hipStream_t s) {
    const int64_t n = (int64_t)in * out;
    hipLaunchKernelGGL(mlp_weights_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, in, out, W, permute,
                       wt);
    return hipGetLastError();
}

hipError_t launch_gate_fused(int B, int K, int D, int L, const uint16_t *h, int ldh, const uint16_t *wt, int ldw,
                             const float *bias, const float *e0, float y_scale, float s_clamp, float *partial,
                             float *layer_e, float *unc, float rho, uint32_t row_base, uint64_t seed,
                             float cnt_thr, float *layer_cnt, const hipEvent_t *ev, hipStream_t s) {
    // ev (optional): four events recorded before the products, between the
    // mean and the log-variance tiles, after the products and after the gate
    GemmArgs g{};
    g.M = B;
    g.N = 2 * D;
    g.K = K;
    g.A = h;
    g.lda = ldh;
    g.B = wt;
    g.ldb = ldw;
    g.bias = bias;
    g.C = partial;
    g.split = D;
    g.s_clamp = s_clamp;
    // a bin is occupied when its energy mu * e0 / y_scale exceeds cnt_thr
    g.e0 = layer_cnt ? e0 : nullptr;
    g.cnt_scale = cnt_thr * y_scale;
    auto mark = [&](int i) { return ev ? hipEventRecord(ev[i], s) : hipSuccess; };
    if (hipError_t e = mark(0); e != hipSuccess) return e;
    if (K == GF_K) {
        // the mean tiles, then the log-variance tiles
        constexpr int JW = GF_JW;
        const dim3 grid((unsigned)((B + GF_ROWS - 1) / GF_ROWS)), block(512 / JW);
        const int tm = D / GF_NT, tiles = 2 * D / GF_NT;
        if (layer_cnt) hipLaunchKernelGGL((gate_fused_k256_kernel<2, JW>), grid, block, 0, s, g, 0, tm);
        else hipLaunchKernelGGL((gate_fused_k256_kernel<1, JW>), grid, block, 0, s, g, 0, tm);
        if (hipError_t e = mark(1); e != hipSuccess) return e;
        hipLaunchKernelGGL((gate_fused_k256_kernel<3, JW>), grid, block, 0, s, g, tm, tiles);
    } else {
        hipError_t e = launch_gemm(0, 1, EPI_GATE, g, s);
        if (e != hipSuccess) return e;
        if (e = mark(1); e != hipSuccess) return e;
    }
    if (hipError_t e = hipGetLastError(); e != hipSuccess) return e;
    if (hipError_t e = mark(2); e != hipSuccess) return e;
    hipLaunchKernelGGL(gate_tiles_kernel, dim3((unsigned)((B + 3) / 4)), dim3(256), 0, s, B, D, L, partial, e0,
                       y_scale, layer_e, unc, rho, row_base, (uint32_t)seed, (uint32_t)(seed >> 32), layer_cnt);
    if (hipError_t e = hipGetLastError(); e != hipSuccess) return e;
    return mark(3);
}

hipError_t launch_transpose_bf16(int rows, int cols, const float *x, uint16_t *y, hipStream_t s) {
    hipLaunchKernelGGL(transpose_bf16_kernel, dim3((unsigned)((cols + 31) / 32), (unsigned)((rows + 31) / 32)),
                       dim3(32, 8), 0, s, rows, cols, x, y);
    return hipGetLastError();
}

hipError_t launch_nll(int B, int D, const float *out, const float *img, const float *e0,
                      float y_scale, float s_clamp, int mse_mean, uint16_t *dout, float *loss,
                      hipStream_t s) {
    const int64_t total = (int64_t)B * D;
    const int blocks = (int)std::min<int64_t>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(nll_kernel, dim3(blocks), dim3(256), 0, s, B, D, out, img, e0, y_scale,
                       s_clamp, mse_mean, dout, loss);
    return hipGetLastError();
}

int64_t colsum_scratch_floats(int M, int N) { return (int64_t)((M + CS_ROWS - 1) / CS_ROWS) * N; }

hipError_t launch_colsum(int M, int N, const uint16_t *X, int ld, float *out, float *scratch, hipStream_t s) {
    if (!scratch) {
        hipLaunchKernelGGL(colsum_kernel, dim3((N + 255) / 256), dim3(256), 0, s, M, N, X, ld, out);
        return hipGetLastError();
    }
    const int slices = (M + CS_ROWS - 1) / CS_ROWS;
    hipLaunchKernelGGL(colsum_part_kernel, dim3((N + 63) / 64, slices), dim3(256), 0, s, M, N, X, ld, scratch);
    hipLaunchKernelGGL(colsum_final_kernel, dim3((N + 255) / 256), dim3(256), 0, s, slices, N, scratch, out);
    return hipGetLastError();
}

hipError_t launch_adam(int64_t n, float *p, const float *g, float *m, float *v, uint16_t *pb,
                       float lr, float b1, float b2, float eps, int step, hipStream_t s) {
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, p, g, m,
                       v, pb, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_to_bf16(int64_t n, const float *x, uint16_t *y, hipStream_t s) {
    hipLaunchKernelGGL(to_bf16_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, x, y);
    return hipGetLastError();
}

hipError_t launch_features(int B, int ld, int n_noise, const float *e0, const float *polar,
                           const float *az, float e_scale, float polar_scale, float az_scale,
                           uint32_t row_base, uint32_t stream, uint64_t seed, uint16_t *x,
                           hipStream_t s) {
    if (ld == 32 && n_noise == 16 && ((uintptr_t)x & 15) == 0) {
        hipLaunchKernelGGL(features32_kernel<16>, dim3((B + 127) / 128), dim3(128), 0, s, B, e0, polar, az, e_scale,
                           polar_scale, az_scale, row_base, stream, (uint32_t)seed, (uint32_t)(seed >> 32), x);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(features_kernel, dim3((B + 127) / 128), dim3(128), 0, s, B, ld, n_noise, e0,
                       polar, az, e_scale, polar_scale, az_scale, row_base, stream, (uint32_t)seed,
                       (uint32_t)(seed >> 32), x);
    return hipGetLastError();
}

// The gate of an output with one bin per layer (a per-layer head: [mean of
// each layer | log-variance of each layer]): one thread per shower, the same
// quantities as gate_kernel (with one bin the layer's sd is its sigma for
// every rho, and the same Philox counters give z).  A wave's 64 rows pass
// through LDS in both directions, so that global reads and writes are
// contiguous; rows are padded to an odd length against bank conflicts, and
// a row's outputs overwrite its means (layer l's mean is read before its
// output is written), which keeps the LDS per workgroup small enough for
// about fifteen waves per CU.  The layers' Philox blocks are independent:
// the loop is unrolled by four so that their work interleaves.
constexpr int GR_ROWS = 64;

__global__ void __launch_bounds__(GR_ROWS) gate_rows_kernel(int B, int L, const float *out, const float *e0,
                                                            float y_scale, float s_clamp, float *layer_e, float *unc,
                                                            float rho, uint32_t row_base, uint32_t k0, uint32_t k1) {
    extern __shared__ float gr_lds[];
    const int in_ld = 2 * L + 1, out_ld = in_ld;
    float *tin = gr_lds, *tout = gr_lds;
    const int b0 = blockIdx.x * GR_ROWS;
    const int rows = min(GR_ROWS, B - b0);
    const float *src = out + (int64_t)b0 * 2 * L;
    for (int i = threadIdx.x; i < rows * 2 * L; i += GR_ROWS) {
        const int r = i / (2 * L);
        tin[r * in_ld + (i - r * 2 * L)] = src[i];
    }
    __syncthreads();
    const int r = threadIdx.x;
    if (r < rows) {
        const int b = b0 + r;
        const float *row = tin + r * in_ld;
        const float scale = e0[b] / y_scale;
        float tm = 0.f, tv = 0.f;
#pragma unroll 4
        for (int l = 0; l < L; ++l) {
            const float mu = row[l];
            const float sv = fminf(fmaxf(row[L + l], -s_clamp), s_clamp);
            float v = mu;
            if (rho >= 0.0f) {
                const uint4 w = philox4x32_10(row_base + (uint32_t)b, (uint32_t)l, 0x9a7eu, 0u, k0, k1);
                const float u1 = ((float)w.x + 0.5f) * 0x1p-32f, u2 = ((float)w.y + 0.5f) * 0x1p-32f;
                float sn, cs;
                sincospif(2.0f * u2, &sn, &cs);
                const float z = sqrtf(-2.0f * logf(u1)) * cs;
                v += __expf(0.5f * sv) * z;
            }
            tout[r * out_ld + l] = v * scale;
            tm += mu;
            tv += __expf(sv);
        }
        unc[b] = sqrtf(tv) / fmaxf(tm, 1e-6f);
    }
    __syncthreads();
    float *dst = layer_e + (int64_t)b0 * L;
    for (int i = threadIdx.x; i < rows * L; i += GR_ROWS) {
        const int rr = i / L;
        dst[i] = tout[rr * out_ld + (i - rr * L)];
    }
}

hipError_t launch_gate(int B, int D, int L, const float *out, const float *e0, float y_scale,
                       float s_clamp, float *layer_e, float *unc, float *img, float rho,
                       uint32_t row_base, uint64_t seed, hipStream_t s) {
    if (D == L && L <= 64 && !img) {
        const size_t lds = (size_t)GR_ROWS * (2 * L + 1) * sizeof(float);      // <= 33 KB for L <= 64
        hipLaunchKernelGGL(gate_rows_kernel, dim3((unsigned)((B + GR_ROWS - 1) / GR_ROWS)), dim3(GR_ROWS), lds, s, B,
                           L, out, e0, y_scale, s_clamp, layer_e, unc, rho, row_base, (uint32_t)seed,
                           (uint32_t)(seed >> 32));
        return hipGetLastError();
    }
    hipLaunchKernelGGL(gate_kernel, dim3(B), dim3(256), 0, s, B, D, L, out, e0, y_scale, s_clamp,
                       layer_e, unc, img, rho, row_base, (uint32_t)seed, (uint32_t)(seed >> 32));
    return hipGetLastError();
}

}  // namespace supa

namespace supa {

// ---------------------------------------------------------------------------
// Fallback selection: indices i with v[i] > tau, in increasing order
// (deterministic): per-block counts, one-block scan of the counts, write.
// ---------------------------------------------------------------------------
constexpr int SEL_THREADS = 1024;

__global__ void select_count_kernel(int n, const float *v, float tau, int32_t *block_counts) {
    const int i = blockIdx.x * SEL_THREADS + threadIdx.x;
    const bool p = i < n && v[i] > tau;
    __shared__ int total;
    if (threadIdx.x == 0) total = 0;
    __syncthreads();
    const uint64_t m = __ballot(p);
    if ((threadIdx.x & 63) == 0) atomicAdd(&total, (int)__popcll(m));
    __syncthreads();
    if (threadIdx.x == 0) block_counts[blockIdx.x] = total;
}

__global__ void select_scan_kernel(int blocks, int32_t *block_counts, int32_t *count) {
    // exclusive scan in place, one thread block of SEL_THREADS, serial over chunks
    __shared__ int buf[SEL_THREADS];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < blocks; base += SEL_THREADS) {
        const int i = base + threadIdx.x;
        const int v = i < blocks ? block_counts[i] : 0;
        buf[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < SEL_THREADS; off <<= 1) {
            const int t = (int)threadIdx.x >= off ? buf[threadIdx.x - off] : 0;
            __syncthreads();
            buf[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < blocks) block_counts[i] = carry + buf[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == 0) carry += buf[SEL_THREADS - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0) *count = carry;
}

__global__ void select_write_kernel(int n, const float *v, float tau, const int32_t *block_offsets,
                                    int32_t *idx) {
    const int i = blockIdx.x * SEL_THREADS + threadIdx.x;
    const bool p = i < n && v[i] > tau;
    __shared__ int wave_base[SEL_THREADS / 64];
    const uint64_t m = __ballot(p);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) wave_base[w] = (int)__popcll(m);
    __syncthreads();
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int q = 0; q < SEL_THREADS / 64; ++q) {
            const int c = wave_base[q];
            wave_base[q] = acc;
            acc += c;
        }
    }
    __syncthreads();
    if (p) idx[block_offsets[blockIdx.x] + wave_base[w] + (int)lanes_below(m)] = i;
}

// gather float arrays by index: out_k[j] = in_k[idx[j]] for three arrays
__global__ void gather3_kernel(int m, const int32_t *idx, const float *a, const float *b,
                               const float *c, float *oa, float *ob, float *oc) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    const int i = idx[j];
    oa[j] = a[i];
    ob[j] = b[i];
    oc[j] = c[i];
}

// rows: dst[idx[j]][0..w) = src[j][0..w)
__global__ void scatter_rows_kernel(int m, int w, const int32_t *idx, const float *src, float *dst) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)m * w) return;
    const int j = (int)(t / w), c = (int)(t - (int64_t)j * w);
    dst[(int64_t)idx[j] * w + c] = src[t];
}

// per-row sums of groups: out[b][l] = sum_{q < g} x[b][l*g + q]
// one wave per group: its lanes read the group's g values with unit stride
// (coalesced) and the partial sums meet in a butterfly reduction
constexpr int GS_WAVES = 4;
__global__ void __launch_bounds__(64 * GS_WAVES) group_sums_kernel(int rows, int L, int g, const float *x,
                                                                  float *out) {
    const int64_t t = (int64_t)blockIdx.x * GS_WAVES + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (t >= (int64_t)rows * L) return;              // whole waves leave together
    const float *p = x + t * g;
    float s = 0.f;
    for (int q = lane; q < g; q += 64) s += p[q];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) out[t] = s;
}

hipError_t launch_select(int n, const float *v, float tau, int32_t *idx, int32_t *count,
                         int32_t *block_scratch, hipStream_t s) {
    const int blocks = (n + SEL_THREADS - 1) / SEL_THREADS;
    if (blocks == 0) {
        hipLaunchKernelGGL(select_scan_kernel, dim3(1), dim3(SEL_THREADS), 0, s, 0, block_scratch, count);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(select_count_kernel, dim3(blocks), dim3(SEL_THREADS), 0, s, n, v, tau, block_scratch);
    hipLaunchKernelGGL(select_scan_kernel, dim3(1), dim3(SEL_THREADS), 0, s, blocks, block_scratch, count);
    hipLaunchKernelGGL(select_write_kernel, dim3(blocks), dim3(SEL_THREADS), 0, s, n, v, tau,
                       block_scratch, idx);
    return hipGetLastError();
}

hipError_t launch_gather3(int m, const int32_t *idx, const float *a, const float *b, const float *c,
                          float *oa, float *ob, float *oc, hipStream_t s) {
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(gather3_kernel, dim3((m + 255) / 256), dim3(256), 0, s, m, idx, a, b, c, oa, ob, oc);
    return hipGetLastError();
}

hipError_t launch_scatter_rows(int m, int w, const int32_t *idx, const float *src, float *dst,
                               hipStream_t s) {
    const int64_t t = (int64_t)m * w;
    if (t <= 0) return hipSuccess;
    hipLaunchKernelGGL(scatter_rows_kernel, dim3((unsigned)((t + 255) / 256)), dim3(256), 0, s, m, w,
                       idx, src, dst);
    return hipGetLastError();
}

hipError_t launch_group_sums(int rows, int L, int g, const float *x, float *out, hipStream_t s) {
    const int64_t t = (int64_t)rows * L;
    if (t <= 0) return hipSuccess;
    hipLaunchKernelGGL(group_sums_kernel, dim3((unsigned)((t + GS_WAVES - 1) / GS_WAVES)), dim3(64 * GS_WAVES),
                       0, s, rows, L, g, x, out);
    return hipGetLastError();
}

}  // namespace supa
