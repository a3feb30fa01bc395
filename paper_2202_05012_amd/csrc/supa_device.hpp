// supa_device.hpp -- device-side building blocks of the SUPA propagation
// kernels for gfx950: the counter-based generator, the fixed-point energy
// split, the split kinematics and the wave-level (64-lane) compaction helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace supa {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of two 32x32
// multiplies whose high halves are mixed with the other counter words and the
// round key; the key advances by the golden-ratio and sqrt(3)-1 Weyl steps.
// The key is the run seed, so on a wave it lives in scalar registers.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                               uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32x32->64 multiply each (v_mad_u64_u32), not separate lo/hi
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return make_uint4(c0, c1, c2, c3);
}

// ---------------------------------------------------------------------------
// Wave helpers (wave64).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// number of set bits of `mask` below this lane
__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint64_t wave_ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ int wave_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ int wave_sum_i32(int v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// ---------------------------------------------------------------------------
// Parameters of one simulate call, passed by value to the kernels.
// ---------------------------------------------------------------------------
// Inputs and outputs used once per shower.  They live in device memory and
// are read at their point of use, so that they do not occupy scalar
// registers through the hot loop.
struct Cold {
    const float *e0, *polar, *azimuth, *x0, *y0;
    const int32_t *order;       // work order (permutation of 0..n-1) or null
    int64_t *hit_offsets;
    float *hit_x, *hit_y, *hit_e;
    int32_t *hit_layer;
    uint64_t *hit_key;
    int64_t hit_capacity;
    float *images;
    int32_t img_nx, img_ny;
    float img_x0, img_y0, img_sx, img_sy;   // cell = floor((x - x0) * sx)
    int32_t img_rows;                       // image rows binned per LDS pass
    int32_t n_layers;
    const int32_t *layer_plane_start;       // [n_layers + 1] CSR of the planes of each layer
    const int32_t *layer_planes;            // [n_planes]
    int64_t *node_offsets;
    int32_t *node_parent, *node_gen;
    float *node_vx, *node_vy, *node_vz, *node_e;
    uint64_t *node_key;
    int64_t node_capacity;
    uint64_t *ledger;
    int32_t *counts;
    // hand-over to the image kernel (library scratch): per shower the start and
    // number of its hits, per hit its integer energy, and its coordinates and
    // layer when the caller's hit arrays are not written
    int64_t *img_seg;           // [n] (when hits are not an output)
    int32_t *img_count;         // [n] hits handed over (0 when they were not written)
    uint32_t *img_e;            // [img_cap]
    float *img_x, *img_y;       // [img_cap] (when hits are not an output)
    int32_t *img_layer;
    int64_t img_cap;
};

// Parameters of one simulate call that the hot loop reads, by value.
struct Params {
    int32_t n_planes;
    float z_first, dz;          // flight lengths: first plane from z = 0, then dz
    const int32_t *layer;       // [n_planes]
    const uint64_t *c1, *c2;    // [n_planes] stop / split thresholds (<= 2^32)
    uint64_t t_cut;             // energy threshold in fixed point
    uint32_t f_lo;              // energy fraction F = f_lo + floor(w1 * f_w / 2^32)
    uint64_t f_w;
    int32_t angle_mode;
    float angle_a, angle_b;
    float e_scale;              // 2^s
    float e_unscale;            // 2^-s
    uint32_t seed_lo, seed_hi;
    int32_t n;                  // showers in the batch
    uint32_t sid_base;
    uint32_t outputs;
    bool keys;                  // write path ids of hits and nodes
    const Cold *cold;
    // per-wave scratch in global memory (wave w owns a contiguous slice)
    int32_t pool_cap;                         // particle-pool entries kept in LDS (power of 2, >= 128)
    int32_t tile_words;                       // LDS image tile size (32-bit words)
    int32_t spill_cap;                        // pool entries that can spill to global memory
    int32_t cap_h, cap_n;                     // per-shower hit / node journal capacity
    uint32_t *spill;                          // per wave: POOL_FIELDS x spill_cap
    uint32_t *jh;                             // per wave: SLOTS x JH_COUNT x cap_h
    uint32_t *hidx;                           // per wave: cap_h (plane-sorted hit order)
    uint32_t *jn;                             // per wave: SLOTS x JN_COUNT x cap_n
    unsigned long long *ctr;                  // device counters, see CTR_*
};

// Arguments of the surrogate's matrix product (supa_mlp.hip).
struct GemmArgs {
    int M, N, K;
    const uint16_t *A;   // TA == 0: [M][lda] (row-major M x K); TA == 1: [K][lda] (K x M)
    const uint16_t *B;   // TB == 0: [K][ldb] (K x N);           TB == 1: [N][ldb] (N x K)
    int lda, ldb;
    const float *bias;   // [N] or null
    void *C;             // float [M][ldc] (EPI_F32, EPI_BIAS_F32) or bf16 [M][ldc]
    int ldc;
    uint16_t *pre;       // EPI_BIAS_GELU: pre-activation out; EPI_GELU_GRAD: in (bf16 [M][ldc])
};

// Parameters of the image kernel (supa_images.hip).
struct ImgParams {
    int32_t n, L, nx, ny, n_planes;
    float x0, y0, sx, sy;        // cell = floor((x - x0) * sx)
    float e_unscale;             // 2^-s
    const int64_t *seg;          // [n] first hit of each shower
    const int32_t *count;        // [n] hits of each shower that were written
    int64_t cap;                 // entries of x, y, e, layer
    const float *x, *y;          // hit coordinates
    const uint32_t *e;           // integer hit energies
    const int32_t *layer;        // hit layers (-1: not read out)
    const int32_t *layer_plane_start, *layer_planes;   // planes of each layer (CSR)
    float *images;               // [n][L][ny][nx]
    int32_t slab_layers;         // whole layers per slab (0: bands of rows)
    int32_t slab_rows;           // rows per band when one layer does not fit
};

enum {
    CTR_WORK = 0,        // next work item
    CTR_HITS = 1,        // hits allocated
    CTR_NODES = 2,       // nodes allocated
    CTR_STEPS = 3,       // particle-steps
    CTR_FLAGS = 4,       // bit 0: scratch overflow, bit 1: energy out of range
    CTR_NEED_F = 5,      // largest particle pool seen
    CTR_NEED_H = 6,      // largest per-shower hit count seen
    CTR_NEED_N = 7,      // largest per-shower node count seen
    CTR_COUNT = 8
};

enum { FLAG_OVERFLOW = 1, FLAG_RANGE = 2, FLAG_INTERNAL = 4 };

constexpr int SLOTS = 4;              // showers in flight per wave
constexpr int QCAP = 128;             // draw-queue entries per wave

// fields of a pending particle (pool, draw queue, spill); KS = plane | slot << 8
enum { PF_X = 0, PF_Y, PF_TX, PF_TY, PF_E, PF_LO, PF_HI, PF_NODE, PF_KS, POOL_FIELDS };
// hit journal fields; PK = plane | KIND_STOP for stops
enum { JH_X = 0, JH_Y, JH_E, JH_LO, JH_HI, JH_PK, JH_COUNT };
constexpr uint32_t KIND_STOP = 0x100u;
// node journal fields
enum { JN_PARENT = 0, JN_GEN, JN_X, JN_Y, JN_Z, JN_E, JN_LO, JN_HI, JN_COUNT };

// ---------------------------------------------------------------------------
// Single-precision elementary functions for the split kinematics.
// ---------------------------------------------------------------------------
// sin and cos of r for |r| <= pi/4: Taylor series of sin to degree 9 and of
// cos to degree 10 (truncation below 2e-9), error about 1.5 ulp.
__device__ __forceinline__ void sincos_poly(float r, float *s, float *c) {
    const float r2 = r * r;
    float ps = fmaf(r2, 2.75573192e-06f, -1.98412698e-04f);
    ps = fmaf(r2, ps, 8.33333333e-03f);
    ps = fmaf(r2, ps, -1.66666667e-01f);
    *s = fmaf(r * r2, ps, r);
    float pc = fmaf(r2, -2.75573192e-07f, 2.48015873e-05f);
    pc = fmaf(r2, pc, -1.38888889e-03f);
    pc = fmaf(r2, pc, 4.16666667e-02f);
    pc = fmaf(r2, pc, -0.5f);
    *c = fmaf(r2, pc, 1.0f);
}

// sin and cos of any x met here: Cody-Waite reduction by pi/2 carried out in
// double (exact for the angles met here), the series above, and the quadrant.
__device__ __forceinline__ void sincos_f32(float x, float *s, float *c) {
    const float n = rintf(x * 0.636619772f);
    const float r = (float)fma(-(double)n, 1.5707963267948966, (double)x);
    float sr, cr;
    sincos_poly(r, &sr, &cr);
    const int q = (int)n;
    const float a = (q & 1) ? cr : sr;
    const float b = (q & 1) ? sr : cr;
    *s = (q & 2) ? -a : a;
    *c = ((q + 1) & 2) ? -b : b;
}

// -ln(u(w)) for u(w) = (w + 1/2) / 2^32 in (0, 1).  Below 1/2 through the
// hardware base-2 logarithm (accurate relative to |log2 u| >= 1); above, with
// v = 1 - u, as 2 atanh(t), t = v / (2 - v) <= 1/3, summed to t^15.
__device__ __forceinline__ float neg_log_unit(uint32_t w) {
    if (w < 0x80000000u) {
        const float u = ((float)w + 0.5f) * 0x1p-32f;
        return -__builtin_amdgcn_logf(u) * 0.693147181f;
    }
    const float v = ((float)(~w) + 0.5f) * 0x1p-32f;
    const float t = v * __builtin_amdgcn_rcpf(2.0f - v);
    const float t2 = t * t;
    float p = fmaf(t2, 1.0f / 15.0f, 1.0f / 13.0f);
    p = fmaf(t2, p, 1.0f / 11.0f);
    p = fmaf(t2, p, 1.0f / 9.0f);
    p = fmaf(t2, p, 1.0f / 7.0f);
    p = fmaf(t2, p, 1.0f / 5.0f);
    p = fmaf(t2, p, 1.0f / 3.0f);
    p = fmaf(t2, p, 1.0f);
    return 2.0f * t * p;
}

}  // namespace supa
