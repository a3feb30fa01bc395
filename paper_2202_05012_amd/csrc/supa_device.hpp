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
        const uint32_t m0 = 0xD2511F53u, m1 = 0xCD9E8D57u;
        const uint32_t hi0 = __umulhi(m0, c0), lo0 = m0 * c0;
        const uint32_t hi1 = __umulhi(m1, c2), lo1 = m1 * c2;
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
struct Params {
    // process
    int32_t n_planes;
    int32_t n_layers;
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
    // batch
    const float *e0, *polar, *azimuth, *x0, *y0;
    int32_t n;
    uint32_t sid_base;
    const int32_t *order;       // work order (permutation of 0..n-1) or null
    // outputs
    uint32_t outputs;
    int64_t *hit_offsets;
    float *hit_x, *hit_y, *hit_e;
    int32_t *hit_layer;
    uint64_t *hit_key;
    int64_t hit_capacity;
    float *images;
    int32_t img_nx, img_ny;
    float img_x0, img_y0, img_sx, img_sy;   // cell = floor((x - x0) * sx)
    int32_t img_rows;                       // image rows binned per LDS pass
    int64_t *node_offsets;
    int32_t *node_parent, *node_gen;
    float *node_vx, *node_vy, *node_vz, *node_e;
    uint64_t *node_key;
    int64_t node_capacity;
    uint64_t *ledger;
    int32_t *counts;
    // per-wave scratch (structure of arrays, wave w owns slice w)
    int32_t cap_f, cap_h, cap_n;
    float *fx, *fy, *ftx, *fty;               // [waves][2][cap_f]
    uint32_t *fe, *fplo, *fphi;
    int32_t *fnode;
    float *jhx, *jhy;                         // hit journal [waves][cap_h]
    uint32_t *jhe;
    int32_t *jhl;
    uint32_t *jhplo, *jhphi;
    int32_t *jnp, *jng;                       // node journal [waves][cap_n]
    float *jnx, *jny, *jnz;
    uint32_t *jne, *jnplo, *jnphi;
    // device counters, zeroed before each launch
    unsigned long long *ctr;                  // see CTR_* below
};

enum {
    CTR_WORK = 0,        // next work item
    CTR_HITS = 1,        // hits allocated
    CTR_NODES = 2,       // nodes allocated
    CTR_STEPS = 3,       // particle-steps
    CTR_FLAGS = 4,       // bit 0: scratch overflow, bit 1: energy out of range
    CTR_NEED_F = 5,      // largest frontier seen
    CTR_NEED_H = 6,      // largest per-shower hit count seen
    CTR_NEED_N = 7,      // largest per-shower node count seen
    CTR_COUNT = 8
};

enum { FLAG_OVERFLOW = 1, FLAG_RANGE = 2 };

}  // namespace supa
