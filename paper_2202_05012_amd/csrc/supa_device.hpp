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
        // three-input xors, one v_bitop3_b32 each (truth table 0x96 = a ^ b ^ c)
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32(hi1, c1, k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32(hi0, c3, k1, 0x96);
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
// Inputs and outputs the propagation kernel touches once per shower.  They
// live in device memory and are read at their point of use, so that they do
// not occupy scalar registers through the hot loop.
struct Cold {
    const float *e0, *polar, *azimuth, *x0, *y0;
    const int32_t *order;       // work order (permutation of 0..n-1) or null
    uint64_t *ledger;           // [n][4]
    int32_t *counts;            // [n][6]
    int64_t *hstart;            // [n]: log position of the shower's first hit record
    float ring_r[4];            // ring radii (regional parameters), +inf past the last
    unsigned long long *wave_clk;   // per wave: wall-clock start and end of its work, or null
};

// Hit records leave the propagation kernel through a log of chunks of
// HIT_CHUNK records: per record 12 bytes {x, y, integer energy}, its plane in
// a byte array of the chunk (the placement counts hits per plane from the
// bytes alone), and with keys the path id in a third array.  Each
// shower slot of a wave fills its own chain of chunks: when the slot's chunk
// is full the next one is claimed with one atomic and linked from it, so the
// records of one shower follow each other along the chain, starting at the
// position (chunk * HIT_CHUNK + offset) noted when the shower started.  The
// placement kernel walks each shower's chain once.
constexpr int HIT_CHUNK_LOG2 = 10;
constexpr int HIT_CHUNK = 1 << HIT_CHUNK_LOG2;
constexpr int HIT_REC_WORDS = 3;                  // x, y, e
constexpr int HIT_KEY_WORDS = 2;                  // path id low, high
constexpr int HIT_PLANE_OFF = HIT_REC_WORDS * HIT_CHUNK;          // plane bytes (words from the chunk start)
constexpr int HIT_KEY_OFF = HIT_PLANE_OFF + HIT_CHUNK / 4;        // path ids
constexpr int64_t HIT_CHUNK_WORDS = HIT_KEY_OFF + (int64_t)HIT_KEY_WORDS * HIT_CHUNK;

// Tree nodes go to a log of chunks of LOG_CHUNK records that a wave fills in
// the order its phases produce them (a chunk is claimed with one atomic and
// its fill count written when it is closed); the scatter kernel moves every
// record to its place once all showers are counted.
constexpr int LOG_CHUNK = 2048;
// A node record holds the two daughters of one split, nodes IDX and IDX + 1
// (IDX odd), which share shower, parent, generation, plane and vertex, or
// the primary (IDX 0, one node): shower index, IDX, parent index,
// generation | plane << 8 (plane 255: the primary, vertex z = 0), vertex x
// and y, the integer energies of node IDX and of node IDX + 1, and with keys
// the path id of node IDX (node IDX + 1: the same with the low bit set).
enum { NL_I = 0, NL_IDX, NL_PARENT, NL_GK, NL_X, NL_Y, NL_E, NL_E2, NL_LO, NL_HI, NL_FIELDS };
constexpr uint32_t GK_PRIMARY = 255u << 8;

// Parameters of one simulate call that the hot loop reads, by value.
struct Params {
    int32_t n_planes;
    float z_first, dz;          // flight lengths: first plane from z = 0, then dz
    const uint64_t *c1, *c2;    // [n_planes] stop / split thresholds (<= 2^32)
    uint64_t t_cut;             // energy threshold in fixed point
    uint32_t f_lo;              // energy fraction F = f_lo + floor(w1 * f_w / 2^32)
    uint64_t f_w;
    int32_t angle_mode;
    float angle_a, angle_b;
    float e_scale;              // 2^s
    uint32_t seed_lo, seed_hi;
    int32_t n;                  // showers in the batch
    uint32_t sid_base;
    uint32_t outputs;
    bool keys;                  // write path ids of hits and nodes
    const Cold *cold;
    int32_t pool_cap;           // particle-pool entries kept in LDS (power of 2, >= 128)
    int32_t spill_cap;          // pool entries per wave that can spill to global memory
    uint32_t *spill;            // per wave: POOL_FIELDS x spill_cap
    uint32_t *hlog, *hnext;     // hit log: h_chunks x HIT_CHUNK_WORDS; chain links
    uint32_t *nlog, *nfill;     // node log: n_chunks x NL_FIELDS x LOG_CHUNK; fill counts
    int32_t h_chunks, n_chunks;
    unsigned long long *ctr;    // the call's counters (CTR_*)
    unsigned long long *sub;    // the sub-batch's counters (SUB_*)
    // subtree work items (section "Propagation Model": a particle's subtree
    // depends only on its own state and path id, so it can be finished by
    // any wave).  Launch `phase` 0 runs the showers; launch p >= 1 runs the
    // items that launch p-1 exported.  Launches before `last_phase` export
    // pending particles of a shower whose pool holds export_top + WAVE or
    // more entries; export_top < 0 disables it.
    int32_t phase, last_phase, export_top;
    uint32_t *items;            // two regions of item_cap items, ITEM_WORDS each
    int32_t item_cap;
    uint32_t *shares;           // share_cap records of SHARE_WORDS
    int32_t share_cap;
    float share_margin;         // hit-log chunks reserved per shared shower / expected
};

// Offsets of the showers' segments: exclusive prefix sums of their hit and
// node counts in batch order (supa_scatter.hip).
struct ScanParams {
    int32_t n;
    const int32_t *counts;      // [n][6]: [0] nodes, [1] hits
    int64_t *hoff, *noff;       // [n] outputs (either may be null)
    int64_t *partial;           // [2][ceil(n / SCAN_TILE)] tile sums, then tile offsets
    unsigned long long *sub;    // SUB_HITS / SUB_NODES receive the running totals
    const unsigned long long *prev;   // the previous sub-batch's counters, or null
};
constexpr int SCAN_THREADS = 256, SCAN_ITEMS = 16, SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

// Moves node records to their final places (supa_scatter.hip).
struct ScatterParams {
    float z_first, dz, e_unscale;
    const unsigned long long *ctr;    // the call's counters (flags)
    const unsigned long long *sub;    // the sub-batch's (node total, end of its chunks)
    const unsigned long long *prev;   // the previous sub-batch's (start of its chunks), or null
    const uint32_t *nlog, *nfill;
    int32_t n_chunks;
    const int64_t *noff;        // [n] segment starts of the nodes
    int64_t ncap;
    int32_t *np, *ng;
    float *nvx, *nvy, *nvz, *ne;
    uint64_t *nk;               // path ids (or null)
};

// Per shower: hit records from the log to the output arrays (grouped by
// plane) and per-layer images binned from them (supa_place.hip).
struct PlaceParams {
    int32_t n, n_planes, L, nx, ny;
    float x0, y0, sx, sy;        // cell = floor((x - x0) * sx)
    float e_unscale;             // 2^-s
    const unsigned long long *ctr;    // the call's counters (flags)
    const unsigned long long *sub;    // the sub-batch's (running hit total)
    const int32_t *counts;       // [n][6]: [1] hits
    const int64_t *hstart;       // [n] log position of each shower's first record
    const uint32_t *hlog, *hnext;
    int32_t h_chunks;
    const int32_t *layer;        // [n_planes]
    const int64_t *hoff;         // [n] segment starts (with hit outputs)
    int64_t hcap;
    float *hx, *hy, *he;         // hit outputs, or null
    int32_t *hl;
    uint64_t *hk;                // path ids, or null
    float *images;               // [n][L][ny][nx], or null
    int32_t slab_rows;           // image rows binned per LDS pass
    uint2 *bucket;               // per workgroup bucket_cap entries: a shower's binned
    int32_t bucket_cap;          //   hits sorted by slab (images of many slabs), or null
};

// Device counters of one call: a block for the whole call, then one block
// per sub-batch (a call runs its batch as up to MAX_SUB consecutive
// sub-batches, so that the placement of one overlaps the propagation of the
// next).
enum {
    CTR_STEPS = 0,       // particle-steps
    CTR_FLAGS = 1,       // FLAG_* bits
    CTR_NEED_F = 2,      // largest particle pool seen
    CTR_HCHUNK = 3,      // hit-log chunks claimed
    CTR_NCHUNK = 4,      // node-log chunks claimed
    CTR_BLOCK = 8        // words per block
};
enum {
    SUB_WORK = 0,        // next work item of the sub-batch
    SUB_HITS = 1,        // hits of the batch up to and including this sub-batch
    SUB_NODES = 2,       // the same for nodes
    SUB_NCHUNK_END = 3   // node-log chunks claimed when the sub-batch's propagation ended
};
constexpr int MAX_SUB = 8;
// Subtree work items: after the sub-batch blocks, the shares handed out,
// then per launch phase the items it exported and the items claimed from it.
constexpr int MAX_PHASES = 4;
constexpr int CTR_ST = CTR_BLOCK * (1 + MAX_SUB);
constexpr int CTR_ST_SHARES = CTR_ST;
__host__ __device__ constexpr int ctr_st_out(int phase) { return CTR_ST + 1 + phase; }
__host__ __device__ constexpr int ctr_st_claim(int phase) { return CTR_ST + 1 + MAX_PHASES + phase; }
constexpr int CTR_WORDS = CTR_ST + 1 + 2 * MAX_PHASES;

enum { FLAG_OVERFLOW = 1, FLAG_RANGE = 2, FLAG_INTERNAL = 4, FLAG_SHARE = 8 };

// A shared shower: one whose pending particles were handed to other waves as
// work items.  Every party (the wave that started the shower, and each item)
// adds its tallies here when its last particle is done; the party that
// brings `SH_OUT` to zero writes the shower's ledger, counts and log start.
// Hit records of all parties continue the shower's run of the log: from the
// conversion point (SH_CONV_C, SH_CONV_F) to the end of that chunk, then
// through SH_KCAP chunks reserved and linked at conversion (SH_BASE ...), at
// positions taken from SH_FILL.  With a tree, node indices come from SH_NODES.
enum {
    SH_I = 0, SH_SID, SH_E0, SH_HS_LO, SH_HS_HI, SH_FILL, SH_CONV_C, SH_CONV_F, SH_BASE, SH_KCAP,
    SH_NODES, SH_HITS, SH_PASSES, SH_ESC, SH_BACK, SH_EESC, SH_ECUT, SH_ESTOP, SH_OUT, SH_FIELDS
};
constexpr int SHARE_WORDS = 32;
static_assert(SH_FIELDS <= SHARE_WORDS, "share record fits");
// An item: up to 64 pending particles of one shared shower, as pool fields
// [POOL_FIELDS][64] (KS = plane | share << 8), then the count.
constexpr int ITEM_WORDS = 9 * 64 + 1;
constexpr int ITEM_MIN = 16;          // fewer particles of one shower are not exported

// true when the propagation of this call failed (its outputs are rerun or
// discarded): the later kernels then write nothing
__device__ __forceinline__ bool batch_failed(const unsigned long long *ctr) {
    return (ctr[CTR_FLAGS] & (unsigned long long)(FLAG_OVERFLOW | FLAG_RANGE | FLAG_INTERNAL | FLAG_SHARE)) != 0;
}

constexpr int SLOTS = 4;              // showers in flight per wave
constexpr int QCAP = 128;             // draw-queue entries per wave

// fields of a pending particle (pool, draw queue, spill); KS = plane | slot << 8
enum { PF_X = 0, PF_Y, PF_TX, PF_TY, PF_E, PF_LO, PF_HI, PF_NODE, PF_KS, POOL_FIELDS };
static_assert(ITEM_WORDS == POOL_FIELDS * 64 + 1, "item layout");

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

// sin and cos of the azimuth omega = 2 pi u(w) of a split: (signed w + 1/2)
// / 2^32 is the same angle mod 2 pi in revolutions, the argument the
// hardware sine and cosine take, so there is no range reduction (within
// 2.5e-7 of the exact values: tests/test_gpu_parity.py checks it against
// the definition in double precision)
__device__ __forceinline__ void azimuth_sincos(uint32_t w, float *s, float *c) {
    const float rev = ((float)(int32_t)w + 0.5f) * 0x1p-32f;
    *s = __builtin_amdgcn_sinf(rev);
    *c = __builtin_amdgcn_cosf(rev);
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
