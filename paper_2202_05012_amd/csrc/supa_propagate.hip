// supa_propagate.hip -- the SUPA propagation kernel for gfx950.
//
// Each wave (64 lanes, one workgroup) keeps up to SLOTS showers in flight and
// pulls new ones from a device work queue, SLOTS at a time, whenever its work
// runs low, so one launch of a few waves per compute unit runs a whole batch
// however uneven its showers are.  A shower is the tree of Algorithm 1
// (section "Propagation Model": at each slice every live particle stops,
// splits or passes).  Every pending particle has already flown to the plane
// where it must draw, and sits, tagged with its shower slot and plane, in a
// per-wave pool in LDS (a stack: depth-first, so it stays small; its oldest
// entries spill to global memory only for very large showers).  One step
// takes up to 64 particles off the pool: one Philox block each, the three-way
// choice, the split kinematics; whatever goes on (daughters, passers) flies
// straight to the next plane, where it either deposits at once (below the
// energy threshold) or goes back on the pool.  So every lane of a step does
// the same work, and a particle costs one pool round trip per plane.
// Deposits become hit records in a log: each shower slot fills its own chain
// of log chunks (positions from a wave ballot and a count of the set lanes
// below), so a shower's records follow each other; the ledger sums live in
// registers.  When a shower's last particle is done the wave writes its
// ledger, counts and the log position of its first hit -- stores only.  The
// placement kernel (supa_place.hip) later puts the hits into the caller's
// arrays and bins the images; tree nodes go through a log of their own.
// Results depend only on (seed, shower id, path id): the random stream is
// keyed by the particle, not by the lane or wave that happens to process it.
// That also lets a shower be split: with subtree work items (SUB), a wave
// whose pool grows hands its oldest pending particles of one shower to a
// later launch as an item; any wave there finishes their subtrees, and the
// shower's tallies meet in a share record (supa_device.hpp).
#include "supa_device.hpp"

namespace supa {

constexpr int WAVE = 64;
// global-memory (address space 1) element types
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) uint32_t gu32;
typedef __attribute__((address_space(1))) uint8_t gu8;
typedef __attribute__((address_space(1))) u32x4 gu4;
typedef __attribute__((address_space(1))) u32x2 gu2;
// Read a field of the per-call Cold block at its point of use, as a global
// memory pointer (a plain pointer read from memory would be accessed with flat
// instructions, which also count against the LDS wait counter).
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T *as_global(T *p) {
    return (__attribute__((address_space(1))) T *)p;
}
#define COLD(field) as_global(((const volatile __attribute__((address_space(1))) Cold *)P.cold)->field)

struct Daughters {
    float txa, tya, txb, tyb;
    uint32_t ea, eb;
    bool fwd_a, fwd_b;
};

// Split of one particle (section "Propagation Model", split bullet; Algorithm 1,
// split branch): exact fixed-point energy split by the 32-bit fraction F drawn
// from w1, opening angle theta from w2, azimuth omega from w3; the daughters
// turn by theta*(1-f) and theta*f to opposite sides of the plane through the
// parent direction at azimuth omega (frame: rotation taking +z to d).
template <bool LIT>
__device__ __forceinline__ Daughters split_particle(const Params &P, float tx, float ty,
                                                    uint32_t e, uint4 w, uint32_t f_lo, uint64_t f_w) {
    Daughters D;
    const uint32_t F = f_lo + (uint32_t)(((uint64_t)w.y * f_w) >> 32);
    D.ea = (uint32_t)(((uint64_t)e * F) >> 32);
    D.eb = e - D.ea;
    const float f = (float)F * 0x1p-32f;     // fraction carried by daughter a
    const float g = 1.0f - f;

    float theta;
    if (P.angle_mode == 0) {
        theta = P.angle_a;
    } else if (P.angle_mode == 1) {
        theta = fmaf(P.angle_b - P.angle_a, ((float)w.z + 0.5f) * 0x1p-32f, P.angle_a);
    } else {
        // Rayleigh(sigma): sigma * sqrt(-2 ln u)
        theta = P.angle_a * __builtin_amdgcn_sqrtf(2.0f * neg_log_unit(w.z));
    }
    if constexpr (LIT) {
        // Algorithm 1 as printed: the daughters are displaced by
        // +-dz (sin(theta/2 + eps), cos(theta/2 + eps)), theta/2 + eps = f theta;
        // the flight to the next plane applies it as slopes, which are not kept
        float sl, cl;
        const float ang = theta * f;
        if (__ballot(ang > 0.785398163f) == 0ull) {
            sincos_poly(ang, &sl, &cl);
        } else {
            sincos_f32(ang, &sl, &cl);
        }
        D.txa = sl;
        D.tya = cl;
        D.txb = -sl;
        D.tyb = -cl;
        D.fwd_a = D.fwd_b = true;
        return D;
    }
    // omega = 2 pi u(w3) from the hardware sine and cosine (two instructions
    // instead of a range reduction and two polynomials): it only orients the
    // deflections, whose size the polynomials below set
    float so, co;
    azimuth_sincos(w.w, &so, &co);

    // unit direction from the slopes
    const float dz = __builtin_amdgcn_rsqf(1.0f + fmaf(tx, tx, ty * ty));
    const float dx = tx * dz, dy = ty * dz;
    const float c = __builtin_amdgcn_rcpf(1.0f + dz);
    const float e1x = fmaf(-dx * dx, c, 1.0f), e1y = -dx * dy * c, e1z = -dx;
    const float e2x = e1y, e2y = fmaf(-dy * dy, c, 1.0f), e2z = -dy;
    const float nx = co * e1x + so * e2x;
    const float ny = co * e1y + so * e2y;
    const float nz = co * e1z + so * e2z;

    // the two deflections are at most theta; the reduction to [-pi/4, pi/4]
    // is skipped when every splitting lane of the wave is already inside
    float sa, ca, sb, cb;
    if (__ballot(theta > 0.785398163f) == 0ull) {
        sincos_poly(theta * g, &sa, &ca);
        sincos_poly(theta * f, &sb, &cb);
    } else {
        sincos_f32(theta * g, &sa, &ca);
        sincos_f32(theta * f, &sb, &cb);
    }
    const float ax = ca * dx + sa * nx, ay = ca * dy + sa * ny, az = ca * dz + sa * nz;
    const float bx = cb * dx - sb * nx, by = cb * dy - sb * ny, bz = cb * dz - sb * nz;
    D.fwd_a = az > 0.0f;
    D.fwd_b = bz > 0.0f;
    const float ia = __builtin_amdgcn_rcpf(az), ib = __builtin_amdgcn_rcpf(bz);
    D.txa = ax * ia;
    D.tya = ay * ia;
    D.txb = bx * ib;
    D.tyb = by * ib;
    return D;
}


struct Entry {
    float x, y, tx, ty;
    uint32_t e, lo, hi;
    int32_t node;
    uint32_t ks;        // plane | slot << 8
};

__device__ __forceinline__ Entry load_entry(const uint32_t *base, int64_t fstride, int64_t j) {
    Entry p;
    p.x = __uint_as_float(base[PF_X * fstride + j]);
    p.y = __uint_as_float(base[PF_Y * fstride + j]);
    p.tx = __uint_as_float(base[PF_TX * fstride + j]);
    p.ty = __uint_as_float(base[PF_TY * fstride + j]);
    p.e = base[PF_E * fstride + j];
    p.lo = base[PF_LO * fstride + j];
    p.hi = base[PF_HI * fstride + j];
    p.node = (int32_t)base[PF_NODE * fstride + j];
    p.ks = base[PF_KS * fstride + j];
    return p;
}

__device__ __forceinline__ void store_entry(uint32_t *base, int64_t fstride, int64_t j, const Entry &p) {
    base[PF_X * fstride + j] = __float_as_uint(p.x);
    base[PF_Y * fstride + j] = __float_as_uint(p.y);
    base[PF_TX * fstride + j] = __float_as_uint(p.tx);
    base[PF_TY * fstride + j] = __float_as_uint(p.ty);
    base[PF_E * fstride + j] = p.e;
    base[PF_LO * fstride + j] = p.lo;
    base[PF_HI * fstride + j] = p.hi;
    base[PF_NODE * fstride + j] = (uint32_t)p.node;
    base[PF_KS * fstride + j] = p.ks;
}

// Per-shower state, one shower slot per lane 0..SLOTS-1 of a few registers.
struct Slots {
    int i;           // batch index of the shower, -1 when the slot is free
    uint32_t sid;    // global shower id
    uint32_t e0;     // fixed-point initial energy
    int live;        // particles of the shower in the pool
    int hits, nodes, passes, escaped, backward;
    uint32_t e_esc;  // escaped energy (fits: energies of a shower sum to e0)
    int hc, hf;      // the slot's hit-log chunk (-1: none) and its fill
    int hs_c, hs_f;  // where the shower's first hit record goes (shared
                     // showers: the reserved chunks' base and count)
    int sh;          // share record of a shared shower, -1 otherwise
};

__device__ __forceinline__ int slot_get(int v, int s) { return __builtin_amdgcn_readlane(v, s); }



// Calls f(s, m) once for every distinct slot s among the lanes of mask, with
// m the lanes of mask whose slot is s (mask is wave-uniform).
template <class F>
__device__ __forceinline__ void for_each_slot(uint64_t mask, int slot, F f) {
    while (mask) {
        const int l0 = __builtin_ctzll(mask);
        const int s0 = __builtin_amdgcn_readlane(slot, l0);
        const uint64_t m = mask & wave_ballot(slot == s0);
        f(s0, m);
        mask &= ~m;
    }
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ int wave_excl_scan(int v) {
    int incl = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int t = __shfl_up(incl, off, 64);
        if ((int)lane_id() >= off) incl += t;
    }
    return incl - v;
}

// parameters of subtree work items, kept in LDS (the scalar file is full)
enum { SL_EXPORT = 0, SL_PHASE, SL_ITEMS_IN, SL_ITEM_CAP, SL_SHARE_CAP, SL_MARGIN, SL_ITEMS, SL_SHARES = SL_ITEMS + 2,
       SUB_LDS_WORDS = 16 };
// LDS words of one wave: pool + the stop / split thresholds of every plane
// pool, then the thresholds c1, c2 (u64) of 64 planes, of 4 rings with
// regional parameters
// (then the energy tallies: cut and stop energy per slot and lane, and the
// slot masks of a step)
__host__ __device__ constexpr int lds_words(int pool_cap, bool rings = false) {
    return POOL_FIELDS * pool_cap + 2 * 2 * 64 * (rings ? 4 : 1) + SUB_LDS_WORDS + 2 * SLOTS * WAVE + 2 * SLOTS;
}

// Keeps a wave-uniform value in scalar registers but hides it from loop-
// invariant code motion, so that quantities derived from it are recomputed
// where they are used instead of being held (and spilled) through the loop.
__device__ __forceinline__ uint32_t opaque_u32(uint32_t v) {
    asm volatile("" : "+s"(v));
    return v;
}


// TREE: node records; KEYS: path ids with hit and node records; LIT: literal
// Algorithm 1 kinematics; REG: regional parameters (rings) (compile-time, so
// that no flag occupies a scalar register through the loop)
template <bool TREE, bool KEYS, int PC, bool LIT, bool REG, bool SUB>
__global__ void __launch_bounds__(WAVE) __attribute__((amdgpu_waves_per_eu(4))) supa_propagate(Params P) {
    extern __shared__ uint32_t lds[];
    const uint32_t lane = lane_id();
    const int64_t wave = blockIdx.x;
    const int N = P.n_planes;
    // the wave's start on the constant-rate clock (stored at once: nothing is
    // held through the loop); the first launch of a call only
    if (lane == 0 && COLD(wave_clk) && (!SUB || P.phase == 0))
        COLD(wave_clk)[2 * wave] = (unsigned long long)wall_clock64();
    // PC: pool entries in LDS, a power of two >= 2 * WAVE (compile-time, so
    // that the field offsets are instruction immediates)
    uint32_t *const pool = lds;            // [POOL_FIELDS][PC], entry j at slot j & (PC-1)
    // c1[ring * 64 + k] then c2 (one ring without regional parameters)
    uint64_t *const thr = (uint64_t *)(pool + POOL_FIELDS * PC);
    constexpr int TN = REG ? 4 * 64 : 64;
    for (int k = (int)lane; k < TN; k += WAVE) {
        const bool in = (k & 63) < N;
        thr[k] = in ? P.c1[k] : 0ull;
        thr[TN + k] = in ? P.c2[k] : 0ull;
    }
    // subtree parameters: export threshold (-1: none in this launch), launch
    // phase, items exported by the previous launch, capacities, buffers
    uint32_t *const sub_l = (uint32_t *)(thr + 2 * TN);
    if (SUB && lane == 0) {
        const int ph = P.phase;
        sub_l[SL_EXPORT] = (uint32_t)((ph < P.last_phase && P.export_top >= 0) ? P.export_top : -1);
        sub_l[SL_PHASE] = (uint32_t)ph;
        const unsigned long long got =
            ph > 0 ? __hip_atomic_load(&P.ctr[ctr_st_out(ph - 1)], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0ull;
        sub_l[SL_ITEMS_IN] = (uint32_t)min<unsigned long long>(got, (unsigned long long)P.item_cap);
        sub_l[SL_ITEM_CAP] = (uint32_t)P.item_cap;
        sub_l[SL_SHARE_CAP] = (uint32_t)P.share_cap;
        sub_l[SL_MARGIN] = __float_as_uint(P.share_margin);
        *(uint64_t *)(sub_l + SL_ITEMS) = (uint64_t)(uintptr_t)P.items;
        *(uint64_t *)(sub_l + SL_SHARES) = (uint64_t)(uintptr_t)P.shares;
    }
    // per-lane partial sums of the energy each slot's shower deposited by
    // cuts ([slot][lane]) and by stops (then [slot][lane]): every lane adds
    // to its own word (LDS atomics without conflicts), a shower's words are
    // summed once when it ends (its energies sum to e0 < 2^32)
    uint32_t *const esum = sub_l + SUB_LDS_WORDS;
    uint32_t *const smask = esum + 2 * SLOTS * WAVE;     // the four slot masks of a step
    for (int q = 0; q < 2 * SLOTS; ++q) esum[q * WAVE + lane] = 0u;
    __syncthreads();
    float rr1 = 0.f, rr2 = 0.f, rr3 = 0.f;        // squared ring radii
    if constexpr (REG) {
        const volatile __attribute__((address_space(1))) Cold *cp =
            (const volatile __attribute__((address_space(1))) Cold *)P.cold;
        const float a = cp->ring_r[0], b = cp->ring_r[1], c = cp->ring_r[2];
        rr1 = a * a;
        rr2 = b * b;
        rr3 = c * c;
    }

    const int64_t G = P.spill_cap;
    // Values the step reads but that are uniform, kept in vector registers:
    // the scalar file is full, and from a spilled scalar each use costs a
    // v_readlane on the step's path.
    uint32_t f_lo = P.f_lo, fw_lo = (uint32_t)P.f_w, fw_hi = (uint32_t)(P.f_w >> 32);
    uint32_t hl_lo = (uint32_t)(uintptr_t)P.hlog, hl_hi = (uint32_t)((uintptr_t)P.hlog >> 32);
    asm volatile("" : "+v"(f_lo), "+v"(fw_lo), "+v"(fw_hi), "+v"(hl_lo), "+v"(hl_hi));
    const uint64_t f_w = ((uint64_t)fw_hi << 32) | fw_lo;
    // (rebuilt as a global-memory pointer, so stores through it stay global)
    gu32 *const hlog = (gu32 *)(((uint64_t)hl_hi << 32) | hl_lo);
    uint32_t *const spill = P.spill + wave * POOL_FIELDS * G;
    constexpr bool keys = KEYS;
    const bool recs = (P.outputs & 3u) != 0;        // hit records (clouds or images)

    Slots S;
    S.i = -1;
    S.sid = S.e0 = 0u;
    S.live = S.hits = S.nodes = S.passes = S.escaped = S.backward = 0;
    S.e_esc = 0u;
    S.hc = S.hs_c = -1;
    S.hf = S.hs_f = 0;
    S.sh = -1;

    // pool: logical entries [bot, top); bot > 0 only after exports
    int top = 0, lo = 0, max_top = 0, bot = 0;
    bool exhausted = false, overflow = false;
    unsigned long long steps = 0;
    const float zf = P.z_first, dzp = P.dz;

    // open node-log chunk (-1: none yet, -2: log full) and its fill
    int nc = -1, nf = 0;
    // room for m more node records in the open chunk: closes it and claims
    // the next one when they do not fit; false once the log is full (the
    // batch is then rerun with a larger log)
    auto claim_nodes = [&](int m) -> bool {
        if (nc >= 0 && nf + m <= LOG_CHUNK) return true;
        if (nc == -2) return false;
        if (nc >= 0 && lane == 0) P.nfill[nc] = (uint32_t)nf;
        unsigned long long got = 0;
        if (lane == 0) got = atomicAdd(&P.ctr[CTR_NCHUNK], 1ull);
        const uint32_t g = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)got);
        if (g >= (uint32_t)P.n_chunks) {
            overflow = true;
            nc = -2;
            return false;
        }
        nc = (int)g;
        nf = 0;
        return true;
    };
    // a fresh hit-log chunk, or -1 once the log is full
    bool hlog_full = false;
    auto claim_hit_chunk = [&]() -> int {
        if (hlog_full) return -1;
        unsigned long long got = 0;
        if (lane == 0) got = atomicAdd(&P.ctr[CTR_HCHUNK], 1ull);
        const uint32_t g = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)got);
        if (g >= (uint32_t)P.h_chunks) {
            hlog_full = true;
            overflow = true;
            return -1;
        }
        return (int)g;
    };
    struct Hit {
        float x, y;
        uint32_t e, k, lo, hi;
    };
    auto write_hit = [&](int c, int pos, const Hit &h) {
        gu32 *chunk = hlog + (int64_t)c * HIT_CHUNK_WORDS;
        gu32 *rec = chunk + HIT_REC_WORDS * pos;
        rec[0] = __float_as_uint(h.x);
        rec[1] = __float_as_uint(h.y);
        rec[2] = h.e;
        ((gu8 *)(chunk + HIT_PLANE_OFF))[pos] = (uint8_t)h.k;
        if (keys) *(gu2 *)(chunk + HIT_KEY_OFF + HIT_KEY_WORDS * pos) = u32x2{h.lo, h.hi};
    };
    // appends the hit records of slot s0 to the slot's chain: lanes of m1
    // have hit h1, lanes of m2 hit h2 (a lane of both: h1 first)
    auto append_hits = [&](int s0, uint64_t m1, uint64_t m2, const Hit &h1, const Hit &h2) {
        int c = slot_get(S.hc, s0), f = slot_get(S.hf, s0);
        if (c < 0) return;
        const int cnt = (int)__popcll(m1) + (int)__popcll(m2);
        int c2 = -1;
        if (f + cnt > HIT_CHUNK) {
            c2 = claim_hit_chunk();
            if (c2 >= 0 && lane == 0) P.hnext[c] = (uint32_t)c2;
        }
        const bool in1 = (m1 >> lane) & 1ull, in2 = (m2 >> lane) & 1ull;
        const int p1 = f + (int)lanes_below(m1) + (int)lanes_below(m2);
        const int p2 = p1 + (in1 ? 1 : 0);
        if (in1) {
            const int cc = p1 < HIT_CHUNK ? c : c2;
            if (cc >= 0) write_hit(cc, p1 & (HIT_CHUNK - 1), h1);
        }
        if (in2) {
            const int cc = p2 < HIT_CHUNK ? c : c2;
            if (cc >= 0) write_hit(cc, p2 & (HIT_CHUNK - 1), h2);
        }
        if (f + cnt > HIT_CHUNK) {
            c = c2;
            f += cnt - HIT_CHUNK;
        } else {
            f += cnt;
        }
        if ((int)lane == s0) {
            S.hc = c;
            S.hf = f;
        }
    };

    // work comes in batches of SLOTS items; lane q < SLOTS prepares the
    // initial state of item base + q.  The next batch is claimed one batch
    // ahead, so its atomic has long returned when it is needed.
    unsigned long long next_base = 0;
    if (lane == 0) next_base = atomicAdd(&P.sub[SUB_WORK], (unsigned long long)SLOTS);
    int b_left = 0, b_at = 0;
    int w_i = 0, w_ok = 0, w_fwd = 0;
    uint32_t w_e = 0u;
    float w_x = 0.f, w_y = 0.f, w_tx = 0.f, w_ty = 0.f;

    // ---- pool access: logical entries [lo, top) are in LDS, [bot, lo)
    // spilled (with exports the spill area is a ring: G is a power of two)
    auto spill_at = [&](int j) -> int { return SUB ? (j & (G - 1)) : j; };
    auto pool_load = [&](int j) -> Entry {
        if (j >= lo) return load_entry(pool, PC, j & (PC - 1));
        if (j - bot < G) return load_entry(spill, (int64_t)opaque_u32((uint32_t)G), spill_at(j));
        overflow = true;          // was never stored: the batch is rerun
        return Entry{0.f, 0.f, 0.f, 0.f, 0u, 0u, 0u, 0, 0u};
    };
    auto pool_store = [&](int j, const Entry &p) {
        const int sl = j & (PC - 1);
        if (j - PC >= lo) {            // slot holds live entry j - PC: move it out
            const Entry old = load_entry(pool, PC, sl);
            if (j - PC - bot < G) store_entry(spill, (int64_t)opaque_u32((uint32_t)G), spill_at(j - PC), old);
            else overflow = true;
        }
        store_entry(pool, PC, sl, p);
    };
    // rewrites live entry j where it is (LDS or spill)
    auto pool_put = [&](int j, const Entry &p) {
        if (j >= lo) store_entry(pool, PC, j & (PC - 1), p);
        else if (j - bot < G) store_entry(spill, (int64_t)opaque_u32((uint32_t)G), spill_at(j), p);
        else overflow = true;
    };
    // share records and items (subtree work items)
    auto share_ptr = [&](int sh, int f) -> uint32_t * {
        uint32_t *base = (uint32_t *)(uintptr_t)(*(const uint64_t *)(sub_l + SL_SHARES));
        return base + (int64_t)sh * SHARE_WORDS + f;
    };
    auto share_load = [&](int sh, int f) -> uint32_t {
        return __hip_atomic_load(share_ptr(sh, f), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    };
    // Turns the shower of slot q into a shared one: a share record holding
    // its identity, where its hit run continues (the rest of the slot's
    // current chunk, then kc chunks reserved and linked now, enough for the
    // expected hits of its energy times the margin) and, with a tree, the
    // next node index (every other tally is added by each party at its end).
    // Returns the share, or -1 (no share or log room left: not exported).
    auto convert = [&](int q) -> int {
        unsigned long long g = 0;
        if (lane == 0) g = atomicAdd(&P.ctr[CTR_ST_SHARES], 1ull);
        const uint32_t sh = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)g);
        if (sh >= (uint32_t)__builtin_amdgcn_readfirstlane((int)sub_l[SL_SHARE_CAP])) return -1;
        const int hc = slot_get(S.hc, q), hf = slot_get(S.hf, q);
        const uint32_t e0q = (uint32_t)slot_get((int)S.e0, q);
        int base = 0, kc = 0;
        if (recs) {
            // a shower of E splits until its parts fall below the threshold:
            // about 2 E / threshold deposits
            const float margin = __uint_as_float(sub_l[SL_MARGIN]);
            const float want = P.t_cut > 0ull ? 2.0f * (float)e0q / (float)P.t_cut : 1048576.0f;
            kc = (int)fminf(4096.0f, ceilf(margin * (want + 256.0f) * (1.0f / HIT_CHUNK)) + 1.0f);
            kc = __builtin_amdgcn_readfirstlane(max(kc, 2));
            unsigned long long gb = 0;
            if (lane == 0) gb = atomicAdd(&P.ctr[CTR_HCHUNK], (unsigned long long)kc);
            base = __builtin_amdgcn_readfirstlane((int)(uint32_t)gb);
            if ((int64_t)(uint32_t)base + kc > (int64_t)P.h_chunks) {
                hlog_full = true;
                overflow = true;        // rerun with a larger log
                return -1;
            }
            for (int t = (int)lane; t < kc - 1; t += WAVE) P.hnext[base + t] = (uint32_t)(base + t + 1);
            if (lane == 0 && hc >= 0) P.hnext[hc] = (uint32_t)base;
        }
        const int hs_c = slot_get(S.hs_c, q), hs_f = slot_get(S.hs_f, q);
        const int64_t hs = hs_c < 0 ? -1 : (int64_t)hs_c * HIT_CHUNK + hs_f;
        const uint32_t f = lane;
        const uint32_t v = f == SH_I ? (uint32_t)slot_get(S.i, q) : f == SH_SID ? (uint32_t)slot_get((int)S.sid, q)
                         : f == SH_E0 ? e0q : f == SH_HS_LO ? (uint32_t)hs : f == SH_HS_HI ? (uint32_t)((uint64_t)hs >> 32)
                         : f == SH_CONV_C ? (uint32_t)hc : f == SH_CONV_F ? (uint32_t)hf
                         : f == SH_BASE ? (uint32_t)base : f == SH_KCAP ? (uint32_t)kc
                         : f == SH_NODES ? (TREE ? (uint32_t)slot_get(S.nodes, q) : 0u)
                         : f == SH_OUT ? 1u : 0u;
        if (f < (uint32_t)SH_FIELDS) *share_ptr((int)sh, (int)f) = v;
        __threadfence();
        if ((int)lane == q) {
            S.sh = (int)sh;
            S.hs_c = base;
            S.hs_f = kc;
        }
        return (int)sh;
    };

    for (;;) {
        if (SUB && top == bot) top = bot = lo = 0;
        // ---- refill: start showers while the pool is short of a full wave
        while (top - bot < WAVE && !exhausted) {
            const uint64_t free_slots = wave_ballot((int)lane < SLOTS && S.i < 0);
            if (!free_slots) break;
            const int s = __builtin_ctzll(free_slots);
            const int ph = SUB ? __builtin_amdgcn_readfirstlane((int)sub_l[SL_PHASE]) : 0;
            if (SUB && ph > 0) {
                // an item exported by the previous launch: pending particles
                // of one shared shower, taken into slot s as one more party
                unsigned long long got = 0;
                if (lane == 0) got = atomicAdd(&P.ctr[ctr_st_claim(ph)], 1ull);
                const uint32_t it = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)got);
                if (it >= (uint32_t)__builtin_amdgcn_readfirstlane((int)sub_l[SL_ITEMS_IN])) {
                    exhausted = true;
                    break;
                }
                const uint32_t *items = (const uint32_t *)(uintptr_t)(*(const uint64_t *)(sub_l + SL_ITEMS));
                const int64_t cap = (int64_t)__builtin_amdgcn_readfirstlane((int)sub_l[SL_ITEM_CAP]);
                const uint32_t *item = items + ((int64_t)((ph - 1) & 1) * cap + it) * ITEM_WORDS;
                const int cnt = min(WAVE, __builtin_amdgcn_readfirstlane((int)item[POOL_FIELDS * WAVE]));
                Entry e{0.f, 0.f, 0.f, 0.f, 0u, 0u, 0u, 0, 0u};
                if ((int)lane < cnt) e = load_entry(item, WAVE, lane);
                const int sh = __builtin_amdgcn_readfirstlane((int)(e.ks >> 8));
                const uint32_t fv = (int)lane < SH_NODES ? share_load(sh, (int)lane) : 0u;
                const int v_i = __builtin_amdgcn_readlane((int)fv, SH_I);
                const uint32_t v_sid = (uint32_t)__builtin_amdgcn_readlane((int)fv, SH_SID);
                const uint32_t v_e0 = (uint32_t)__builtin_amdgcn_readlane((int)fv, SH_E0);
                const int v_cc = __builtin_amdgcn_readlane((int)fv, SH_CONV_C);
                const int v_cf = __builtin_amdgcn_readlane((int)fv, SH_CONV_F);
                const int v_base = __builtin_amdgcn_readlane((int)fv, SH_BASE);
                const int v_kc = __builtin_amdgcn_readlane((int)fv, SH_KCAP);
                if ((int)lane == s) {
                    S.i = v_i;
                    S.sid = v_sid;
                    S.e0 = v_e0;
                    S.sh = sh;
                    S.hc = v_cc;
                    S.hf = v_cf;
                    S.hs_c = v_base;
                    S.hs_f = v_kc;
                    S.live = cnt;
                    S.hits = S.nodes = S.passes = S.escaped = S.backward = 0;
                    S.e_esc = 0u;
                }
                if ((int)lane < cnt) {
                    e.ks = (e.ks & 255u) | ((uint32_t)s << 8);
                    pool_store(top + (int)lane, e);
                }
                top += cnt;
                lo = max(lo, top - PC);
                max_top = max(max_top, top - bot);
                continue;
            }
            if (b_at == b_left) {
                const uint32_t base = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)next_base);
                if (base >= (uint32_t)P.n) {
                    exhausted = true;
                    break;
                }
                if (lane == 0) next_base = atomicAdd(&P.sub[SUB_WORK], (unsigned long long)SLOTS);
                b_left = min(SLOTS, P.n - (int)base);
                b_at = 0;
                if ((int)lane < b_left) {
                    // initial condition (section "Using SUPA": energy, angle, impact point)
                    const int item = (int)base + (int)lane;
                    const auto ord = COLD(order);
                    const int i = ord ? ord[item] : item;
                    const float sc = COLD(e0)[i] * P.e_scale;
                    const bool ok = sc >= 0.0f && sc < 4294967296.0f;
                    float sp, cp, sa, ca;
                    sincosf(COLD(polar)[i], &sp, &cp);
                    sincosf(COLD(azimuth)[i], &sa, &ca);
                    const float tpol = sp / cp;
                    const auto x0p = COLD(x0), y0p = COLD(y0);
                    w_i = i;
                    w_ok = ok ? 1 : 0;
                    w_e = ok ? (uint32_t)rintf(sc) : 0u;
                    // literal kinematics: lateral position only, no drift
                    w_fwd = (cp > 0.0f || LIT) ? 1 : 0;
                    w_tx = LIT ? 0.0f : tpol * ca;
                    w_ty = LIT ? 0.0f : tpol * sa;
                    w_x = x0p ? x0p[i] : 0.0f;
                    w_y = y0p ? y0p[i] : 0.0f;
                }
            }
            const int i = __builtin_amdgcn_readlane(w_i, b_at);
            const bool ok = __builtin_amdgcn_readlane(w_ok, b_at) != 0;
            const bool fwd0 = __builtin_amdgcn_readlane(w_fwd, b_at) != 0;
            const uint32_t e_first = (uint32_t)__builtin_amdgcn_readlane((int)w_e, b_at);
            const float x_first = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(w_x), b_at));
            const float y_first = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(w_y), b_at));
            const float tx0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(w_tx), b_at));
            const float ty0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(w_ty), b_at));
            ++b_at;
            if (!ok) {
                if (lane == 0) atomicOr(&P.ctr[CTR_FLAGS], (unsigned long long)FLAG_RANGE);
                if ((int)lane < 4) COLD(ledger)[4 * (int64_t)i + lane] = 0;
                if ((int)lane < 6) COLD(counts)[6 * (int64_t)i + lane] = 0;
                continue;
            }
            int hc0 = -1, hf0 = 0;
            if (recs) {
                // the shower's hits start at its slot's chain position
                hc0 = slot_get(S.hc, s);
                hf0 = slot_get(S.hf, s);
                if (hc0 < 0 || hf0 >= HIT_CHUNK) {
                    hc0 = claim_hit_chunk();
                    hf0 = 0;
                }
            }
            // the primary flies from z = 0 to the first plane (a particle
            // below threshold deposits on arrival)
            const float x1 = fmaf(zf, tx0, x_first), y1 = fmaf(zf, ty0, y_first);
            const bool cut0 = fwd0 && (uint64_t)e_first < P.t_cut;
            if ((int)lane == s) {
                S.hc = S.hs_c = hc0;
                S.hf = S.hs_f = hf0;
                S.i = i;
                S.sid = P.sid_base + (uint32_t)i;
                S.e0 = e_first;
                S.live = (fwd0 && !cut0) ? 1 : 0;
                S.hits = 0;
                S.nodes = 1;
                S.passes = 0;
                S.escaped = fwd0 ? 0 : 1;
                S.backward = fwd0 ? 0 : 1;
                S.e_esc = fwd0 ? 0u : e_first;
            }
            if (cut0) {
                const Hit h{x1, y1, e_first, 0u, 1u, 0u};
                if (recs) append_hits(s, 1ull, 0ull, h, h);
                if ((int)lane == s) S.hits = 1;
                if (lane == 0) atomicAdd(&esum[s * WAVE], e_first);
            } else if (fwd0) {
                if (lane == 0) {
                    const Entry p0{x1, y1, tx0, ty0, e_first, 1u, 0u, 0, (uint32_t)s << 8};
                    pool_store(top, p0);
                }
                ++top;
                lo = max(lo, top - PC);
            }
            if (TREE && claim_nodes(1)) {
                if (lane == 0) {
                    uint32_t *r = P.nlog + (int64_t)nc * (NL_FIELDS * LOG_CHUNK) + nf;
                    r[NL_I * LOG_CHUNK] = (uint32_t)i;
                    r[NL_IDX * LOG_CHUNK] = 0u;
                    r[NL_PARENT * LOG_CHUNK] = (uint32_t)-1;
                    r[NL_GK * LOG_CHUNK] = GK_PRIMARY;
                    r[NL_X * LOG_CHUNK] = __float_as_uint(x_first);
                    r[NL_Y * LOG_CHUNK] = __float_as_uint(y_first);
                    r[NL_E * LOG_CHUNK] = e_first;
                    r[NL_E2 * LOG_CHUNK] = 0u;
                    if (keys) {
                        r[NL_LO * LOG_CHUNK] = 1u;
                        r[NL_HI * LOG_CHUNK] = 0u;
                    }
                }
                nf += 1;
            }
        }
        const uint64_t active = wave_ballot((int)lane < SLOTS && S.i >= 0);
        if (!active) break;

        if (top > bot) {
            // ---- one step of Algorithm 1 for up to 64 particles, each at its
            // own plane k: draw, three-way choice, split; what goes on flies
            // to plane k+1 at once, and deposits there if below threshold
            const int nb = min(WAVE, top - bot);
            const bool valid = (int)lane < nb;
            const int j = top - 1 - (int)lane;
            if (top - nb < lo) __threadfence_block();    // spilled entries: see other lanes' stores
            // lanes past the pending particles load the top entry again: every
            // use of p below is masked by this step's flags, so its values
            // need no clearing first
            const Entry p = pool_load(valid ? j : top - 1);
            top -= nb;
            lo = min(lo, top);
            const int k = (int)(p.ks & 255u), slot = (int)(p.ks >> 8);
            // the lanes of each shower slot; `mine`: this lane's slot, `own`:
            // in lanes 0..SLOTS-1, the lanes of slot `lane` (whose state the
            // lane holds).  Named registers: a run-time-indexed array would
            // go to scratch memory.  Taken before the draw, so that lane 0's
            // write below is a branch around which hardly any lane mask is
            // live (masks live across a divergent branch are copied through
            // vector registers, two instructions each)
            const uint64_t sm0 = wave_ballot(valid && slot == 0), sm1 = wave_ballot(valid && slot == 1);
            const uint64_t sm2 = wave_ballot(valid && slot == 2), sm3 = wave_ballot(valid && slot == 3);
            // own and mine: the scalar masks through LDS (lane 0 writes all
            // four; lane q < SLOTS reads mask q, every lane the mask of its
            // particle's slot), with no selection per lane
            if (lane == 0) {
                *(uint4 *)(smask) = make_uint4((uint32_t)sm0, (uint32_t)(sm0 >> 32), (uint32_t)sm1, (uint32_t)(sm1 >> 32));
                *(uint4 *)(smask + 4) = make_uint4((uint32_t)sm2, (uint32_t)(sm2 >> 32), (uint32_t)sm3, (uint32_t)(sm3 >> 32));
            }
            const uint2 ow = *(const uint2 *)(smask + 2 * (lane & (SLOTS - 1)));
            const uint64_t own = (int)lane < SLOTS ? (((uint64_t)ow.y << 32) | ow.x) : 0ull;
            const uint2 mn = *(const uint2 *)(smask + 2 * (slot & (SLOTS - 1)));
            const uint64_t mine = ((uint64_t)mn.y << 32) | mn.x;
            const uint32_t sid = (uint32_t)__shfl((int)S.sid, slot, WAVE);
            const uint4 w = philox4x32_10((uint32_t)k, sid, p.lo, p.hi, opaque_u32(P.seed_lo),
                                          opaque_u32(P.seed_hi));
            int ring = 0;
            if constexpr (REG) {
                // ring from the position at arrival: r^2 against the squared radii
                const float r2 = fmaf(p.x, p.x, p.y * p.y);
                ring = (r2 >= rr1 ? 1 : 0) + (r2 >= rr2 ? 1 : 0) + (r2 >= rr3 ? 1 : 0);
            }
            const uint64_t c1 = thr[ring * 64 + k], c2 = thr[TN + ring * 64 + k];
            const bool is_stop = valid && (uint64_t)w.x < c1;
            const bool is_split = valid && !is_stop && (uint64_t)w.x < c2;
            const bool is_pass = valid && !is_stop && !is_split;
            const bool last = (k == N - 1);
            const uint64_t path = ((uint64_t)p.hi << 32) | p.lo;

            Daughters D;
            D.fwd_a = D.fwd_b = false;
            D.ea = D.eb = 0;
            D.txa = D.tya = D.txb = D.tyb = 0.f;
            if (is_split) D = split_particle<LIT>(P, p.tx, p.ty, p.e, w, f_lo, f_w);
            // outgoing particles: a = first daughter or the passer, b = second daughter
            const bool has_a = is_split || is_pass, has_b = is_split;
            const uint32_t ea = is_split ? D.ea : p.e, eb = D.eb;
            const float txa = is_split ? D.txa : p.tx, tya = is_split ? D.tya : p.ty;
            const bool fwd_a = is_split ? D.fwd_a : true, fwd_b = D.fwd_b;
            const bool go_a = has_a && !last && fwd_a, go_b = has_b && !last && fwd_b;
            // flight to plane k+1
            const float xa = fmaf(dzp, txa, p.x), ya = fmaf(dzp, tya, p.y);
            const float xb = fmaf(dzp, D.txb, p.x), yb = fmaf(dzp, D.tyb, p.y);
            const bool cut_a = go_a && (uint64_t)ea < P.t_cut, cut_b = go_b && (uint64_t)eb < P.t_cut;
            const bool push_a = go_a && !cut_a, push_b = go_b && !cut_b;
            // leaking out: after the last plane, or turned away from +z
            int esc_n = 0, back_n = 0;
            uint32_t esc_e = 0u;
            if (last) {
                if (has_a) { esc_n += 1; esc_e += ea; }
                if (has_b) { esc_n += 1; esc_e += eb; }
            } else {
                if (has_a && !fwd_a) { esc_n += 1; back_n += 1; esc_e += ea; }
                if (has_b && !fwd_b) { esc_n += 1; back_n += 1; esc_e += eb; }
            }
            // deposits: a stop at plane k, daughters below threshold at k+1
            const bool hit1 = is_stop || cut_a, hit2 = cut_b;
            const uint64_t pa = path << 1;
            atomicAdd(&esum[slot * WAVE + (int)lane], (cut_a ? ea : 0u) + (cut_b ? eb : 0u));
            if (wave_ballot(is_stop)) atomicAdd(&esum[(SLOTS + slot) * WAVE + (int)lane], is_stop ? p.e : 0u);

            const uint64_t mh1 = wave_ballot(hit1), mh2 = wave_ballot(hit2);
            const uint64_t mpa = wave_ballot(push_a), mpb = wave_ballot(push_b);
            const uint64_t msplit = wave_ballot(is_split), mpass = wave_ballot(is_pass);
            const uint64_t mesc = wave_ballot(esc_n > 0);
            // node index of daughter a: the slot's node count + 2 per split
            // below (a shared shower's next indices come from its share)
            if (SUB && TREE && msplit) {
                const bool shs = (int)lane < SLOTS && S.sh >= 0;
                if (wave_ballot(shs)) {
                    const int ns = (int)__popcll(msplit & own);
                    if (shs && ns > 0) S.nodes = (int)atomicAdd(share_ptr(S.sh, SH_NODES), (uint32_t)(2 * ns));
                }
            }
            const int node_a = __shfl(S.nodes, slot, WAVE) + 2 * (int)lanes_below(msplit & mine);
            if (recs && (mh1 | mh2)) {
                // hit records of every slot at once: the slot's chain position
                // + this lane's rank among the slot's records of the step
                const int c = __shfl(S.hc, slot, WAVE), f = __shfl(S.hf, slot, WAVE);
                const int cnt_own = (int)__popcll(mh1 & own) + (int)__popcll(mh2 & own);
                const bool over_own = S.hc >= 0 && (!SUB || S.sh < 0) && S.hf + cnt_own > HIT_CHUNK;
                // a slot whose chunk fills up links a fresh one (rare)
                int c2_own = -1;
                for (uint64_t mo = wave_ballot(over_own); mo; mo &= mo - 1) {
                    const int q = __builtin_ctzll(mo);
                    const int c2 = claim_hit_chunk();
                    const int hc_q = slot_get(S.hc, q);
                    if (c2 >= 0 && lane == 0) P.hnext[hc_q] = (uint32_t)c2;
                    if ((int)lane == q) c2_own = c2;
                }
                const int c2 = __shfl(c2_own, slot, WAVE);
                const int r1 = (int)lanes_below(mh1 & mine) + (int)lanes_below(mh2 & mine);
                const int p1 = f + r1;
                const int p2 = p1 + (hit1 ? 1 : 0);
                int cc1 = p1 < HIT_CHUNK ? c : c2, o1 = p1 & (HIT_CHUNK - 1);
                int cc2 = p2 < HIT_CHUNK ? c : c2, o2 = p2 & (HIT_CHUNK - 1);
                if (SUB) {
                    // shared showers: positions in the shower's run from its
                    // fill counter, past the conversion point (c, f), then
                    // through the reserved chunks
                    const bool shs = (int)lane < SLOTS && S.sh >= 0;
                    if (wave_ballot(shs)) {
                        int fb = 0;
                        if (shs && cnt_own > 0) fb = (int)atomicAdd(share_ptr(S.sh, SH_FILL), (uint32_t)cnt_own);
                        const int fbs = __shfl(fb, slot, WAVE);
                        const bool mysh = __shfl(S.sh, slot, WAVE) >= 0;
                        const int kb = __shfl(S.hs_c, slot, WAVE), kn = __shfl(S.hs_f, slot, WAVE);
                        if (mysh) {
                            const int room = c >= 0 ? HIT_CHUNK - f : 0;
                            auto place = [&](int q, int &cc, int &o) {
                                if (q < room) {
                                    cc = c;
                                    o = f + q;
                                } else {
                                    const int t = q - room;
                                    cc = (t >> HIT_CHUNK_LOG2) < kn ? kb + (t >> HIT_CHUNK_LOG2) : -1;
                                    o = t & (HIT_CHUNK - 1);
                                }
                            };
                            place(fbs + r1, cc1, o1);
                            place(fbs + r1 + (hit1 ? 1 : 0), cc2, o2);
                            if ((hit1 && cc1 < 0) || (hit2 && cc2 < 0))
                                atomicOr(&P.ctr[CTR_FLAGS], (unsigned long long)FLAG_SHARE);
                        }
                    }
                }
                if (hit1) {
                    const Hit h1 = is_stop ? Hit{p.x, p.y, p.e, (uint32_t)k, p.lo, p.hi}
                                           : Hit{xa, ya, ea, (uint32_t)k + 1u, (uint32_t)pa, (uint32_t)(pa >> 32)};
                    if (cc1 >= 0) write_hit(cc1, o1, h1);
                }
                if (hit2) {
                    const Hit h2{xb, yb, eb, (uint32_t)k + 1u, (uint32_t)pa | 1u, (uint32_t)(pa >> 32)};
                    if (cc2 >= 0) write_hit(cc2, o2, h2);
                }
                if ((int)lane < SLOTS && S.hc >= 0 && (!SUB || S.sh < 0)) {
                    if (over_own) {
                        S.hc = c2_own;
                        S.hf += cnt_own - HIT_CHUNK;
                    } else {
                        S.hf += cnt_own;
                    }
                }
            }
            // per-shower counts of slot `lane` (lanes 0..SLOTS-1)
            if ((int)lane < SLOTS) {
                S.hits += (int)__popcll(mh1 & own) + (int)__popcll(mh2 & own);
                S.live += (int)__popcll(mpa & own) + (int)__popcll(mpb & own) - (int)__popcll(own);
                if (mpass) S.passes += (int)__popcll(mpass & own);
                S.nodes += 2 * (int)__popcll(msplit & own);
            }
            // leaks (after the last plane or backward): rare, per slot
            if (mesc) {
                for_each_slot(mesc, slot, [&](int s0, uint64_t m) {
                    const bool in = (m >> lane) & 1ull;
                    const int sn = wave_sum_i32(in ? esc_n : 0);
                    const int sb = wave_sum_i32(in ? back_n : 0);
                    const uint32_t se = wave_sum_u32(in ? esc_e : 0u);
                    if ((int)lane == s0) {
                        S.escaped += sn;
                        S.backward += sb;
                        S.e_esc += se;
                    }
                });
            }
            if (TREE && msplit) {
                // one record per split: both daughters; the step's records
                // grouped by slot, so that consecutive records are
                // consecutive nodes of one shower (the scatter then writes
                // runs instead of single nodes)
                const int m = (int)__popcll(msplit);
                const int ish = __shfl(S.i, slot, WAVE);
                if (claim_nodes(m)) {
                    if (is_split) {
                        const int n0 = (int)__popcll(msplit & sm0), n1 = (int)__popcll(msplit & sm1);
                        const int n2 = (int)__popcll(msplit & sm2);
                        const int below = slot == 0 ? 0 : slot == 1 ? n0 : slot == 2 ? n0 + n1 : n0 + n1 + n2;
                        uint32_t *r = P.nlog + (int64_t)nc * (NL_FIELDS * LOG_CHUNK) + nf + below +
                                      (int)lanes_below(msplit & mine);
                        r[NL_I * LOG_CHUNK] = (uint32_t)ish;
                        r[NL_IDX * LOG_CHUNK] = (uint32_t)node_a;
                        r[NL_PARENT * LOG_CHUNK] = (uint32_t)p.node;
                        r[NL_GK * LOG_CHUNK] = (uint32_t)(64 - __clzll(path)) | ((uint32_t)k << 8);
                        r[NL_X * LOG_CHUNK] = __float_as_uint(p.x);
                        r[NL_Y * LOG_CHUNK] = __float_as_uint(p.y);
                        r[NL_E * LOG_CHUNK] = D.ea;
                        r[NL_E2 * LOG_CHUNK] = D.eb;
                        if (keys) {
                            r[NL_LO * LOG_CHUNK] = (uint32_t)pa;
                            r[NL_HI * LOG_CHUNK] = (uint32_t)(pa >> 32);
                        }
                    }
                    nf += m;
                }
            }
            // survivors go back on the pool, bound for plane k+1
            const int pos = top + (int)lanes_below(mpa) + (int)lanes_below(mpb);
            const uint32_t ks1 = (uint32_t)(k + 1) | ((uint32_t)slot << 8);
            // (with literal kinematics the displacement was the flight: no slope is kept)
            const float sxa = LIT ? 0.0f : txa, sya = LIT ? 0.0f : tya;
            const float sxb = LIT ? 0.0f : D.txb, syb = LIT ? 0.0f : D.tyb;
            if (push_a) {
                const Entry q = is_split ? Entry{xa, ya, sxa, sya, ea, (uint32_t)pa, (uint32_t)(pa >> 32),
                                                 node_a, ks1}
                                         : Entry{xa, ya, sxa, sya, ea, p.lo, p.hi, p.node, ks1};
                pool_store(pos, q);
            }
            if (push_b) {
                const Entry q{xb, yb, sxb, syb, eb, (uint32_t)pa | 1u, (uint32_t)(pa >> 32),
                              node_a + 1, ks1};
                pool_store(pos + (push_a ? 1 : 0), q);
            }
            top += (int)__popcll(mpa) + (int)__popcll(mpb);
            lo = max(lo, top - PC);
            max_top = max(max_top, top - bot);
            if (SUB) {
                // ---- export: once the wave has no new work to take and its
                // pool holds export_top + WAVE entries, the oldest WAVE are
                // looked at, and those of the shower with most of them (at
                // least ITEM_MIN) leave as an item that the next launch
                // finishes; the others move up against the new bottom of the
                // pool.  (While showers remain to be started, every wave is
                // busy and an export would only add shared-shower traffic;
                // the wave's claim of its next showers is already back.)
                const int et = __builtin_amdgcn_readfirstlane((int)sub_l[SL_EXPORT]);
                const bool no_new = __builtin_amdgcn_readfirstlane((int)sub_l[SL_PHASE]) > 0 ||
                                    (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)next_base) >= (uint32_t)P.n;
                if (no_new && et >= 0 && top - bot >= et + WAVE) {
                    if (bot < lo) __threadfence_block();
                    const Entry e = pool_load(bot + (int)lane);
                    const int es = (int)(e.ks >> 8);
                    const uint64_t b0 = wave_ballot(es == 0), b1 = wave_ballot(es == 1);
                    const uint64_t b2 = wave_ballot(es == 2), b3 = wave_ballot(es == 3);
                    int q = 0;
                    uint64_t m = b0;
                    if (__popcll(b1) > __popcll(m)) { q = 1; m = b1; }
                    if (__popcll(b2) > __popcll(m)) { q = 2; m = b2; }
                    if (__popcll(b3) > __popcll(m)) { q = 3; m = b3; }
                    const int cnt = (int)__popcll(m);
                    int sh = cnt >= ITEM_MIN ? slot_get(S.sh, q) : -1;
                    if (cnt >= ITEM_MIN && sh < 0) sh = convert(q);
                    if (sh >= 0) {
                        const int ph = __builtin_amdgcn_readfirstlane((int)sub_l[SL_PHASE]);
                        unsigned long long got = 0;
                        if (lane == 0) got = atomicAdd(&P.ctr[ctr_st_out(ph)], 1ull);
                        const uint32_t it = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)got);
                        const int64_t cap = (int64_t)__builtin_amdgcn_readfirstlane((int)sub_l[SL_ITEM_CAP]);
                        if ((int64_t)it < cap) {
                            if (lane == 0) atomicAdd(share_ptr(sh, SH_OUT), 1u);
                            uint32_t *items = (uint32_t *)(uintptr_t)(*(const uint64_t *)(sub_l + SL_ITEMS));
                            uint32_t *item = items + ((int64_t)(ph & 1) * cap + it) * ITEM_WORDS;
                            const bool out_e = (m >> lane) & 1ull;
                            if (out_e) {
                                Entry x = e;
                                x.ks = (e.ks & 255u) | ((uint32_t)sh << 8);
                                store_entry(item, WAVE, (int64_t)lanes_below(m), x);
                            } else {
                                pool_put(bot + cnt + (int)lanes_below(~m), e);
                            }
                            if (lane == 0) item[POOL_FIELDS * WAVE] = (uint32_t)cnt;
                            bot += cnt;
                            lo = max(lo, bot);
                            if ((int)lane == q) S.live -= cnt;
                        }
                    }
                }
            }
        } else if (wave_ballot((int)lane < SLOTS && S.i >= 0 && S.live > 0)) {
            // nothing pending although a shower still counts live particles:
            // its accounting is inconsistent; report it and close it
            if (lane == 0) atomicOr(&P.ctr[CTR_FLAGS], (unsigned long long)FLAG_INTERNAL);
            if ((int)lane < SLOTS) S.live = 0;
        }

        // ---- showers whose last particle is done: ledger, counts and where
        // its hit records start (only stores)
        uint64_t done = wave_ballot((int)lane < SLOTS && S.i >= 0 && S.live <= 0);
        while (done) {
            const int s = __builtin_ctzll(done);
            done &= done - 1;
            const int i = slot_get(S.i, s);
            const int nh = slot_get(S.hits, s);
            const int nn = slot_get(S.nodes, s);
            const int npass = slot_get(S.passes, s);
            const int nesc = slot_get(S.escaped, s);
            const int nback = slot_get(S.backward, s);
            const uint32_t eesc = (uint32_t)slot_get((int)S.e_esc, s);
            const uint32_t e_first = (uint32_t)slot_get((int)S.e0, s);
            const int nsplit = (nn - 1) / 2;
            const uint32_t e_cut = wave_sum_u32(esum[s * WAVE + lane]);
            const uint32_t e_stop = wave_sum_u32(esum[(SLOTS + s) * WAVE + lane]);
            esum[s * WAVE + lane] = 0u;
            esum[(SLOTS + s) * WAVE + lane] = 0u;
            if (SUB && slot_get(S.sh, s) >= 0) {
                // one party of a shared shower is done: its tallies go to the
                // share; the last party writes the shower's results
                const int shs = slot_get(S.sh, s);
                uint32_t last_party = 0;
                if (lane == 0) {
                    atomicAdd(share_ptr(shs, SH_HITS), (uint32_t)nh);
                    if (!TREE) atomicAdd(share_ptr(shs, SH_NODES), (uint32_t)nn);
                    atomicAdd(share_ptr(shs, SH_PASSES), (uint32_t)npass);
                    atomicAdd(share_ptr(shs, SH_ESC), (uint32_t)nesc);
                    atomicAdd(share_ptr(shs, SH_BACK), (uint32_t)nback);
                    atomicAdd(share_ptr(shs, SH_EESC), eesc);
                    atomicAdd(share_ptr(shs, SH_ECUT), e_cut);
                    atomicAdd(share_ptr(shs, SH_ESTOP), e_stop);
                    __threadfence();
                    last_party = atomicSub(share_ptr(shs, SH_OUT), 1u) == 1u ? 1u : 0u;
                }
                if (__builtin_amdgcn_readfirstlane((int)last_party)) {
                    __threadfence();
                    const uint32_t v = (int)lane < SH_FIELDS ? share_load(shs, (int)lane) : 0u;
                    const int fi = __builtin_amdgcn_readlane((int)v, SH_I);
                    const int fnn = __builtin_amdgcn_readlane((int)v, SH_NODES);
                    const int fnh = __builtin_amdgcn_readlane((int)v, SH_HITS);
                    const int fpass = __builtin_amdgcn_readlane((int)v, SH_PASSES);
                    const int fesc = __builtin_amdgcn_readlane((int)v, SH_ESC);
                    const int fback = __builtin_amdgcn_readlane((int)v, SH_BACK);
                    const uint32_t fe0 = (uint32_t)__builtin_amdgcn_readlane((int)v, SH_E0);
                    const uint32_t fstop = (uint32_t)__builtin_amdgcn_readlane((int)v, SH_ESTOP);
                    const uint32_t fcut = (uint32_t)__builtin_amdgcn_readlane((int)v, SH_ECUT);
                    const uint32_t fesce = (uint32_t)__builtin_amdgcn_readlane((int)v, SH_EESC);
                    const uint32_t hs_lo = (uint32_t)__builtin_amdgcn_readlane((int)v, SH_HS_LO);
                    const uint32_t hs_hi = (uint32_t)__builtin_amdgcn_readlane((int)v, SH_HS_HI);
                    const int fsplit = (fnn - 1) / 2;
                    if (recs && lane == 0) COLD(hstart)[fi] = (int64_t)(((uint64_t)hs_hi << 32) | hs_lo);
                    steps += (unsigned long long)(fnh + fsplit + fpass);
                    if ((int)lane < 4) {
                        const uint32_t w = lane == 0 ? fe0 : lane == 1 ? fstop : lane == 2 ? fcut : fesce;
                        COLD(ledger)[4 * (int64_t)fi + lane] = w;
                    }
                    if ((int)lane < 6) {
                        const int w = lane == 0 ? fnn : lane == 1 ? fnh : lane == 2 ? fnh + fsplit + fpass
                                    : lane == 3 ? fsplit : lane == 4 ? fesc : fback;
                        COLD(counts)[6 * (int64_t)fi + lane] = w;
                    }
                }
                // the slot's next shower starts a fresh chunk: this one's
                // chunk belongs to the shared run
                if ((int)lane == s) {
                    S.i = -1;
                    S.sh = -1;
                    S.hc = -1;
                    S.hf = 0;
                }
                continue;
            }
            if (recs && lane == 0) {
                const int hs_c = slot_get(S.hs_c, s), hs_f = slot_get(S.hs_f, s);
                COLD(hstart)[i] = hs_c < 0 ? -1 : (int64_t)hs_c * HIT_CHUNK + hs_f;
            }
            steps += (unsigned long long)(nh + nsplit + npass);
            if ((int)lane < 4) {
                const uint32_t v = lane == 0 ? e_first : lane == 1 ? e_stop : lane == 2 ? e_cut : eesc;
                COLD(ledger)[4 * (int64_t)i + lane] = v;
            }
            if ((int)lane < 6) {
                const int v = lane == 0 ? nn : lane == 1 ? nh : lane == 2 ? nh + nsplit + npass
                            : lane == 3 ? nsplit : lane == 4 ? nesc : nback;
                COLD(counts)[6 * (int64_t)i + lane] = v;
            }
            if ((int)lane == s) S.i = -1;
        }
    }
    // close the open node-log chunk
    if (lane == 0) {
        if (TREE && nc >= 0) P.nfill[nc] = (uint32_t)nf;
        atomicAdd(&P.ctr[CTR_STEPS], steps);
        atomicMax(&P.ctr[CTR_NEED_F], (unsigned long long)max_top);
    }
    if (wave_ballot(overflow) && lane == 0) atomicOr(&P.ctr[CTR_FLAGS], (unsigned long long)FLAG_OVERFLOW);
    if (lane == 0 && COLD(wave_clk) && (!SUB || P.phase == 0))
        COLD(wave_clk)[2 * wave + 1] = (unsigned long long)wall_clock64();
}

__global__ void supa_zero_counters(unsigned long long *ctr) {
    if (threadIdx.x < CTR_WORDS) ctr[threadIdx.x] = 0ull;
}

// the node-log chunks claimed so far, noted for a sub-batch
__global__ void supa_note_chunks(const unsigned long long *ctr, unsigned long long *sub) {
    if (threadIdx.x == 0) sub[SUB_NCHUNK_END] = ctr[CTR_NCHUNK];
}

__global__ void supa_philox_kernel(const uint32_t *ctr, int64_t n, uint32_t k0, uint32_t k1,
                                   uint32_t *out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const uint4 w = philox4x32_10(ctr[4 * t], ctr[4 * t + 1], ctr[4 * t + 2], ctr[4 * t + 3], k0, k1);
    out[4 * t] = w.x;
    out[4 * t + 1] = w.y;
    out[4 * t + 2] = w.z;
    out[4 * t + 3] = w.w;
}

__global__ void supa_azimuth_kernel(const uint32_t *w, int64_t n, float *s, float *c) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    azimuth_sincos(w[t], &s[t], &c[t]);
}

// ---------------------------------------------------------------------------
// host-side launchers (called by the C ABI in supa_api.hip)
// ---------------------------------------------------------------------------
hipError_t launch_zero_counters(unsigned long long *ctr, hipStream_t s) {
    static_assert(CTR_WORDS <= 128, "one workgroup clears the counters");
    hipLaunchKernelGGL(supa_zero_counters, dim3(1), dim3(128), 0, s, ctr);
    return hipGetLastError();
}

hipError_t launch_note_chunks(const unsigned long long *ctr, unsigned long long *sub, hipStream_t s) {
    hipLaunchKernelGGL(supa_note_chunks, dim3(1), dim3(64), 0, s, ctr, sub);
    return hipGetLastError();
}

size_t propagate_lds_bytes(int pool_cap, bool rings) {
    return (size_t)lds_words(pool_cap, rings) * 4;
}

template <bool TREE, bool KEYS, bool LIT, bool REG, bool SUB>
static hipError_t launch_pc(const Params &P, int blocks, size_t lds, hipStream_t s) {
    switch (P.pool_cap) {
    case 128: hipLaunchKernelGGL((supa_propagate<TREE, KEYS, 128, LIT, REG, SUB>), dim3(blocks), dim3(WAVE), lds, s, P); break;
    case 256: hipLaunchKernelGGL((supa_propagate<TREE, KEYS, 256, LIT, REG, SUB>), dim3(blocks), dim3(WAVE), lds, s, P); break;
    case 512: hipLaunchKernelGGL((supa_propagate<TREE, KEYS, 512, LIT, REG, SUB>), dim3(blocks), dim3(WAVE), lds, s, P); break;
    case 1024: hipLaunchKernelGGL((supa_propagate<TREE, KEYS, 1024, LIT, REG, SUB>), dim3(blocks), dim3(WAVE), lds, s, P); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <bool LIT, bool REG, bool SUB>
static hipError_t launch_kin(const Params &P, int blocks, size_t lds, hipStream_t s) {
    const bool tree = (P.outputs & 4u) != 0;
    if (tree)
        return P.keys ? launch_pc<true, true, LIT, REG, SUB>(P, blocks, lds, s)
                      : launch_pc<true, false, LIT, REG, SUB>(P, blocks, lds, s);
    return P.keys ? launch_pc<false, true, LIT, REG, SUB>(P, blocks, lds, s)
                  : launch_pc<false, false, LIT, REG, SUB>(P, blocks, lds, s);
}

// Subtree work items (P.last_phase > 0) exist for the plain kinematics only.
hipError_t launch_propagate(const Params &P, bool literal, bool rings, int blocks, hipStream_t s) {
    const size_t lds = propagate_lds_bytes(P.pool_cap, rings);
    if (P.last_phase > 0) {
        if (literal || rings) return hipErrorInvalidValue;
        return launch_kin<false, false, true>(P, blocks, lds, s);
    }
    if (rings) return literal ? launch_kin<true, true, false>(P, blocks, lds, s) : launch_kin<false, true, false>(P, blocks, lds, s);
    return literal ? launch_kin<true, false, false>(P, blocks, lds, s) : launch_kin<false, false, false>(P, blocks, lds, s);
}

hipError_t launch_azimuth(const uint32_t *w, int64_t n, float *sn, float *cs, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int threads = 256;
    const int64_t blocks = (n + threads - 1) / threads;
    hipLaunchKernelGGL(supa_azimuth_kernel, dim3((unsigned)blocks), dim3(threads), 0, s, w, n, sn, cs);
    return hipGetLastError();
}

hipError_t launch_philox(const uint32_t *ctr, int64_t n, uint32_t k0, uint32_t k1, uint32_t *out,
                         hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int threads = 256;
    const int64_t blocks = (n + threads - 1) / threads;
    hipLaunchKernelGGL(supa_philox_kernel, dim3((unsigned)blocks), dim3(threads), 0, s, ctr, n, k0,
                       k1, out);
    return hipGetLastError();
}

}  // namespace supa
