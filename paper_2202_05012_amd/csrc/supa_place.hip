// supa_place.hip -- hit clouds and per-layer images from the hit log.
//
// One 512-thread workgroup takes one shower at a time and walks the chain of
// log chunks that holds its hit records (the propagation kernel wrote them
// there in the order it produced them):
//   hit clouds  count the records per plane (LDS), turn the counts into plane
//               starts within the shower's segment, planes taken in order of
//               (layer, plane), and put every record at segment start + the
//               next free place of its plane, so the segment is grouped by
//               layer and, within a layer, by plane (order within a plane is
//               free; with a non-decreasing layer map this is plane order);
//               a segment of up to PL_WIN hits is sorted in LDS first and
//               leaves with contiguous stores;
//   images      (paper, appendix "Downsampling": a region of interest per
//               layer, a grid of cells, and per cell the summed energy of the
//               points in it) an LDS slab holding whole layers, or a band of
//               rows of one large layer, is cleared, the integer energies of
//               its hits are added with LDS atomics (integer sums: order-free
//               and exact) and the slab is streamed out as float once, so
//               every image byte is written exactly once.
// Up to PL_WIN records per shower stay in registers between these passes;
// larger showers are read again per pass.
#include <algorithm>

#include "supa_device.hpp"

namespace supa {

constexpr int PL_THREADS = 512;
constexpr int PL_UNROLL = 4;
constexpr int PL_WIN = PL_THREADS * PL_UNROLL;      // records per window (two chunks)
constexpr int PL_SLAB_WORDS = 16384;                // image slab: 64 KB of LDS per workgroup
constexpr int PL_STAGE_WORDS = 4 * PL_WIN;          // hit staging: 32 KB (hit clouds only)
constexpr int PL_MAX_SLABS = 1024;                  // slabs per image bucketed in LDS counts
constexpr int PL_BUCKET_MIN_SLABS = 9;              // fewer slabs: bin the cached hits per slab
constexpr int PL_CLIST = 512;                       // chunk ids of a shower's chain listed in LDS
// Hits per plane are counted into PL_COPIES histograms, thread t adding to
// copy t mod PL_COPIES, and summed afterwards: a wave's count instruction
// then has at most four lanes on one LDS word (one histogram had up to 64
// lanes of a plane on one word, serialised by the LDS).  Copies are
// PL_CSTRIDE words apart, so equal planes of different copies fall on
// different banks.  (Placing through one cursor per copy as well spread the
// lanes of a plane over sixteen ranges and broke up the stores: twice as
// slow; placement keeps one cursor per plane.)
constexpr int PL_COPIES = 16, PL_CSTRIDE = 65;
static_assert(PL_WIN <= 2 * HIT_CHUNK, "a window spans at most three chunks");

// Barrier for hand-offs through LDS only: waits for this wave's LDS
// operations, not for its global stores, which stay in flight (a full
// __syncthreads would also wait for every store to reach memory).
__device__ __forceinline__ void lds_barrier() {
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// records of one window held by a thread (path ids only with KEYS)
template <bool KEYS>
struct Window {
    float x[PL_UNROLL], y[PL_UNROLL];
    uint32_t e[PL_UNROLL];
    int k[PL_UNROLL];            // plane, -1 for no record
    uint32_t lo[KEYS ? PL_UNROLL : 1], hi[KEYS ? PL_UNROLL : 1];
};

// Shared state of the chain walk of the current shower.
struct Chain {
    int c0, f0;                  // chunk and offset of the first record
    int cur_h, cur_c;            // last chunk reached (hop index, chunk id)
    int win[3];                  // chunks of the current window
    int bad;                     // a link pointed outside the log
    int listed;                  // the whole chain is in the chunk list (no walks per window)
};

// Thread 0 walks a shower's whole chain once and lists its chunk ids in LDS
// (when it has at most PL_CLIST chunks): every window then finds its chunks
// there, with no walk and no barrier per window.
__device__ __forceinline__ void list_chain(const PlaceParams &Q, Chain &ch, int *clist, int nh) {
    ch.listed = 0;
    if (ch.bad || nh <= 0) return;
    const int nch = ((ch.f0 + nh - 1) >> HIT_CHUNK_LOG2) + 1;
    if (nch > PL_CLIST) return;
    int c = ch.c0;
    clist[0] = c;
    for (int h = 1; h < nch; ++h) {
        c = (int)Q.hnext[c];
        if (c < 0 || c >= Q.h_chunks) {
            ch.bad = 1;
            return;
        }
        clist[h] = c;
    }
    ch.listed = 1;
}

// Thread 0 follows the links up to the chunks of window w (records
// [w*PL_WIN, min(nh, (w+1)*PL_WIN))); every thread then reads them from ch.
// The barrier on entry keeps thread 0 from rewriting the window's chunk ids
// while other waves still read those of the previous window.
__device__ __forceinline__ void walk_to_window(const PlaceParams &Q, Chain &ch, int w, int nh) {
    lds_barrier();
    if (threadIdx.x == 0 && !ch.bad) {
        const int lo = (ch.f0 + w * PL_WIN) >> HIT_CHUNK_LOG2;
        const int hi = (ch.f0 + min(nh, (w + 1) * PL_WIN) - 1) >> HIT_CHUNK_LOG2;
        int h = ch.cur_h, c = ch.cur_c;
        if (h > lo) {                // new pass: start over
            h = 0;
            c = ch.c0;
        }
        while (h < lo && c >= 0) {
            c = (int)Q.hnext[c];
            c = c < Q.h_chunks ? c : -1;
            ++h;
        }
        ch.cur_h = h;
        ch.cur_c = c;
        for (int q = 0; q <= hi - lo; ++q) {
            ch.win[q] = c;
            if (c < 0) ch.bad = 1;
            if (q < hi - lo && c >= 0) {
                c = (int)Q.hnext[c];
                c = c < Q.h_chunks ? c : -1;
            }
        }
    }
    lds_barrier();
}

template <bool KEYS>
__device__ __forceinline__ Window<KEYS> empty_window() {
    Window<KEYS> W;
#pragma unroll
    for (int u = 0; u < PL_UNROLL; ++u) {
        W.x[u] = W.y[u] = 0.0f;
        W.e[u] = 0u;
        W.k[u] = -1;
        if (KEYS) W.lo[KEYS ? u : 0] = W.hi[KEYS ? u : 0] = 0u;
    }
    return W;
}

// Records of window w held by this thread (after walk_to_window(w); nothing
// when a link of the chain was bad).
template <bool KEYS>
__device__ __forceinline__ Window<KEYS> load_window(const PlaceParams &Q, const Chain &ch, const int *clist, int w,
                                                   int nh) {
    Window<KEYS> W = empty_window<KEYS>();
    if (ch.bad) return W;
    const int lo = (ch.f0 + w * PL_WIN) >> HIT_CHUNK_LOG2;
    const bool listed = ch.listed;
#pragma unroll
    for (int u = 0; u < PL_UNROLL; ++u) {
        const int j = w * PL_WIN + u * PL_THREADS + (int)threadIdx.x;
        if (j < nh) {
            const int pos = ch.f0 + j;
            const int hop = (pos >> HIT_CHUNK_LOG2) - lo;
            const int c = listed ? clist[pos >> HIT_CHUNK_LOG2] : (hop >= 0 && hop < 3) ? ch.win[hop] : -1;
            if (c < 0 || c >= Q.h_chunks) continue;          // never outside the log
            const uint32_t *chunk = Q.hlog + (int64_t)c * HIT_CHUNK_WORDS;
            const int o = pos & (HIT_CHUNK - 1);
            const uint32_t *rec = chunk + HIT_REC_WORDS * o;
            W.x[u] = __uint_as_float(rec[0]);
            W.y[u] = __uint_as_float(rec[1]);
            W.e[u] = rec[2];
            W.k[u] = (int)((const uint8_t *)(chunk + HIT_PLANE_OFF))[o];
            if (KEYS) {
                const uint2 kk = *(const uint2 *)(chunk + HIT_KEY_OFF + HIT_KEY_WORDS * o);
                W.lo[KEYS ? u : 0] = kk.x;
                W.hi[KEYS ? u : 0] = kk.y;
            }
        }
    }
    return W;
}

template <bool KEYS>
__device__ __forceinline__ void count_planes(const Window<KEYS> &W, uint32_t *hcnt, int N) {
    uint32_t *const mine = hcnt + (threadIdx.x & (PL_COPIES - 1)) * PL_CSTRIDE;
#pragma unroll
    for (int u = 0; u < PL_UNROLL; ++u)
        if (W.k[u] >= 0 && W.k[u] < N) atomicAdd(&mine[W.k[u]], 1u);
}

// counts per plane of window w (after walk_to_window(w)) from the plane bytes
// alone: one byte per record read instead of the whole record
__device__ __forceinline__ void count_window_planes(const PlaceParams &Q, const Chain &ch, const int *clist, int w,
                                                    int nh, uint32_t *hcnt, int N) {
    if (ch.bad) return;
    uint32_t *const mine = hcnt + (threadIdx.x & (PL_COPIES - 1)) * PL_CSTRIDE;
    const int lo = (ch.f0 + w * PL_WIN) >> HIT_CHUNK_LOG2;
    const bool listed = ch.listed;
#pragma unroll
    for (int u = 0; u < PL_UNROLL; ++u) {
        const int j = w * PL_WIN + u * PL_THREADS + (int)threadIdx.x;
        if (j < nh) {
            const int pos = ch.f0 + j;
            const int hop = (pos >> HIT_CHUNK_LOG2) - lo;
            const int c = listed ? clist[pos >> HIT_CHUNK_LOG2] : (hop >= 0 && hop < 3) ? ch.win[hop] : -1;
            if (c < 0 || c >= Q.h_chunks) continue;          // never outside the log
            const int k = ((const uint8_t *)(Q.hlog + (int64_t)c * HIT_CHUNK_WORDS + HIT_PLANE_OFF))[pos & (HIT_CHUNK - 1)];
            if (k < N) atomicAdd(&mine[k], 1u);
        }
    }
}

// counts per plane of a listed shower's records beyond window 0 from their
// plane bytes, sixteen at a time: one 16-byte load per thread and aligned
// group of sixteen chain positions (a group never straddles a chunk), two
// groups in flight per thread; bytes outside the shower are skipped.  (Read
// window by window, one byte per thread and record, the count pass of a
// large shower was a chain of dependent round trips.)
__device__ __forceinline__ void count_listed_planes(const PlaceParams &Q, const Chain &ch, const int *clist,
                                                    int nh, uint32_t *hcnt, int N) {
    if (ch.bad) return;
    uint32_t *const mine = hcnt + (threadIdx.x & (PL_COPIES - 1)) * PL_CSTRIDE;
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    typedef __attribute__((address_space(1))) const u32x4 gcu4;
    const int p0 = ch.f0 + PL_WIN, p1 = ch.f0 + nh;
    const int g0 = p0 >> 4, g1 = (p1 + 15) >> 4;
    auto group = [&](int g) -> uint4 {
        const int pos = g << 4;
        const int c = clist[pos >> HIT_CHUNK_LOG2];
        if (c < 0 || c >= Q.h_chunks) return make_uint4(~0u, ~0u, ~0u, ~0u);   // never outside the log
        const uint8_t *pb = (const uint8_t *)(Q.hlog + (int64_t)c * HIT_CHUNK_WORDS + HIT_PLANE_OFF);
        const u32x4 v = *(gcu4 *)(pb + (pos & (HIT_CHUNK - 1)));
        return make_uint4(v.x, v.y, v.z, v.w);
    };
    auto add = [&](int g, uint4 b) {
        const uint32_t wv[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int p = (g << 4) + q;
            const int k = (int)((wv[q >> 2] >> (8 * (q & 3))) & 255u);
            if (p >= p0 && p < p1 && k < N) atomicAdd(&mine[k], 1u);
        }
    };
    for (int g = g0 + (int)threadIdx.x; g < g1; g += 2 * PL_THREADS) {
        const int g2 = g + PL_THREADS;
        const uint4 a = group(g);
        const uint4 b = g2 < g1 ? group(g2) : make_uint4(~0u, ~0u, ~0u, ~0u);
        add(g, a);
        if (g2 < g1) add(g2, b);
    }
}

template <bool KEYS>
__device__ __forceinline__ void place_hits(const PlaceParams &Q, const Window<KEYS> &W, uint32_t *cur,
                                           const int32_t *lay, int64_t seg, int nh, int N) {
#pragma unroll
    for (int u = 0; u < PL_UNROLL; ++u) {
        const int k = W.k[u];
        if (k < 0 || k >= N) continue;
        const uint32_t r = atomicAdd(&cur[k], 1u);
        if (r >= (uint32_t)nh) continue;                  // never outside the segment
        const int64_t o = seg + r;
        Q.hx[o] = W.x[u];
        Q.hy[o] = W.y[u];
        Q.he[o] = (float)W.e[u] * Q.e_unscale;
        Q.hl[o] = lay[k];
        if (KEYS) Q.hk[o] = ((uint64_t)W.hi[KEYS ? u : 0] << 32) | W.lo[KEYS ? u : 0];
    }
}

// Hit fields of a segment staged in the LDS slab: x, y, energy (float bits)
// and layer, PL_WIN words each, at the hit's place within the segment.
static_assert(PL_STAGE_WORDS <= PL_SLAB_WORDS, "a staged segment fits the slab");

template <bool KEYS>
__device__ __forceinline__ void stage_hits(const PlaceParams &Q, const Window<KEYS> &W, uint32_t *cur,
                                           const int32_t *lay, uint32_t *slab, int64_t seg, int nh, int N) {
#pragma unroll
    for (int u = 0; u < PL_UNROLL; ++u) {
        const int k = W.k[u];
        if (k < 0 || k >= N) continue;
        const uint32_t r = atomicAdd(&cur[k], 1u);
        if (r >= (uint32_t)nh) continue;                  // nh <= PL_WIN: inside the slab
        slab[r] = __float_as_uint(W.x[u]);
        slab[PL_WIN + r] = __float_as_uint(W.y[u]);
        slab[2 * PL_WIN + r] = __float_as_uint((float)W.e[u] * Q.e_unscale);
        slab[3 * PL_WIN + r] = (uint32_t)lay[k];
        if (KEYS) Q.hk[seg + r] = ((uint64_t)W.hi[KEYS ? u : 0] << 32) | W.lo[KEYS ? u : 0];
    }
}

// (and leaves the slab zero again)
__device__ __forceinline__ void copy_out_hits(const PlaceParams &Q, uint32_t *slab, int64_t seg, int nh) {
    for (int q = (int)threadIdx.x; q < nh; q += PL_THREADS) {
        Q.hx[seg + q] = __uint_as_float(slab[q]);
        Q.hy[seg + q] = __uint_as_float(slab[PL_WIN + q]);
        Q.he[seg + q] = __uint_as_float(slab[2 * PL_WIN + q]);
        Q.hl[seg + q] = (int32_t)slab[3 * PL_WIN + q];
        slab[q] = slab[PL_WIN + q] = slab[2 * PL_WIN + q] = slab[3 * PL_WIN + q] = 0u;
    }
}

// Image row and column of each hit of a window (row -1: outside the window or
// not read out); the same arithmetic as binning.
template <bool KEYS>
__device__ __forceinline__ void cells(const PlaceParams &Q, const Window<KEYS> &W, const int32_t *lay,
                                      int N, int (&row)[PL_UNROLL], int (&col)[PL_UNROLL]) {
#pragma unroll
    for (int u = 0; u < PL_UNROLL; ++u) {
        const int k = W.k[u];
        const int l = (k >= 0 && k < N) ? lay[k] : -1;
        const float cx = floorf((W.x[u] - Q.x0) * Q.sx);
        const float cy = floorf((W.y[u] - Q.y0) * Q.sy);
        const bool in = l >= 0 && cx >= 0.0f && cx < (float)Q.nx && cy >= 0.0f && cy < (float)Q.ny;
        row[u] = in ? l * Q.ny + (int)cy : -1;
        col[u] = in ? (int)cx : 0;
    }
}

// adds the window's hits that fall in image rows [row0, row0 + rows) to the slab
template <bool KEYS>
__device__ __forceinline__ void bin_window(const PlaceParams &Q, const Window<KEYS> &W, const int32_t *lay,
                                           uint32_t *slab, int row0, int rows, int N) {
#pragma unroll
    for (int u = 0; u < PL_UNROLL; ++u) {
        const int k = W.k[u];
        const int l = (k >= 0 && k < N) ? lay[k] : -1;
        const float cx = floorf((W.x[u] - Q.x0) * Q.sx);
        const float cy = floorf((W.y[u] - Q.y0) * Q.sy);
        const bool in = l >= 0 && cx >= 0.0f && cx < (float)Q.nx && cy >= 0.0f && cy < (float)Q.ny;
        const int r = (in ? l * Q.ny + (int)cy : -1) - row0;
        if (in && r >= 0 && r < rows) atomicAdd(&slab[r * Q.nx + (int)cx], W.e[u]);
    }
}

// streams the slab out as float and leaves it zero
__device__ __forceinline__ void write_slab(const PlaceParams &Q, uint32_t *slab, float *dst, int words) {
    if ((words & 3) == 0 && (((uintptr_t)dst) & 15) == 0) {
        for (int q = 4 * (int)threadIdx.x; q < words; q += 4 * PL_THREADS) {
            const uint4 v = *(const uint4 *)(slab + q);
            *(uint4 *)(slab + q) = make_uint4(0u, 0u, 0u, 0u);
            // streamed out once: non-temporal
            typedef float f4 __attribute__((ext_vector_type(4)));
            const f4 f = {(float)v.x * Q.e_unscale, (float)v.y * Q.e_unscale,
                          (float)v.z * Q.e_unscale, (float)v.w * Q.e_unscale};
            __builtin_nontemporal_store(f, (f4 *)(dst + q));
        }
    } else {
        for (int q = (int)threadIdx.x; q < words; q += PL_THREADS) {
            dst[q] = (float)slab[q] * Q.e_unscale;
            slab[q] = 0u;
        }
    }
}

// a slab without hits: zeros straight to memory
__device__ __forceinline__ void write_zeros(float *dst, int words) {
    if ((words & 3) == 0 && (((uintptr_t)dst) & 15) == 0) {
        typedef float f4 __attribute__((ext_vector_type(4)));
        const f4 z = {0.0f, 0.0f, 0.0f, 0.0f};
        for (int q = 4 * (int)threadIdx.x; q < words; q += 4 * PL_THREADS)
            __builtin_nontemporal_store(z, (f4 *)(dst + q));
    } else {
        for (int q = (int)threadIdx.x; q < words; q += PL_THREADS) dst[q] = 0.0f;
    }
}

__device__ __forceinline__ void clear_slab(uint32_t *slab, int words) {
    int q = 4 * (int)threadIdx.x;
    for (; q + 3 < words; q += 4 * PL_THREADS) *(uint4 *)(slab + q) = make_uint4(0u, 0u, 0u, 0u);
    for (int r = (words & ~3) + (int)threadIdx.x; r < words; r += PL_THREADS) slab[r] = 0u;
}

// Variants (MODE): hit clouds only (LDS: the 32 KB staging area); images
// (a 64 KB slab: the 20 layers of 32x32 of a shower in two slabs); images
// whose hits are first sorted by slab (many slabs per shower).  KEYS writes
// path ids.  The hit-cloud variant without ids is held to 64 VGPRs so that
// four 512-thread workgroups share a compute unit.
enum { PM_HITS = 0, PM_IMAGES = 1, PM_BUCKET = 2 };

// dynamic LDS words of a variant: slab (or staging area), and the per-slab
// counts when bucketing
constexpr int place_lds_words(int mode) {
    return mode == PM_HITS ? PL_STAGE_WORDS : PL_SLAB_WORDS + (mode == PM_BUCKET ? PL_MAX_SLABS + 1 : 0);
}

template <bool KEYS, int MODE>
__global__ void __launch_bounds__(PL_THREADS)
__attribute__((amdgpu_waves_per_eu((!KEYS && MODE == PM_HITS) ? 8 : 1))) supa_place(PlaceParams Q) {
    constexpr bool BUCKET = MODE == PM_BUCKET;
    extern __shared__ __attribute__((aligned(16))) uint32_t slab[];    // zero between uses; 16-byte aligned for b128
    uint32_t *const scnt = slab + PL_SLAB_WORDS;       // [PL_MAX_SLABS + 1], BUCKET only
    __shared__ int32_t lay[64];
    __shared__ int32_t pord[64];     // planes in order of (layer, plane)
    __shared__ uint32_t cnt[64];
    __shared__ uint32_t hcnt[PL_COPIES * PL_CSTRIDE];     // zero between showers
    __shared__ Chain ch;
    __shared__ int clist[PL_CLIST];
    // records are valid only when the propagation succeeded; hit outputs
    // only when they all fit
    if (batch_failed(Q.ctr)) return;
    const bool hits = Q.hx != nullptr, img = MODE != PM_HITS && Q.images != nullptr;
    if (hits && (int64_t)Q.sub[SUB_HITS] > Q.hcap) return;
    const int N = Q.n_planes;
    if (threadIdx.x < 64) lay[threadIdx.x] = (int)threadIdx.x < N ? Q.layer[threadIdx.x] : -1;
    lds_barrier();
    if (threadIdx.x < 64) {
        // the rank of plane t among the planes in order of (layer, plane);
        // planes past the last keep their place (they have no hits)
        const int t = (int)threadIdx.x;
        int r = t;
        if (t < N) {
            r = 0;
            for (int k = 0; k < N; ++k) r += (lay[k] < lay[t] || (lay[k] == lay[t] && k < t)) ? 1 : 0;
        }
        pord[r] = t;
    }
    clear_slab(slab, MODE == PM_HITS ? PL_STAGE_WORDS : PL_SLAB_WORDS);
    for (int q = (int)threadIdx.x; q < PL_COPIES * PL_CSTRIDE; q += PL_THREADS) hcnt[q] = 0u;
    const int total_rows = Q.L * Q.ny;

    for (int i = blockIdx.x; i < Q.n; i += gridDim.x) {
        const int nh = Q.counts[6 * (int64_t)i + 1];
        const int64_t st = Q.hstart[i];
        if (threadIdx.x == 0) {
            ch.c0 = st >= 0 ? (int)(st >> HIT_CHUNK_LOG2) : -1;
            ch.f0 = (int)(st & (HIT_CHUNK - 1));
            ch.cur_h = 0;
            ch.cur_c = ch.c0;
            ch.bad = (nh > 0 && (st < 0 || ch.c0 >= Q.h_chunks)) ? 1 : 0;
            list_chain(Q, ch, clist, nh);
        }
        lds_barrier();
        const int nwin = (nh + PL_WIN - 1) / PL_WIN;
        // window 0 stays in registers for every pass; a listed chain needs no
        // walk (ch.listed is uniform: read after the barrier)
        const bool listed = ch.listed;
        if (!listed) walk_to_window(Q, ch, 0, nh);
        const bool ok = !ch.bad;
        const Window<KEYS> W0 = load_window<KEYS>(Q, ch, clist, 0, nh);

        if (hits && ok) {
            const int64_t seg = Q.hoff[i];
            if (seg >= 0 && seg + nh <= Q.hcap) {
                // hits per plane -> first place of each plane in the segment
                count_planes(W0, hcnt, N);
                if (listed) {
                    count_listed_planes(Q, ch, clist, nh, hcnt, N);
                } else {
                    for (int w = 1; w < nwin; ++w) {
                        walk_to_window(Q, ch, w, nh);
                        count_window_planes(Q, ch, clist, w, nh, hcnt, N);
                    }
                }
                lds_barrier();
                if (threadIdx.x < 64) {
                    // the copies summed (and cleared for the next shower),
                    // plane totals -> plane starts, thread t taking the t-th
                    // plane in order of (layer, plane)
                    const int pl = pord[threadIdx.x];
                    uint32_t v = 0u;
#pragma unroll
                    for (int c = 0; c < PL_COPIES; ++c) {
                        v += hcnt[c * PL_CSTRIDE + pl];
                        hcnt[c * PL_CSTRIDE + pl] = 0u;
                    }
                    uint32_t incl = v;
#pragma unroll
                    for (int off = 1; off < 64; off <<= 1) {
                        const uint32_t t = __shfl_up(incl, off, 64);
                        if ((int)threadIdx.x >= off) incl += t;
                    }
                    cnt[pl] = incl - v;
                }
                lds_barrier();
                if (nh <= PL_WIN) {
                    // the whole segment fits the LDS slab: sort into it, then
                    // write it out with contiguous stores
                    stage_hits(Q, W0, cnt, lay, slab, seg, nh, N);
                    lds_barrier();
                    copy_out_hits(Q, slab, seg, nh);
                    lds_barrier();
                } else {
                    place_hits(Q, W0, cnt, lay, seg, nh, N);
                    for (int w = 1; w < nwin; ++w) {
                        if (!listed) walk_to_window(Q, ch, w, nh);
                        place_hits(Q, load_window<KEYS>(Q, ch, clist, w, nh), cnt, lay, seg, nh, N);
                    }
                }
            }
        }

        const int nslab = (total_rows + Q.slab_rows - 1) / Q.slab_rows;
        if (BUCKET && img && ok && Q.bucket && nslab >= PL_BUCKET_MIN_SLABS && nslab <= PL_MAX_SLABS &&
            nh <= Q.bucket_cap) {
            // many slabs: sort the shower's binned hits by slab first (counts
            // in LDS, entries in the workgroup's global bucket), so that each
            // slab adds only its own hits
            float *dst = Q.images + (int64_t)i * total_rows * Q.nx;
            uint2 *bk = Q.bucket + (int64_t)blockIdx.x * Q.bucket_cap;
            for (int q = (int)threadIdx.x; q <= nslab; q += PL_THREADS) scnt[q] = 0u;
            lds_barrier();
            for (int w = 0; w < nwin; ++w) {
                if (w > 0 && !listed) walk_to_window(Q, ch, w, nh);
                const Window<KEYS> W = w == 0 ? W0 : load_window<KEYS>(Q, ch, clist, w, nh);
                int row[PL_UNROLL], col[PL_UNROLL];
                cells(Q, W, lay, N, row, col);
#pragma unroll
                for (int u = 0; u < PL_UNROLL; ++u)
                    if (row[u] >= 0) atomicAdd(&scnt[row[u] / Q.slab_rows + 1], 1u);
            }
            lds_barrier();
            if (threadIdx.x < 64) {
                // scnt[1 + s] -> start of slab s, in place (one wave, 64 per pass)
                uint32_t carry = 0u;
                for (int b0 = 1; b0 <= nslab; b0 += 64) {
                    const int q = b0 + (int)threadIdx.x;
                    const uint32_t v = q <= nslab ? scnt[q] : 0u;
                    uint32_t incl = v;
#pragma unroll
                    for (int off = 1; off < 64; off <<= 1) {
                        const uint32_t t = __shfl_up(incl, off, 64);
                        if ((int)threadIdx.x >= off) incl += t;
                    }
                    if (q <= nslab) scnt[q] = carry + incl - v;
                    carry += __shfl(incl, 63, 64);
                }
                if (threadIdx.x == 0) scnt[0] = carry;      // binned hits in all
            }
            lds_barrier();
            // scnt[1 + s] now runs as the fill cursor of slab s
            for (int w = 0; w < nwin; ++w) {
                if (w > 0 && !listed) walk_to_window(Q, ch, w, nh);
                const Window<KEYS> W = w == 0 ? W0 : load_window<KEYS>(Q, ch, clist, w, nh);
                int row[PL_UNROLL], col[PL_UNROLL];
                cells(Q, W, lay, N, row, col);
#pragma unroll
                for (int u = 0; u < PL_UNROLL; ++u) {
                    if (row[u] < 0) continue;
                    const int sl = row[u] / Q.slab_rows;
                    const uint32_t pos = atomicAdd(&scnt[sl + 1], 1u);
                    if (pos < (uint32_t)Q.bucket_cap)
                        bk[pos] = make_uint2((uint32_t)((row[u] - sl * Q.slab_rows) * Q.nx + col[u]), W.e[u]);
                }
            }
            __syncthreads();                 // the bucket entries (global) are visible
            // after the fill, scnt[1 + s] is the end of slab s: starts are the
            // previous slab's end
            for (int sl = 0; sl < nslab; ++sl) {
                const int row0 = sl * Q.slab_rows;
                const int rows = min(total_rows - row0, Q.slab_rows);
                const int words = rows * Q.nx;
                const uint32_t b0 = sl == 0 ? 0u : scnt[sl];
                const uint32_t b1 = min(scnt[sl + 1], (uint32_t)Q.bucket_cap);
                if (b0 == b1) {
                    write_zeros(dst + (int64_t)row0 * Q.nx, words);
                    continue;
                }
                for (uint32_t q = b0 + threadIdx.x; q < b1; q += PL_THREADS) {
                    const uint2 v = bk[q];
                    if (v.x < (uint32_t)words) atomicAdd(&slab[v.x], v.y);
                }
                lds_barrier();
                write_slab(Q, slab, dst + (int64_t)row0 * Q.nx, words);
                lds_barrier();
            }
        } else if (img) {
            float *dst = Q.images + (int64_t)i * total_rows * Q.nx;
            for (int row0 = 0; row0 < total_rows; row0 += Q.slab_rows) {
                const int rows = min(total_rows - row0, Q.slab_rows);
                const int words = rows * Q.nx;
                if (ok) {
                    bin_window(Q, W0, lay, slab, row0, rows, N);
                    for (int w = 1; w < nwin; ++w) {
                        if (!listed) walk_to_window(Q, ch, w, nh);
                        bin_window(Q, load_window<false>(Q, ch, clist, w, nh), lay, slab, row0, rows, N);
                    }
                }
                lds_barrier();
                write_slab(Q, slab, dst + (int64_t)row0 * Q.nx, words);
                lds_barrier();
            }
        }
        lds_barrier();
    }
}

// rows of one LDS slab: whole layers when they fit, else bands of rows
static int slab_rows_for(int nx, int ny) {
    const int64_t lw = (int64_t)ny * nx;
    return lw <= PL_SLAB_WORDS ? (int)(PL_SLAB_WORDS / lw) * ny : std::max(1, PL_SLAB_WORDS / nx);
}

// workgroups of one launch per compute unit (queried once per variant, so no
// runtime query happens while a caller captures a graph)
template <bool KEYS, int MODE>
static int place_per_cu_of() {
    static int per_cu = 0;
    if (per_cu == 0) {
        int q = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&q, (const void *)supa_place<KEYS, MODE>, PL_THREADS,
                                                         place_lds_words(MODE) * 4) != hipSuccess ||
            q < 1) {
            (void)hipGetLastError();
            q = 1;
        }
        per_cu = q;
    }
    return per_cu;
}

static int place_per_cu(bool keys, int mode) {
    switch (mode) {
    case PM_HITS: return keys ? place_per_cu_of<true, PM_HITS>() : place_per_cu_of<false, PM_HITS>();
    case PM_IMAGES: return keys ? place_per_cu_of<true, PM_IMAGES>() : place_per_cu_of<false, PM_IMAGES>();
    default: return keys ? place_per_cu_of<true, PM_BUCKET>() : place_per_cu_of<false, PM_BUCKET>();
    }
}

// slabs of one image set of L x ny x nx
static int slabs_of(int L, int nx, int ny) {
    const int rows = slab_rows_for(nx, ny);
    return (L * ny + rows - 1) / rows;
}

static bool bucketed(int L, int nx, int ny) {
    const int slabs = slabs_of(L, nx, ny);
    return slabs >= PL_BUCKET_MIN_SLABS && slabs <= PL_MAX_SLABS;
}

// Bucket scratch the placement of images of L x ny x nx needs: entries per
// workgroup (0: none) and workgroups.
void place_bucket_size(int L, int nx, int ny, bool keys, int n_cu, int64_t *per_block, int64_t *blocks) {
    const bool b = bucketed(L, nx, ny);
    *per_block = b ? 65536 : 0;
    *blocks = (int64_t)n_cu * place_per_cu(keys, b ? PM_BUCKET : PM_IMAGES);
}

template <bool KEYS>
static void launch_mode(const PlaceParams &P, int mode, int blocks, hipStream_t s) {
    const size_t lds = (size_t)place_lds_words(mode) * 4;
    if (mode == PM_HITS)
        hipLaunchKernelGGL((supa_place<KEYS, PM_HITS>), dim3(blocks), dim3(PL_THREADS), lds, s, P);
    else if (mode == PM_IMAGES)
        hipLaunchKernelGGL((supa_place<KEYS, PM_IMAGES>), dim3(blocks), dim3(PL_THREADS), lds, s, P);
    else
        hipLaunchKernelGGL((supa_place<KEYS, PM_BUCKET>), dim3(blocks), dim3(PL_THREADS), lds, s, P);
}

hipError_t launch_place(const PlaceParams &P0, int n_cu, hipStream_t s) {
    if (P0.n <= 0 || (!P0.hx && !P0.images)) return hipSuccess;
    PlaceParams P = P0;
    if (P.images) P.slab_rows = slab_rows_for(P.nx, P.ny);
    // the bucketing variant only where its scratch was sized
    const int mode = !P.images ? PM_HITS : (P.bucket && bucketed(P.L, P.nx, P.ny)) ? PM_BUCKET : PM_IMAGES;
    const bool keys = P.hk != nullptr;
    // as many workgroups as fit on the device at once (each loops over showers)
    const int blocks = (int)std::min<int64_t>(P.n, (int64_t)n_cu * place_per_cu(keys, mode));
    if (keys)
        launch_mode<true>(P, mode, blocks, s);
    else
        launch_mode<false>(P, mode, blocks, s);
    return hipGetLastError();
}

}  // namespace supa
