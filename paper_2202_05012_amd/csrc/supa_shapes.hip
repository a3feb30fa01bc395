// supa_shapes.hip -- evaluation kernels of include/supa_shapes.h: shower
// shape variables of hit point clouds (paper, section "Shower Shape
// Variables" and appendix "More shower shape variables") and the normalised
// Wasserstein-1 distance between histograms of two samples (section
// "Performance Analysis of Generative Models").
//
// Shape variables: one lane per shower.  A lane streams its shower's segment
// of the hit arrays in aligned blocks of four hits (one 16-byte load per
// array), keeps the double-precision sums of the layer run it is in, and
// writes that layer's record when the run ends; lanes take showers from a
// queue (one atomic counter), so a lane that finishes a short shower goes on
// with the next one.  HBM traffic is one read of the hits and one write of
// the records.
//
// W1: per column, (1) count, shifted sums and min/max of both samples (per
// block partials, reduced in a fixed order), (2) one histogram per sample
// over the shared range (LDS histograms of a tile of columns, added into the
// global ones with integer atomics: exact), (3) one wave per column walks the
// cumulative counts.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <string>

#include "../../include/supa_shapes.h"

namespace {

constexpr int WAVE = 64;
constexpr int LV = SUPA_LAYER_VARS;
constexpr int SV = SUPA_SHOWER_VARS;

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

struct ShapeArgs {
    int64_t n;
    int L;
    const int64_t *off;
    const int32_t *cnt;
    int cstride;
    int64_t len;  // entries of each hit array
    const float *x, *y, *e;
    const int32_t *layer;
    float *lv, *sv;
    int32_t *work;         // [0] showers in error, [1] next shower (queue)
    const int32_t *order;  // [n] showers in the order they are taken
};

// Sums of one layer run, in double precision.
struct Run {
    double sx, sxx, sy, syy, sr, se, see, sex, sexx, sey, seyy, ser;
    int n;
    float e1, e2;  // the two largest point energies
};

// sqrt of s >= 0: hardware reciprocal square root, then one Newton step on
// the residual (relative error about 1e-15), 0 for s = 0.
__device__ inline double sqrt_pos(double s) {
    const double y = __builtin_amdgcn_rsq(s);
    const double r0 = s * y;
    const double e = __builtin_fma(-r0, r0, s);
    const double r = __builtin_fma(0.5 * y, e, r0);
    return s > 0.0 ? r : 0.0;
}

// 1 / v for v > 0: hardware reciprocal and two Newton steps (about 1 ulp).
__device__ inline double recip(double v) {
    double y = __builtin_amdgcn_rcp(v);
    y = __builtin_fma(__builtin_fma(-v, y, 1.0), y, y);
    y = __builtin_fma(__builtin_fma(-v, y, 1.0), y, y);
    return y;
}

__device__ inline void run_clear(Run &a) {
    a.sx = a.sxx = a.sy = a.syy = a.sr = a.se = a.see = 0.0;
    a.sex = a.sexx = a.sey = a.seyy = a.ser = 0.0;
    a.n = 0;
    a.e1 = a.e2 = -__builtin_inff();
}

// Adds one point when `take` (otherwise adds zeros: no branch).
__device__ inline void run_add(Run &a, float xf, float yf, float ef, bool take) {
    const double x = take ? xf : 0.0f, y = take ? yf : 0.0f, e = take ? ef : 0.0f;
    const double xx = x * x, yy = y * y;
    const double r = sqrt_pos(xx + yy);
    const double ex = e * x, ey = e * y;
    a.sx += x;
    a.sxx += xx;
    a.sy += y;
    a.syy += yy;
    a.sr += r;
    a.se += e;
    a.see = __builtin_fma(e, e, a.see);
    a.sex += ex;
    a.sexx = __builtin_fma(ex, x, a.sexx);
    a.sey += ey;
    a.seyy = __builtin_fma(ey, y, a.seyy);
    a.ser = __builtin_fma(e, r, a.ser);
    a.n += take ? 1 : 0;
    const float et = take ? ef : -__builtin_inff();  // running two largest
    a.e2 = __builtin_fmaxf(a.e2, __builtin_fminf(a.e1, et));
    a.e1 = __builtin_fmaxf(a.e1, et);
}

__device__ inline float dev_of(double m1, double m2) {
    const double v = __builtin_fma(-m1, m1, m2);
    return __builtin_amdgcn_sqrtf((float)(v > 0.0 ? v : 0.0));
}

// Writes every field of a layer record except FRACTION.  Sum of E r^2 is
// sum E x^2 + sum E y^2; sum r^2 is sum x^2 + sum y^2.
__device__ inline void write_layer(float *rec, const Run &a) {
    const float nan = __builtin_nanf("");
    const double in = recip((double)a.n);
    const double mx = a.sx * in, my = a.sy * in, mr = a.sr * in, me = a.se * in;
    f32x2 *r2 = (f32x2 *)rec;
    r2[0] = f32x2{(float)a.n, (float)mx};
    r2[1] = f32x2{(float)my, (float)mr};
    r2[2] = f32x2{(float)me, dev_of(mx, a.sxx * in)};
    r2[3] = f32x2{dev_of(my, a.syy * in), dev_of(mr, (a.sxx + a.syy) * in)};
    r2[4] = f32x2{dev_of(me, a.see * in), (float)a.se};
    if (a.se > 0.0) {
        const double ie = recip(a.se);
        const double cx = a.sex * ie, cy = a.sey * ie, cr = a.ser * ie;
        r2[5] = f32x2{(float)cx, (float)cy};
        r2[6] = f32x2{(float)cr, dev_of(cx, a.sexx * ie)};
        r2[7] = f32x2{dev_of(cy, a.seyy * ie), dev_of(cr, (a.sexx + a.seyy) * ie)};
    } else {
        r2[5] = f32x2{nan, nan};
        r2[6] = f32x2{nan, nan};
        r2[7] = f32x2{nan, nan};
    }
    const double e1 = a.e1, e2 = a.n > 1 ? (double)a.e2 : 0.0;  // E[2] = 0 for one point
    rec[SUPA_LV_ENERGY_RATIO] = (e1 + e2 > 0.0) ? (float)((e1 - e2) / (e1 + e2)) : nan;
}

__device__ inline void write_empty_layer(float *rec) {
    const float nan = __builtin_nanf("");
    f32x2 *r2 = (f32x2 *)rec;
    r2[0] = f32x2{0.0f, nan};
    r2[1] = f32x2{nan, nan};
    r2[2] = f32x2{nan, nan};
    r2[3] = f32x2{nan, nan};
    r2[4] = f32x2{nan, 0.0f};
    r2[5] = f32x2{nan, nan};
    r2[6] = f32x2{nan, nan};
    r2[7] = f32x2{nan, nan};
    rec[SUPA_LV_ENERGY_RATIO] = nan;
}

// work: [0] showers in error, [1] queue, [2, 4) unused, then the global
// order's bucket sizes and cursors (ORDER_BUCKETS each), then the order [n].
constexpr int ORDER_BUCKETS = 1024;
constexpr int WORK_HEAD = 4 + 2 * ORDER_BUCKETS;

__global__ void shapes_clear(int32_t *work) {
    for (int i = threadIdx.x; i < WORK_HEAD; i += blockDim.x) work[i] = 0;
}

// Order in which the lanes take showers: longest first, within windows of
// consecutive showers.  A wave's lanes then carry showers of similar length,
// so fewer lanes idle while the longest one finishes.  When every shower is
// in flight at once (one per lane) the window is the whole batch, sorted by
// two kernels (global bucket sizes, then each block reserves its range of
// every bucket with one atomic); otherwise windows of ORDER_WIN keep the
// showers in flight close together in memory, each sorted by one workgroup,
// and hold 63 waves' worth of showers so that the first (longest) wave of
// consecutive windows falls on different XCDs.  Both are counting sorts into
// 1024 buckets of the hit count on a log scale (32 per octave); the order
// within a bucket is whatever the atomics give, which changes no result (each
// shower is summed by one lane in its own hit order).
constexpr int ORDER_WIN = 63 * WAVE;
constexpr int ORDER_THREADS = 1024;

__device__ inline int count_bucket(int32_t c) {  // 0..1023, non-decreasing in c
    const uint32_t v = (c > 0 ? (uint32_t)c : 0u) + 1u;
    const int e = 31 - __builtin_clz(v);
    const uint32_t m = e >= 5 ? (v >> (e - 5)) & 31u : (v << (5 - e)) & 31u;
    return e * 32 + (int)m;
}

// dst[b] = sum of src[0 .. b) over the ORDER_BUCKETS buckets, by one wave
// (lane t < 64 of the caller); dst may be src.
__device__ inline void bucket_starts(const uint32_t *src, uint32_t *dst, int t) {
    constexpr int Q = ORDER_BUCKETS / WAVE;
    uint32_t v[Q], sum = 0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        v[q] = src[t * Q + q];
        sum += v[q];
    }
    uint32_t inc = sum;
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        const uint32_t o = __shfl_up(inc, d);
        if (t >= d) inc += o;
    }
    uint32_t run = inc - sum;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        dst[t * Q + q] = run;
        run += v[q];
    }
}

__global__ void __launch_bounds__(ORDER_THREADS)
    shapes_order(int64_t n, int64_t win, const int32_t *cnt, int cstride, int32_t *order) {
    __shared__ uint32_t hist[ORDER_BUCKETS];
    const int t = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * win;
    const int64_t m = n - base < win ? n - base : win;
    for (int i = t; i < ORDER_BUCKETS; i += ORDER_THREADS) hist[i] = 0;
    __syncthreads();
    for (int64_t i = t; i < m; i += ORDER_THREADS)
        atomicAdd(&hist[ORDER_BUCKETS - 1 - count_bucket(cnt[(size_t)(base + i) * cstride])], 1u);
    __syncthreads();
    if (t < WAVE) bucket_starts(hist, hist, t);
    __syncthreads();
    // hist now holds each bucket's next free position
    for (int64_t i = t; i < m; i += ORDER_THREADS) {
        const int b = ORDER_BUCKETS - 1 - count_bucket(cnt[(size_t)(base + i) * cstride]);
        order[base + atomicAdd(&hist[b], 1u)] = (int32_t)(base + i);
    }
}

// Whole-batch order, pass 1: sizes of the buckets (gsize, zeroed before).
constexpr int ORDER_CHUNK = 4 * ORDER_THREADS;  // showers per block of the two passes

__global__ void __launch_bounds__(ORDER_THREADS)
    shapes_order_sizes(int64_t n, const int32_t *cnt, int cstride, uint32_t *gsize) {
    __shared__ uint32_t hist[ORDER_BUCKETS];
    const int t = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * ORDER_CHUNK;
    const int64_t m = n - base < ORDER_CHUNK ? n - base : ORDER_CHUNK;
    for (int i = t; i < ORDER_BUCKETS; i += ORDER_THREADS) hist[i] = 0;
    __syncthreads();
    for (int64_t i = t; i < m; i += ORDER_THREADS)
        atomicAdd(&hist[ORDER_BUCKETS - 1 - count_bucket(cnt[(size_t)(base + i) * cstride])], 1u);
    __syncthreads();
    for (int i = t; i < ORDER_BUCKETS; i += ORDER_THREADS)
        if (hist[i]) atomicAdd(&gsize[i], hist[i]);
}

// Pass 2: each block reserves its range of every bucket (gcur, zeroed
// before) and places its showers.
__global__ void __launch_bounds__(ORDER_THREADS)
    shapes_order_place(int64_t n, const int32_t *cnt, int cstride, const uint32_t *gsize, uint32_t *gcur,
                       int32_t *order) {
    __shared__ uint32_t hist[ORDER_BUCKETS], start[ORDER_BUCKETS];
    const int t = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * ORDER_CHUNK;
    const int64_t m = n - base < ORDER_CHUNK ? n - base : ORDER_CHUNK;
    for (int i = t; i < ORDER_BUCKETS; i += ORDER_THREADS) {
        hist[i] = 0;
        start[i] = gsize[i];
    }
    __syncthreads();
    if (t < WAVE) bucket_starts(start, start, t);
    int bk[4];
    uint32_t rank[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int64_t i = t + (int64_t)u * ORDER_THREADS;
        bk[u] = i < m ? ORDER_BUCKETS - 1 - count_bucket(cnt[(size_t)(base + i) * cstride]) : -1;
        rank[u] = bk[u] >= 0 ? atomicAdd(&hist[bk[u]], 1u) : 0u;
    }
    __syncthreads();
    for (int i = t; i < ORDER_BUCKETS; i += ORDER_THREADS)
        if (hist[i]) start[i] += atomicAdd(&gcur[i], hist[i]);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u)
        if (bk[u] >= 0) order[start[bk[u]] + rank[u]] = (int32_t)(base + t + (int64_t)u * ORDER_THREADS);
}

// Records of finished layer runs wait in a per-wave LDS ring until 64 are
// ready, then the wave computes and writes 64 records at once (one per lane):
// the division and square roots of a record run with every lane busy instead
// of once per lane whose run happens to end.
constexpr int QCAP = 128;      // ring entries (a step adds at most 64)
constexpr int BLK = 32;        // hits per lane per step: one 128-byte line per array

struct Ring {
    double d[12][QCAP];
    int n[QCAP], s[QCAP], l[QCAP];
    float e1[QCAP], e2[QCAP];
};

// Adds the runs of the lanes with `cond` to the ring at t (wave-uniform).
__device__ inline void ring_put(Ring &q, int &t, bool cond, int s, int l, const Run &a) {
    const uint64_t m = __ballot(cond);
    if (cond) {
        const int slot = (t + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                              __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0))) &
                         (QCAP - 1);
        q.d[0][slot] = a.sx;
        q.d[1][slot] = a.sxx;
        q.d[2][slot] = a.sy;
        q.d[3][slot] = a.syy;
        q.d[4][slot] = a.sr;
        q.d[5][slot] = a.se;
        q.d[6][slot] = a.see;
        q.d[7][slot] = a.sex;
        q.d[8][slot] = a.sexx;
        q.d[9][slot] = a.sey;
        q.d[10][slot] = a.seyy;
        q.d[11][slot] = a.ser;
        q.n[slot] = a.n;
        q.s[slot] = s;
        q.l[slot] = l;
        q.e1[slot] = a.e1;
        q.e2[slot] = a.e2;
    }
    t += __builtin_popcountll(m);
}

// Writes up to `most` (<= 64) records from the ring head h (wave-uniform call).
__device__ inline void ring_drain(Ring &q, int &h, int t, int most, float *lv, int L) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int k = (t - h) < most ? (t - h) : most;
    const int lane = threadIdx.x;
    if (lane < k) {
        const int slot = (h + lane) & (QCAP - 1);
        Run a;
        a.sx = q.d[0][slot];
        a.sxx = q.d[1][slot];
        a.sy = q.d[2][slot];
        a.syy = q.d[3][slot];
        a.sr = q.d[4][slot];
        a.se = q.d[5][slot];
        a.see = q.d[6][slot];
        a.sex = q.d[7][slot];
        a.sexx = q.d[8][slot];
        a.sey = q.d[9][slot];
        a.seyy = q.d[10][slot];
        a.ser = q.d[11][slot];
        a.n = q.n[slot];
        a.e1 = q.e1[slot];
        a.e2 = q.e2[slot];
        write_layer(lv + ((size_t)q.s[slot] * L + q.l[slot]) * LV, a);
    }
    h += k;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One wave per workgroup; static LDS: the ring; dynamic LDS: float [L][64],
// the layer energies of each lane's current shower (for the fractions,
// written once E_tot is known).  Every cross-lane step (ring, drain, exit)
// runs in wave-uniform control flow.
__global__ void __launch_bounds__(WAVE) shapes_kernel(ShapeArgs A) {
    __shared__ Ring q;
    extern __shared__ float ef[];
    const int lane = threadIdx.x;
    const int L = A.L;
    const float nan = __builtin_nanf("");
    uint32_t *queue = (uint32_t *)A.work + 1;

    int h = 0, t = 0;  // ring head and tail (wave-uniform)
    bool active = true;
    int64_t s = -1, pos = 0, end = 0;
    int cur = -1, depth = -1;
    bool bad = false;
    uint64_t seen = 0;
    double etot = 0.0, ld = 0.0, ld2 = 0.0;
    Run acc;
    run_clear(acc);

    for (;;) {
        // --- lanes whose shower is done: last run, empty layers, totals
        const bool closing = active && s >= 0 && pos >= end;
        ring_put(q, t, closing && !bad && cur >= 0, (int)s, cur, acc);
        if (closing && !bad) {
            float *base = A.lv + (size_t)s * L * LV;
            if (cur >= 0) {
                ef[cur * WAVE + lane] = (float)acc.se;
                etot += acc.se;
                ld += (double)cur * acc.se;
                ld2 += (double)cur * (double)cur * acc.se;
                if (acc.se > 0.0 && cur > depth) depth = cur;
            }
            const double it = etot > 0.0 ? recip(etot) : 0.0;
            for (int l = 0; l < L; ++l) {
                float *rec = base + (size_t)l * LV;
                if (!((seen >> l) & 1)) write_empty_layer(rec);
                rec[SUPA_LV_FRACTION] = etot > 0.0 ? (float)((double)ef[l * WAVE + lane] * it) : nan;
            }
            float *sv = A.sv + (size_t)s * SV;
            const double sd = ld * it;
            sv[SUPA_SV_E_TOT] = (float)etot;
            sv[SUPA_SV_DEPTH] = (float)depth;
            sv[SUPA_SV_L_D] = (float)ld;
            sv[SUPA_SV_S_D] = etot > 0.0 ? (float)sd : nan;
            sv[SUPA_SV_S_D_WIDTH] = etot > 0.0 ? dev_of(sd, ld2 * it) : nan;
        }
        // a shower in error: its earlier runs leave the ring first, then NaN
        if (__ballot(closing && bad)) {
            while (t - h > 0) ring_drain(q, h, t, WAVE, A.lv, L);
            if (closing && bad) {
                float *base = A.lv + (size_t)s * L * LV;
                for (int f = 0; f < L * LV; ++f) base[f] = nan;
                for (int f = 0; f < SV; ++f) A.sv[(size_t)s * SV + f] = nan;
                atomicAdd(A.work, 1);
            }
        }
        if (t - h >= WAVE) ring_drain(q, h, t, WAVE, A.lv, L);
        // --- next shower from the queue
        if (active && pos >= end) {
            const uint32_t next = atomicAdd(queue, 1u);
            if ((int64_t)next >= A.n) {
                active = false;
            } else {
                s = A.order[next];
                pos = A.off[s];
                end = pos + A.cnt[(size_t)s * A.cstride];
                // a segment reaching outside the arrays is the caller's error;
                // never read outside them
                pos = pos < 0 ? 0 : (pos > A.len ? A.len : pos);
                end = end < pos ? pos : (end > A.len ? A.len : end);
                cur = -1;
                depth = -1;
                bad = false;
                seen = 0;
                etot = ld = ld2 = 0.0;
                run_clear(acc);
                for (int l = 0; l < L; ++l) ef[l * WAVE + lane] = 0.0f;
            }
        }
        if (!__ballot(active)) break;

        // --- one aligned block of BLK hits per lane, clipped to [pos, end)
        const bool work = active && pos < end;
        const int64_t b0 = pos & ~(int64_t)(BLK - 1);
        float vx[BLK], vy[BLK], ve[BLK];
        int vl[BLK];
        // whole aligned blocks are read with 16-byte loads whenever they lie
        // inside the arrays (entries outside [pos, end) are then dropped);
        // only the arrays' last partial block is read entry by entry
        if (work && b0 + BLK <= A.len) {
#pragma unroll
            for (int k = 0; k < BLK; k += 4) {
                const f32x4 a = *(const f32x4 *)(A.x + b0 + k);
                const f32x4 b = *(const f32x4 *)(A.y + b0 + k);
                const f32x4 c = *(const f32x4 *)(A.e + b0 + k);
                const i32x4 d = *(const i32x4 *)(A.layer + b0 + k);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int64_t i = b0 + k + j;
                    vx[k + j] = a[j];
                    vy[k + j] = b[j];
                    ve[k + j] = c[j];
                    vl[k + j] = (i >= pos && i < end) ? d[j] : -1;
                }
            }
        } else {
#pragma unroll
            for (int j = 0; j < BLK; ++j) {
                const int64_t i = b0 + j;
                const bool in = work && i >= pos && i < end;
                vx[j] = in ? A.x[i] : 0.0f;
                vy[j] = in ? A.y[i] : 0.0f;
                ve[j] = in ? A.e[i] : 0.0f;
                vl[j] = in ? A.layer[i] : -1;
            }
        }
        // bit j: a new run starts at hit j of this lane's block; their OR
        // over the wave decides (uniformly) which steps need the switch code
        uint32_t msk = 0;
        {
            int p = cur;
#pragma unroll
            for (int j = 0; j < BLK; ++j) {
                const int l = vl[j];
                msk |= (uint32_t)(l >= 0 && l != p) << j;
                p = l >= 0 ? l : p;
            }
            if (bad) msk = 0;
        }
        uint32_t any = msk;
#pragma unroll
        for (int d = 1; d < WAVE; d <<= 1) any |= (uint32_t)__shfl_xor((int)any, d);
        any = __builtin_amdgcn_readfirstlane(any);
#pragma unroll
        for (int j = 0; j < BLK; ++j) {
            const int l = vl[j];
            if ((any >> j) & 1) {
                const bool sw = ((msk >> j) & 1) && !bad;  // a new run starts here
                ring_put(q, t, sw && cur >= 0, (int)s, cur, acc);
                if (sw) {
                    if (cur >= 0) {
                        ef[cur * WAVE + lane] = (float)acc.se;
                        etot += acc.se;
                        ld += (double)cur * acc.se;
                        ld2 += (double)cur * (double)cur * acc.se;
                        if (acc.se > 0.0 && cur > depth) depth = cur;
                    }
                    run_clear(acc);
                    if (l >= L || ((seen >> l) & 1)) {
                        bad = true;
                        cur = -1;
                    } else {
                        seen |= 1ull << l;
                        cur = l;
                    }
                }
                if (t - h >= WAVE) ring_drain(q, h, t, WAVE, A.lv, L);
            }
            run_add(acc, vx[j], vy[j], ve[j], l >= 0 && !bad);
        }
        if (work) pos = bad ? end : (b0 + BLK < end ? b0 + BLK : end);
    }
    while (t - h > 0) ring_drain(q, h, t, WAVE, A.lv, L);
}

__global__ void radius_kernel(int64_t n, const float *x, const float *y, float *r) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double a = x[i], b = y[i];
        r[i] = (float)__builtin_sqrt(a * a + b * b);
    }
}

// ---------------------------------------------------------------------------
// W1 between histograms
// ---------------------------------------------------------------------------

constexpr int W1_THREADS = 256;
constexpr int W1_HIST_WORDS = 8192;  // LDS histogram words per block (32 KB)

struct Partial {  // per (row block, column); sums shifted by the column's pivot
    double cnt, s1, s2, mn, mx;
};

struct ColInfo {
    double lo, scale, width, sigma, n_ref, n_smp;
    int32_t skip, pad;
};

__host__ __device__ inline int w1_cols_per_tile(int n_cols, int n_bins) {
    int ct = 1;
    while (ct < 64 && ct < n_cols && (ct * 2) * n_bins <= W1_HIST_WORDS) ct *= 2;
    return ct;
}

__host__ __device__ inline int w1_row_blocks(int64_t rows, int n_cols, int ct) {
    const int64_t tiles = (n_cols + ct - 1) / ct;
    int64_t rb = (rows + 255) / 256;
    const int64_t cap = 2048 / tiles > 1 ? 2048 / tiles : 1;
    if (rb > cap) rb = cap;
    if (rb < 1) rb = 1;
    return (int)rb;
}

__device__ inline bool finite(float v) { return __builtin_isfinite(v); }

// grid (tiles, row blocks); one sample per launch.
__global__ void __launch_bounds__(W1_THREADS)
    w1_stats(const float *m, int64_t rows, int64_t ld, int n_cols, int ct, int rb, Partial *part) {
    __shared__ double sh[5][W1_THREADS];
    const int t = threadIdx.x;
    const int cl = t % ct, ph = t / ct, rpt = W1_THREADS / ct;
    const int c = blockIdx.x * ct + cl;
    const int64_t per = (rows + rb - 1) / rb;
    const int64_t r0 = (int64_t)blockIdx.y * per;
    const int64_t r1 = r0 + per < rows ? r0 + per : rows;
    double cnt = 0.0, s1 = 0.0, s2 = 0.0;
    float mn = __builtin_inff(), mx = -__builtin_inff();
    if (c < n_cols) {
        const float p0 = m[c];
        const double piv = finite(p0) ? (double)p0 : 0.0;
        // four rows per round, all requested before any is used
        for (int64_t r = r0 + ph; r < r1; r += 4 * (int64_t)rpt) {
            float v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t q = r + (int64_t)u * rpt;
                v[u] = q < r1 ? m[q * ld + c] : __builtin_nanf("");
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (!finite(v[u])) continue;
                const double d = (double)v[u] - piv;
                cnt += 1.0;
                s1 += d;
                s2 = __builtin_fma(d, d, s2);
                mn = v[u] < mn ? v[u] : mn;
                mx = v[u] > mx ? v[u] : mx;
            }
        }
    }
    sh[0][t] = cnt;
    sh[1][t] = s1;
    sh[2][t] = s2;
    sh[3][t] = mn;
    sh[4][t] = mx;
    __syncthreads();
    if (ph == 0 && c < n_cols) {
        for (int k = 1; k < rpt; ++k) {
            const int u = k * ct + cl;
            cnt += sh[0][u];
            s1 += sh[1][u];
            s2 += sh[2][u];
            mn = (float)sh[3][u] < mn ? (float)sh[3][u] : mn;
            mx = (float)sh[4][u] > mx ? (float)sh[4][u] : mx;
        }
        part[(size_t)blockIdx.y * n_cols + c] = Partial{cnt, s1, s2, (double)mn, (double)mx};
    }
}

// One wave per column: lane k adds the partials of row blocks k, k + 64, ...
// in order, then the lanes' sums are combined by a fixed butterfly (the same
// order on every run).
__global__ void __launch_bounds__(WAVE) w1_colinfo(int n_cols, int n_bins, const Partial *pr, int rbr,
                                                   const Partial *ps, int rbs, ColInfo *info) {
    const int c = blockIdx.x;
    const int lane = threadIdx.x;
    if (c >= n_cols) return;
    double nr = 0.0, s1 = 0.0, s2 = 0.0, mnr = __builtin_inf(), mxr = -__builtin_inf();
    for (int b = lane; b < rbr; b += WAVE) {
        const Partial p = pr[(size_t)b * n_cols + c];
        nr += p.cnt;
        s1 += p.s1;
        s2 += p.s2;
        mnr = p.mn < mnr ? p.mn : mnr;
        mxr = p.mx > mxr ? p.mx : mxr;
    }
    double ns = 0.0, mns = __builtin_inf(), mxs = -__builtin_inf();
    for (int b = lane; b < rbs; b += WAVE) {
        const Partial p = ps[(size_t)b * n_cols + c];
        ns += p.cnt;
        mns = p.mn < mns ? p.mn : mns;
        mxs = p.mx > mxs ? p.mx : mxs;
    }
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        nr += __shfl_xor(nr, d);
        s1 += __shfl_xor(s1, d);
        s2 += __shfl_xor(s2, d);
        ns += __shfl_xor(ns, d);
        const double a = __shfl_xor(mnr, d), b = __shfl_xor(mxr, d);
        const double e = __shfl_xor(mns, d), f = __shfl_xor(mxs, d);
        mnr = a < mnr ? a : mnr;
        mxr = b > mxr ? b : mxr;
        mns = e < mns ? e : mns;
        mxs = f > mxs ? f : mxs;
    }
    if (lane != 0) return;
    ColInfo ci;
    ci.skip = (nr < 2.0 || ns < 1.0 || mnr == mxr) ? 1 : 0;
    ci.pad = 0;
    ci.n_ref = nr;
    ci.n_smp = ns;
    const double m1 = nr > 0.0 ? s1 / nr : 0.0;
    const double var = nr > 0.0 ? s2 / nr - m1 * m1 : 0.0;
    ci.sigma = __builtin_sqrt(var > 0.0 ? var : 0.0);
    ci.lo = mnr < mns ? mnr : mns;
    const double hi = mxr > mxs ? mxr : mxs;
    ci.width = ci.skip ? 0.0 : hi - ci.lo;
    ci.scale = ci.width > 0.0 ? (double)n_bins / ci.width : 0.0;
    info[c] = ci;
}

__global__ void w1_zero(uint32_t *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// grid (tiles, row blocks); hist: [n_cols][n_bins] of this sample.
__global__ void __launch_bounds__(W1_THREADS)
    w1_hist(const float *m, int64_t rows, int64_t ld, int n_cols, int ct, int rb, int n_bins,
            const ColInfo *info, uint32_t *hist) {
    extern __shared__ uint32_t hb[];  // [ct][n_bins]
    const int t = threadIdx.x;
    for (int i = t; i < ct * n_bins; i += W1_THREADS) hb[i] = 0;
    __syncthreads();
    const int cl = t % ct, ph = t / ct, rpt = W1_THREADS / ct;
    const int c = blockIdx.x * ct + cl;
    const int64_t per = (rows + rb - 1) / rb;
    const int64_t r0 = (int64_t)blockIdx.y * per;
    const int64_t r1 = r0 + per < rows ? r0 + per : rows;
    if (c < n_cols) {
        const ColInfo ci = info[c];
        if (!ci.skip) {
            uint32_t *h = hb + cl * n_bins;
            for (int64_t r = r0 + ph; r < r1; r += 4 * (int64_t)rpt) {
                float v[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int64_t q = r + (int64_t)u * rpt;
                    v[u] = q < r1 ? m[q * ld + c] : __builtin_nanf("");
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (!finite(v[u])) continue;
                    int k = (int)__builtin_floor(((double)v[u] - ci.lo) * ci.scale);
                    k = k < 0 ? 0 : (k >= n_bins ? n_bins - 1 : k);
                    atomicAdd(h + k, 1u);
                }
            }
        }
    }
    __syncthreads();
    for (int i = t; i < ct * n_bins; i += W1_THREADS) {
        const int cc = blockIdx.x * ct + i / n_bins;
        const uint32_t v = hb[i];
        if (cc < n_cols && v) atomicAdd(hist + (size_t)cc * n_bins + i % n_bins, v);
    }
}

// One wave per column: cumulative counts of both histograms, sum of the
// absolute differences of the cumulative fractions.
__global__ void __launch_bounds__(WAVE)
    w1_distance(int n_cols, int n_bins, const ColInfo *info, const uint32_t *hr, const uint32_t *hs,
                double *w1) {
    const int c = blockIdx.x;
    const int lane = threadIdx.x;
    const ColInfo ci = info[c];
    if (ci.skip) {
        if (lane == 0) w1[c] = __builtin_nan("");
        return;
    }
    const uint32_t *a = hr + (size_t)c * n_bins;
    const uint32_t *b = hs + (size_t)c * n_bins;
    uint64_t carry_a = 0, carry_b = 0;
    double acc = 0.0;
    for (int k0 = 0; k0 < n_bins; k0 += WAVE) {
        const int k = k0 + lane;
        uint64_t va = k < n_bins ? a[k] : 0, vb = k < n_bins ? b[k] : 0;
        // inclusive prefix sums across the wave
        for (int d = 1; d < WAVE; d <<= 1) {
            const uint64_t ua = __shfl_up(va, d), ub = __shfl_up(vb, d);
            if (lane >= d) {
                va += ua;
                vb += ub;
            }
        }
        va += carry_a;
        vb += carry_b;
        if (k < n_bins) {
            const double fa = (double)va / ci.n_ref, fb = (double)vb / ci.n_smp;
            acc += __builtin_fabs(fa - fb);
        }
        carry_a = __shfl(va, WAVE - 1);
        carry_b = __shfl(vb, WAVE - 1);
    }
    for (int d = WAVE / 2; d > 0; d >>= 1) acc += __shfl_xor(acc, d);
    if (lane == 0) w1[c] = ci.width / (double)n_bins * acc / ci.sigma;
}

// One wave per group: lanes take columns c = lane, lane + 64, ...; the sums
// are combined by a fixed butterfly.
__global__ void __launch_bounds__(WAVE) w1_groups(int n_cols, const int32_t *group, int n_groups,
                                                  const double *w1, double *out) {
    const int g = blockIdx.x;
    const int lane = threadIdx.x;
    if (g >= n_groups) return;
    double s = 0.0;
    int k = 0;
    for (int c = lane; c < n_cols; c += WAVE) {
        const double v = w1[c];
        const bool in = group[c] == g && v == v;
        s += in ? v : 0.0;
        k += in ? 1 : 0;
    }
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        s += __shfl_xor(s, d);
        k += __shfl_xor(k, d);
    }
    if (lane == 0) out[g] = k ? s / k : __builtin_nan("");
}

inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

struct W1Layout {
    int ct, tiles, rbr, rbs;
    size_t off_pr, off_ps, off_info, off_hr, off_hs, total;
};

W1Layout w1_layout(int n_cols, int n_bins, int64_t n_ref, int64_t n_smp) {
    W1Layout w;
    w.ct = w1_cols_per_tile(n_cols, n_bins);
    w.tiles = (n_cols + w.ct - 1) / w.ct;
    w.rbr = w1_row_blocks(n_ref, n_cols, w.ct);
    w.rbs = w1_row_blocks(n_smp, n_cols, w.ct);
    size_t o = 0;
    w.off_pr = o;
    o += align256((size_t)w.rbr * n_cols * sizeof(Partial));
    w.off_ps = o;
    o += align256((size_t)w.rbs * n_cols * sizeof(Partial));
    w.off_info = o;
    o += align256((size_t)n_cols * sizeof(ColInfo));
    w.off_hr = o;
    o += align256((size_t)n_cols * n_bins * 4);
    w.off_hs = o;
    o += align256((size_t)n_cols * n_bins * 4);
    w.total = o;
    return w;
}

int g_cu_count = 0;

int cu_count() {
    if (g_cu_count == 0) {
        int dev = 0, n = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
            g_cu_count = n;
        else
            g_cu_count = 256;
    }
    return g_cu_count;
}

thread_local std::string t_err;

supa_status bad_arg(const char *msg) {
    t_err = msg;
    return SUPA_ERR_INVALID_ARG;
}

supa_status dev_err(hipError_t e, const char *what) {
    if (e == hipSuccess) return SUPA_OK;
    t_err = std::string(what) + ": " + hipGetErrorString(e);
    return SUPA_ERR_DEVICE;
}

}  // namespace

extern "C" const char *supa_shapes_last_error(void) { return t_err.c_str(); }

extern "C" int64_t supa_shapes_work_ints(int64_t n) { return n < 0 ? -1 : WORK_HEAD + n; }

extern "C" supa_status supa_shower_shapes(void *stream, int64_t n, int32_t n_layers,
                                          const int64_t *hit_offsets, const int32_t *hit_counts,
                                          int32_t counts_stride, int64_t hit_len, const float *hit_x,
                                          const float *hit_y, const float *hit_e,
                                          const int32_t *hit_layer, float *layer_vars,
                                          float *shower_vars, int32_t *work, int64_t work_ints) {
    if (n < 0 || n > INT32_MAX) return bad_arg("n out of range");
    if (n_layers < 1 || n_layers > 64) return bad_arg("n_layers must be 1..64");
    if (counts_stride < 1) return bad_arg("counts_stride must be >= 1");
    if (hit_len < 0) return bad_arg("hit_len < 0");
    if (!work) return bad_arg("work is NULL");
    if (work_ints < supa_shapes_work_ints(n)) return bad_arg("work holds fewer than supa_shapes_work_ints(n) int32");
    if (n > 0 && (!hit_offsets || !hit_counts || !hit_x || !hit_y || !hit_e || !hit_layer ||
                  !layer_vars || !shower_vars))
        return bad_arg("NULL array");
    // blocks of four hits are read with 16-byte loads
    if (n > 0 && (((uintptr_t)hit_x | (uintptr_t)hit_y | (uintptr_t)hit_e | (uintptr_t)hit_layer) & 15))
        return bad_arg("hit arrays must be 16-byte aligned");
    if (n > 0 && ((uintptr_t)layer_vars & 7)) return bad_arg("layer_vars must be 8-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(shapes_clear, dim3(1), dim3(1024), 0, s, work);
    if (n == 0) return dev_err(hipGetLastError(), "shapes_clear");
    const int64_t waves = (n + WAVE - 1) / WAVE;
    const int64_t cap = (int64_t)cu_count() * 16;
    const int grid = (int)(waves < cap ? waves : cap);
    int32_t *order = work + WORK_HEAD;
    if (waves <= cap) {  // every shower in flight at once (one per lane): one order
        uint32_t *gsize = (uint32_t *)work + 4, *gcur = gsize + ORDER_BUCKETS;
        const int blocks = (int)((n + ORDER_CHUNK - 1) / ORDER_CHUNK);
        hipLaunchKernelGGL(shapes_order_sizes, dim3(blocks), dim3(ORDER_THREADS), 0, s, n, hit_counts,
                           counts_stride, gsize);
        hipLaunchKernelGGL(shapes_order_place, dim3(blocks), dim3(ORDER_THREADS), 0, s, n, hit_counts,
                           counts_stride, gsize, gcur, order);
    } else {
        hipLaunchKernelGGL(shapes_order, dim3((int)((n + ORDER_WIN - 1) / ORDER_WIN)), dim3(ORDER_THREADS), 0,
                           s, n, (int64_t)ORDER_WIN, hit_counts, counts_stride, order);
    }
    ShapeArgs A{n, n_layers, hit_offsets, hit_counts, counts_stride, hit_len, hit_x, hit_y, hit_e,
                hit_layer, layer_vars, shower_vars, work, order};
    hipLaunchKernelGGL(shapes_kernel, dim3(grid), dim3(WAVE), (size_t)n_layers * WAVE * sizeof(float),
                       s, A);
    return dev_err(hipGetLastError(), "shapes_kernel");
}

extern "C" supa_status supa_hit_radius(void *stream, int64_t n, const float *x, const float *y,
                                       float *r) {
    if (n < 0) return bad_arg("n < 0");
    if (n == 0) return SUPA_OK;
    if (!x || !y || !r) return bad_arg("NULL array");
    int64_t blocks = (n + 255) / 256;
    const int64_t cap = (int64_t)cu_count() * 8;
    if (blocks > cap) blocks = cap;
    hipLaunchKernelGGL(radius_kernel, dim3((int)blocks), dim3(256), 0, (hipStream_t)stream, n, x, y, r);
    return dev_err(hipGetLastError(), "radius_kernel");
}

extern "C" size_t supa_w1_workspace_bytes(int32_t n_cols, int32_t n_bins, int64_t n_ref,
                                          int64_t n_smp) {
    if (n_cols < 1 || n_bins < 1 || n_ref < 1 || n_smp < 1) return 0;
    return w1_layout(n_cols, n_bins, n_ref, n_smp).total;
}

extern "C" supa_status supa_w1_normalized(void *stream, int32_t n_cols, const float *ref,
                                          int64_t n_ref, int64_t ref_ld, const float *smp,
                                          int64_t n_smp, int64_t smp_ld, int32_t n_bins,
                                          const int32_t *group_of_col, int32_t n_groups,
                                          double *w1, double *group_mean, void *workspace,
                                          size_t workspace_bytes) {
    if (n_cols < 1 || n_cols > 65535) return bad_arg("n_cols must be 1..65535");
    if (n_bins < 1 || n_bins > 4096) return bad_arg("n_bins must be 1..4096");
    if (n_ref < 1 || n_ref > INT32_MAX || n_smp < 1 || n_smp > INT32_MAX)
        return bad_arg("row counts must be 1..2^31-1");
    if (ref_ld < n_cols || smp_ld < n_cols) return bad_arg("leading dimension < n_cols");
    if (!ref || !smp || !w1 || !workspace) return bad_arg("NULL pointer");
    if (group_of_col && (n_groups < 1 || !group_mean)) return bad_arg("groups need n_groups >= 1 and group_mean");
    const W1Layout w = w1_layout(n_cols, n_bins, n_ref, n_smp);
    if (workspace_bytes < w.total) return bad_arg("workspace too small");
    hipStream_t s = (hipStream_t)stream;
    char *ws = (char *)workspace;
    Partial *pr = (Partial *)(ws + w.off_pr), *ps = (Partial *)(ws + w.off_ps);
    ColInfo *info = (ColInfo *)(ws + w.off_info);
    uint32_t *hr = (uint32_t *)(ws + w.off_hr), *hs = (uint32_t *)(ws + w.off_hs);

    const int64_t zero_words = (int64_t)(w.total - w.off_hr) / 4;
    hipLaunchKernelGGL(w1_zero, dim3(cu_count() * 4), dim3(256), 0, s, hr, zero_words);
    hipLaunchKernelGGL(w1_stats, dim3(w.tiles, w.rbr), dim3(W1_THREADS), 0, s, ref, n_ref, ref_ld,
                       n_cols, w.ct, w.rbr, pr);
    hipLaunchKernelGGL(w1_stats, dim3(w.tiles, w.rbs), dim3(W1_THREADS), 0, s, smp, n_smp, smp_ld,
                       n_cols, w.ct, w.rbs, ps);
    hipLaunchKernelGGL(w1_colinfo, dim3(n_cols), dim3(WAVE), 0, s, n_cols, n_bins, pr,
                       w.rbr, ps, w.rbs, info);
    const size_t lds = (size_t)w.ct * n_bins * 4;
    hipLaunchKernelGGL(w1_hist, dim3(w.tiles, w.rbr), dim3(W1_THREADS), lds, s, ref, n_ref, ref_ld,
                       n_cols, w.ct, w.rbr, n_bins, info, hr);
    hipLaunchKernelGGL(w1_hist, dim3(w.tiles, w.rbs), dim3(W1_THREADS), lds, s, smp, n_smp, smp_ld,
                       n_cols, w.ct, w.rbs, n_bins, info, hs);
    hipLaunchKernelGGL(w1_distance, dim3(n_cols), dim3(WAVE), 0, s, n_cols, n_bins, info, hr, hs, w1);
    if (group_of_col)
        hipLaunchKernelGGL(w1_groups, dim3(n_groups), dim3(WAVE), 0, s, n_cols, group_of_col,
                           n_groups, w1, group_mean);
    return dev_err(hipGetLastError(), "w1 kernels");
}
