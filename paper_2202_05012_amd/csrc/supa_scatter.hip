// supa_scatter.hip -- segment offsets, and tree nodes to their places.
//
//   scan     hit and node segment offsets = exclusive prefix sums of the
//            showers' counts in batch order (three small kernels: tile sums,
//            one-block scan of the tile sums, per-tile scan), so the output
//            layout is the same on every run;
//   scatter  every node record of the log (chunks filled in whatever order
//            the waves produced them) goes to its shower's segment start +
//            its index within the shower.  Pure data movement.
// Nothing is written when the propagation reported an overflow (the batch is
// rerun) or when the totals exceed the destination capacity.
#include <algorithm>

#include "supa_device.hpp"

namespace supa {

__device__ __forceinline__ long long block_sum_ll(long long v, long long *sh) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int w = (int)threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    long long t = 0;
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) t += sh[q];
    __syncthreads();
    return t;
}

// Exclusive scan across the block of one value per thread (blockDim.x a
// multiple of 64, at most 1024); also returns the block total.
__device__ __forceinline__ long long block_excl_scan_ll(long long v, long long *sh, long long *total) {
    const int lane = (int)(threadIdx.x & 63), w = (int)threadIdx.x >> 6;
    long long incl = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const long long t = __shfl_up(incl, off, 64);
        if (lane >= off) incl += t;
    }
    if (lane == 63) sh[w] = incl;
    __syncthreads();
    long long before = 0, all = 0;
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) {
        if (q < w) before += sh[q];
        all += sh[q];
    }
    __syncthreads();
    *total = all;
    return before + incl - v;
}

// tile sums of the hit and node counts
__global__ void __launch_bounds__(SCAN_THREADS) scan_tiles(ScanParams S) {
    __shared__ long long sh[SCAN_THREADS / 64];
    const int64_t t0 = (int64_t)blockIdx.x * SCAN_TILE;
    long long h = 0, nn = 0;
    for (int q = 0; q < SCAN_ITEMS; ++q) {
        const int64_t i = t0 + q * SCAN_THREADS + threadIdx.x;
        if (i < S.n) {
            nn += S.counts[6 * i];
            h += S.counts[6 * i + 1];
        }
    }
    h = block_sum_ll(h, sh);
    nn = block_sum_ll(nn, sh);
    const int nt = (int)((S.n + SCAN_TILE - 1) / SCAN_TILE);
    if (threadIdx.x == 0) {
        S.partial[blockIdx.x] = h;
        S.partial[nt + blockIdx.x] = nn;
    }
}

// one block: tile sums -> tile offsets (in place), totals into the counters
__global__ void __launch_bounds__(1024) scan_top(ScanParams S) {
    __shared__ long long sh[16];
    const int nt = (int)((S.n + SCAN_TILE - 1) / SCAN_TILE);
    for (int a = 0; a < 2; ++a) {
        // sub-batches after the first continue the previous running total
        long long carry = S.prev ? (long long)S.prev[a == 0 ? SUB_HITS : SUB_NODES] : 0;
        for (int b0 = 0; b0 < nt; b0 += 1024) {
            const int b = b0 + (int)threadIdx.x;
            const long long v = b < nt ? S.partial[a * nt + b] : 0;
            long long tot = 0;
            const long long ex = block_excl_scan_ll(v, sh, &tot);
            if (b < nt) S.partial[a * nt + b] = carry + ex;
            carry += tot;
        }
        if (threadIdx.x == 0) S.sub[a == 0 ? SUB_HITS : SUB_NODES] = (unsigned long long)carry;
    }
}

// per tile: offsets of its showers (SCAN_ITEMS consecutive showers per thread)
__global__ void __launch_bounds__(SCAN_THREADS) scan_apply(ScanParams S) {
    __shared__ long long sh[SCAN_THREADS / 64];
    __shared__ int32_t cnt[2][SCAN_TILE];
    const int64_t t0 = (int64_t)blockIdx.x * SCAN_TILE;
    const int nt = (int)((S.n + SCAN_TILE - 1) / SCAN_TILE);
    for (int q = 0; q < SCAN_ITEMS; ++q) {
        const int l = q * SCAN_THREADS + (int)threadIdx.x;
        const int64_t i = t0 + l;
        cnt[0][l] = i < S.n ? S.counts[6 * i + 1] : 0;
        cnt[1][l] = i < S.n ? S.counts[6 * i] : 0;
    }
    __syncthreads();
    const int l0 = (int)threadIdx.x * SCAN_ITEMS;
    for (int a = 0; a < 2; ++a) {
        int64_t *out = a == 0 ? S.hoff : S.noff;
        long long mine = 0;
        for (int q = 0; q < SCAN_ITEMS; ++q) mine += cnt[a][l0 + q];
        long long tot = 0;
        long long o = S.partial[a * nt + blockIdx.x] + block_excl_scan_ll(mine, sh, &tot);
        if (out) {
            for (int q = 0; q < SCAN_ITEMS; ++q) {
                const int64_t i = t0 + l0 + q;
                if (i < S.n) out[i] = o;
                o += cnt[a][l0 + q];
            }
        }
    }
}

constexpr int SCATTER_THREADS = 256;
constexpr int SCATTER_UNROLL = 4;      // records per thread in flight

__global__ void __launch_bounds__(SCATTER_THREADS) scatter_nodes(ScatterParams Q, int32_t n) {
    if (batch_failed(Q.ctr) || (int64_t)Q.sub[SUB_NODES] > Q.ncap) return;
    // the chunks this sub-batch's propagation claimed
    const int c_end = (int)min(Q.sub[SUB_NCHUNK_END], (unsigned long long)Q.n_chunks);
    const int c_begin = Q.prev ? (int)min(Q.prev[SUB_NCHUNK_END], (unsigned long long)c_end) : 0;
    for (int c = c_begin + (int)blockIdx.x; c < c_end; c += gridDim.x) {
        const int fill = min((int)Q.nfill[c], LOG_CHUNK);
        const uint32_t *rec = Q.nlog + (int64_t)c * (NL_FIELDS * LOG_CHUNK);
        // a record: the primary (index 0) or the two daughters of a split;
        // SCATTER_UNROLL records per thread are read before any is written
        // (one round trip for the records, one for their showers' offsets)
        for (int j0 = 0; j0 < fill; j0 += SCATTER_THREADS * SCATTER_UNROLL) {
            uint32_t ri[SCATTER_UNROLL], rx[SCATTER_UNROLL], rp[SCATTER_UNROLL], rg[SCATTER_UNROLL];
            uint32_t xx[SCATTER_UNROLL], yy[SCATTER_UNROLL], e1[SCATTER_UNROLL], e2[SCATTER_UNROLL];
            uint32_t lo[SCATTER_UNROLL], hi[SCATTER_UNROLL];
            int64_t o[SCATTER_UNROLL];
#pragma unroll
            for (int u = 0; u < SCATTER_UNROLL; ++u) {
                const int j = j0 + u * SCATTER_THREADS + (int)threadIdx.x;
                const bool in = j < fill;
                ri[u] = in ? rec[NL_I * LOG_CHUNK + j] : 0xffffffffu;
                rx[u] = in ? rec[NL_IDX * LOG_CHUNK + j] : 0u;
                rp[u] = in ? rec[NL_PARENT * LOG_CHUNK + j] : 0u;
                rg[u] = in ? rec[NL_GK * LOG_CHUNK + j] : 0u;
                xx[u] = in ? rec[NL_X * LOG_CHUNK + j] : 0u;
                yy[u] = in ? rec[NL_Y * LOG_CHUNK + j] : 0u;
                e1[u] = in ? rec[NL_E * LOG_CHUNK + j] : 0u;
                e2[u] = in ? rec[NL_E2 * LOG_CHUNK + j] : 0u;
                lo[u] = (in && Q.nk) ? rec[NL_LO * LOG_CHUNK + j] : 0u;
                hi[u] = (in && Q.nk) ? rec[NL_HI * LOG_CHUNK + j] : 0u;
            }
#pragma unroll
            for (int u = 0; u < SCATTER_UNROLL; ++u)
                o[u] = ri[u] < (uint32_t)n ? Q.noff[ri[u]] + rx[u] : -1;
#pragma unroll
            for (int u = 0; u < SCATTER_UNROLL; ++u) {
                if (o[u] < 0) continue;
                const uint32_t k = rg[u] >> 8;
                const float z = k == 255u ? 0.0f : Q.z_first + (float)k * Q.dz;
                const int nn = rx[u] == 0u ? 1 : 2;
                for (int q = 0; q < nn; ++q) {
                    const int64_t oq = o[u] + q;
                    if (oq >= Q.ncap) continue;
                    Q.np[oq] = (int32_t)rp[u];
                    Q.ng[oq] = (int32_t)(rg[u] & 255u);
                    Q.nvx[oq] = __uint_as_float(xx[u]);
                    Q.nvy[oq] = __uint_as_float(yy[u]);
                    Q.nvz[oq] = z;
                    Q.ne[oq] = (float)(q ? e2[u] : e1[u]) * Q.e_unscale;
                    if (Q.nk) Q.nk[oq] = (((uint64_t)hi[u] << 32) | lo[u]) | (uint64_t)q;
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------
int64_t scan_partial_words(int64_t n) { return 2 * ((n + SCAN_TILE - 1) / SCAN_TILE); }

hipError_t launch_scan(const ScanParams &S, hipStream_t s) {
    if (S.n <= 0) return hipSuccess;
    const int nt = (int)((S.n + SCAN_TILE - 1) / SCAN_TILE);
    hipLaunchKernelGGL(scan_tiles, dim3(nt), dim3(SCAN_THREADS), 0, s, S);
    hipLaunchKernelGGL(scan_top, dim3(1), dim3(1024), 0, s, S);
    hipLaunchKernelGGL(scan_apply, dim3(nt), dim3(SCAN_THREADS), 0, s, S);
    return hipGetLastError();
}

hipError_t launch_scatter_nodes(const ScatterParams &Q, int32_t n, int n_cu, hipStream_t s) {
    if (Q.n_chunks <= 0) return hipSuccess;
    hipLaunchKernelGGL(scatter_nodes, dim3(std::min(n_cu * 8, Q.n_chunks)), dim3(SCATTER_THREADS), 0,
                       s, Q, n);
    return hipGetLastError();
}

}  // namespace supa
