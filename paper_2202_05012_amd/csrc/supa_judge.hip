// supa_judge.hip -- the surrogate's judge on the GPU: exact 1-D Wasserstein
// distances between two samples of equal size, column by column (the
// distance of the paper's section "Performance Analysis of Generative
// Models", here between the simulator's per-layer quantities and those of
// surrogate + fallback), and the occupied-cell counts of per-layer images.
//
// For two samples a, b of n values each, W1(a, b) = (1/n) sum_i |a_(i) - b_(i)|
// with a_(i), b_(i) the order statistics.  Each column of both samples is
// sorted by a stable least-significant-digit radix sort of its float keys
// (four passes of 8 bits; per pass: digit counts per tile of 4096 keys, one
// scan of the counts per column, then every key to its place, ranked within
// its tile in input order with wave ballots), then one kernel sums
// |a_(i) - b_(i)| per column in double, by fixed blocks summed in order, so
// the result does not depend on scheduling.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "supa_device.hpp"

namespace supa {

constexpr int RS_THREADS = 256;
constexpr int RS_ITEMS = 16;
constexpr int RS_TILE = RS_THREADS * RS_ITEMS;   // keys per tile
constexpr int RS_DIGITS = 256;
constexpr int RS_WAVES = RS_THREADS / 64;

// float -> unsigned key with the same order (negative values reversed)
__device__ __forceinline__ uint32_t float_key(float f) {
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ float key_float(uint32_t k) {
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

// Key j of column c in pass `pass`: from the caller's row-major matrix in
// the first pass, from the column-major buffer afterwards.
struct SortSrc {
    const float *x;        // first pass: x[j * ld + c]
    int64_t ld;
    const uint32_t *keys;  // later passes: keys[c * n + j]
};

__device__ __forceinline__ uint32_t load_key(const SortSrc &S, int c, int64_t n, int64_t j) {
    return S.keys ? S.keys[(int64_t)c * n + j] : float_key(S.x[j * S.ld + c]);
}

// counts of the digit of each tile: hist[(c * 256 + d) * nt + t]
__global__ void __launch_bounds__(RS_THREADS) rs_hist(SortSrc S, int64_t n, int shift, uint32_t *hist) {
    __shared__ uint32_t h[RS_DIGITS];
    const int t = blockIdx.x, c = blockIdx.y, nt = gridDim.x;
    h[threadIdx.x] = 0u;
    __syncthreads();
    for (int q = 0; q < RS_ITEMS; ++q) {
        const int64_t j = (int64_t)t * RS_TILE + q * RS_THREADS + threadIdx.x;
        if (j < n) atomicAdd(&h[(load_key(S, c, n, j) >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[((int64_t)c * RS_DIGITS + threadIdx.x) * nt + t] = h[threadIdx.x];
}

// one block per column: the counts, digit-major then tile, to exclusive
// starts within the column (in place)
__global__ void __launch_bounds__(1024) rs_scan(uint32_t *hist, int nt) {
    __shared__ uint32_t part[1024 / 64];
    uint32_t *h = hist + (int64_t)blockIdx.y * RS_DIGITS * nt;
    const int m = RS_DIGITS * nt;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t carry = 0;
    for (int b0 = 0; b0 < m; b0 += 1024) {
        const int i = b0 + (int)threadIdx.x;
        const uint32_t v = i < m ? h[i] : 0u;
        uint32_t incl = v;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(incl, off, 64);
            if (lane >= off) incl += y;
        }
        if (lane == 63) part[w] = incl;
        __syncthreads();
        uint32_t before = 0, all = 0;
        for (int q = 0; q < 1024 / 64; ++q) {
            before += q < w ? part[q] : 0u;
            all += part[q];
        }
        if (i < m) h[i] = carry + before + incl - v;
        carry += all;
        __syncthreads();
    }
}

// every key of a tile to its place: column start of its digit in this tile
// + its rank among the tile's keys of that digit, in input order
__global__ void __launch_bounds__(RS_THREADS) rs_scatter(SortSrc S, int64_t n, int shift, const uint32_t *hist,
                                                         uint32_t *out) {
    __shared__ uint32_t base[RS_DIGITS];            // next place of each digit in this tile
    __shared__ uint32_t wcnt[RS_WAVES][RS_DIGITS];  // keys per digit of each wave in a round
    const int t = blockIdx.x, c = blockIdx.y, nt = gridDim.x;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    base[threadIdx.x] = hist[((int64_t)c * RS_DIGITS + threadIdx.x) * nt + t];
    for (int q = 0; q < RS_WAVES; ++q) wcnt[q][threadIdx.x] = 0u;
    __syncthreads();
    const uint64_t below = (1ull << lane) - 1ull;
    for (int q = 0; q < RS_ITEMS; ++q) {
        // a round: 256 consecutive keys, one per thread, in thread order
        const int64_t j = (int64_t)t * RS_TILE + q * RS_THREADS + threadIdx.x;
        const bool valid = j < n;
        const uint32_t k = valid ? load_key(S, c, n, j) : 0u;
        const uint32_t d = (k >> shift) & 255u;
        // the lanes of this wave holding the same digit
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & below);
        if (valid && rank == 0u) wcnt[w][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        // per digit: where each wave's keys start, and the tile's next place
        {
            const int dd = threadIdx.x;
            uint32_t run = base[dd];
            for (int q2 = 0; q2 < RS_WAVES; ++q2) {
                const uint32_t cnt = wcnt[q2][dd];
                wcnt[q2][dd] = run;
                run += cnt;
            }
            base[dd] = run;
        }
        __syncthreads();
        if (valid) out[(int64_t)c * n + wcnt[w][d] + rank] = k;
        __syncthreads();
        for (int q2 = 0; q2 < RS_WAVES; ++q2) wcnt[q2][threadIdx.x] = 0u;
        __syncthreads();
    }
}

// per column: partial sums of |a_(i) - b_(i)| over fixed blocks of rows
constexpr int W1S_THREADS = 256;
constexpr int W1S_ROWS = W1S_THREADS * 16;

__global__ void __launch_bounds__(W1S_THREADS) w1_sorted_partials(const uint32_t *ka, const uint32_t *kb, int64_t n,
                                                                   double *part) {
    __shared__ double sh[W1S_THREADS / 64];
    const int blk = blockIdx.x, c = blockIdx.y, nb = gridDim.x;
    double s = 0.0;
    for (int q = 0; q < 16; ++q) {
        const int64_t i = (int64_t)blk * W1S_ROWS + q * W1S_THREADS + threadIdx.x;
        if (i < n) {
            const float a = key_float(ka[(int64_t)c * n + i]), b = key_float(kb[(int64_t)c * n + i]);
            s += fabs((double)a - (double)b);
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int q = 0; q < W1S_THREADS / 64; ++q) t += sh[q];
        part[(int64_t)c * nb + blk] = t;
    }
}

// one wave per column: the block partials in order, divided by n
__global__ void w1_sorted_final(const double *part, int nb, int64_t n, int cols, double *w1) {
    const int c = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (c >= cols) return;
    double s = 0.0;
    for (int b = lane; b < nb; b += 64) s += part[(int64_t)c * nb + b];
    // fixed butterfly: the same result on every run
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) w1[c] = s / (double)n;
}

// sorted values back to floats, column-major [cols][n]
__global__ void keys_to_floats(const uint32_t *k, int64_t total, float *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < total) out[i] = key_float(k[i]);
}

// cnt[r][l] = number of q < g with img[r][l * g + q] > thr
__global__ void occupied_counts(int64_t rows, int L, int g, const float *img, float thr, float *cnt) {
    const int64_t rl = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (rl >= rows * L) return;
    const float *p = img + rl * g;
    int m = 0;
    for (int q = lane; q < g; q += 64) m += p[q] > thr ? 1 : 0;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m += __shfl_xor(m, off, 64);
    if (lane == 0) cnt[rl] = (float)m;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static int64_t rs_tiles(int64_t n) { return (n + RS_TILE - 1) / RS_TILE; }

// bytes of workspace for sorting `cols` columns of n keys (two key buffers
// and the digit counts)
size_t sort_work_bytes(int64_t n, int cols) {
    const size_t keys = (size_t)cols * n * 4;
    const size_t hist = (size_t)cols * RS_DIGITS * rs_tiles(n) * 4;
    return 2 * ((keys + 255) & ~(size_t)255) + ((hist + 255) & ~(size_t)255);
}

// sorts the columns of x (row-major, ld) into keys (column-major [cols][n]);
// work: sort_work_bytes(n, cols); returns the buffer holding the result
hipError_t launch_sort_columns(const float *x, int64_t ld, int64_t n, int cols, void *work, uint32_t **sorted,
                               hipStream_t s) {
    const size_t keys_b = (((size_t)cols * n * 4) + 255) & ~(size_t)255;
    uint32_t *k0 = (uint32_t *)work, *k1 = (uint32_t *)((char *)work + keys_b);
    uint32_t *hist = (uint32_t *)((char *)work + 2 * keys_b);
    const int nt = (int)rs_tiles(n);
    const dim3 grid(nt, cols);
    SortSrc src{x, ld, nullptr};
    uint32_t *dst = k0;
    for (int pass = 0; pass < 4; ++pass) {
        const int shift = 8 * pass;
        hipLaunchKernelGGL(rs_hist, grid, dim3(RS_THREADS), 0, s, src, n, shift, hist);
        hipLaunchKernelGGL(rs_scan, dim3(1, cols), dim3(1024), 0, s, hist, nt);
        hipLaunchKernelGGL(rs_scatter, grid, dim3(RS_THREADS), 0, s, src, n, shift, hist, dst);
        src = SortSrc{nullptr, 0, dst};
        dst = dst == k0 ? k1 : k0;
    }
    *sorted = (uint32_t *)src.keys;
    return hipGetLastError();
}

hipError_t launch_w1_sorted(const uint32_t *ka, const uint32_t *kb, int64_t n, int cols, double *part, double *w1,
                            hipStream_t s) {
    const int nb = (int)((n + W1S_ROWS - 1) / W1S_ROWS);
    hipLaunchKernelGGL(w1_sorted_partials, dim3(nb, cols), dim3(W1S_THREADS), 0, s, ka, kb, n, part);
    hipLaunchKernelGGL(w1_sorted_final, dim3((cols + 3) / 4), dim3(256), 0, s, part, nb, n, cols, w1);
    return hipGetLastError();
}

int64_t w1_sorted_partial_words(int64_t n, int cols) { return (int64_t)cols * ((n + W1S_ROWS - 1) / W1S_ROWS); }

hipError_t launch_keys_to_floats(const uint32_t *k, int64_t total, float *out, hipStream_t s) {
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(keys_to_floats, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, k, total, out);
    return hipGetLastError();
}

hipError_t launch_occupied_counts(int64_t rows, int L, int g, const float *img, float thr, float *cnt,
                                  hipStream_t s) {
    const int64_t groups = rows * L;
    if (groups <= 0) return hipSuccess;
    hipLaunchKernelGGL(occupied_counts, dim3((unsigned)((groups + 3) / 4)), dim3(256), 0, s, rows, L, g, img, thr,
                       cnt);
    return hipGetLastError();
}

}  // namespace supa
