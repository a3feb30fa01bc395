// supa_order.hip -- the order in which the propagation kernel takes showers.
//
// A shower's expected cost grows linearly with its energy (about 4 E0 / e_cut
// particle-steps when nothing escapes: each split halves the energy on
// average and the cascade stops at the threshold).  Handing out the most
// expensive showers first leaves the cheap ones to fill the end of the
// launch, so no wave starts a long shower when the others are done (longest
// processing time first).  The order is a counting sort of the showers by
// a bucket of log2 of their fixed-point energy, descending: three kernels
// (histogram, scan of the buckets, scatter).  The order within a bucket is
// arbitrary; results do not depend on the order at all.
#include <algorithm>

#include "supa_device.hpp"

namespace supa {

constexpr int ORDER_BUCKETS = 1024;           // 32 per octave of E_int
constexpr int ORDER_THREADS = 256;

// bucket 0 = most expensive
__device__ __forceinline__ int cost_bucket(float e0, float e_scale) {
    const float v = e0 * e_scale;
    if (!(v >= 1.0f)) return ORDER_BUCKETS - 1;           // tiny, zero, negative or NaN
    const float l = __log2f(v) * 32.0f;                    // < 32 * 32 for v < 2^32
    const int b = (int)l;
    return ORDER_BUCKETS - 1 - min(max(b, 0), ORDER_BUCKETS - 1);
}

__global__ void __launch_bounds__(ORDER_THREADS) order_hist(const float *e0, int n, float e_scale,
                                                             uint32_t *hist) {
    __shared__ uint32_t h[ORDER_BUCKETS];
    for (int q = threadIdx.x; q < ORDER_BUCKETS; q += ORDER_THREADS) h[q] = 0u;
    __syncthreads();
    for (int i = blockIdx.x * ORDER_THREADS + threadIdx.x; i < n; i += gridDim.x * ORDER_THREADS)
        atomicAdd(&h[cost_bucket(e0[i], e_scale)], 1u);
    __syncthreads();
    for (int q = threadIdx.x; q < ORDER_BUCKETS; q += ORDER_THREADS)
        if (h[q]) atomicAdd(&hist[q], h[q]);
}

// one block: hist -> exclusive starts, in place
__global__ void __launch_bounds__(ORDER_BUCKETS) order_scan(uint32_t *hist) {
    __shared__ uint32_t s[ORDER_BUCKETS];
    const int t = threadIdx.x;
    s[t] = hist[t];
    __syncthreads();
    for (int off = 1; off < ORDER_BUCKETS; off <<= 1) {
        const uint32_t v = t >= off ? s[t - off] : 0u;
        __syncthreads();
        s[t] += v;
        __syncthreads();
    }
    hist[t] = s[t] - hist[t];
}

// Each block takes a contiguous run of ORDER_RUN showers: counts per bucket
// in LDS, one global reservation per bucket it holds (instead of one atomic
// per shower on a few hot counters), then LDS ranks within its reservation.
constexpr int ORDER_RUN = ORDER_THREADS * 16;

__global__ void __launch_bounds__(ORDER_THREADS) order_scatter(const float *e0, int n, float e_scale,
                                                                uint32_t *cursor, int32_t *order) {
    __shared__ uint32_t cnt[ORDER_BUCKETS], base[ORDER_BUCKETS];
    const int i0 = blockIdx.x * ORDER_RUN, i1 = min(n, i0 + ORDER_RUN);
    for (int q = threadIdx.x; q < ORDER_BUCKETS; q += ORDER_THREADS) cnt[q] = 0u;
    __syncthreads();
    for (int i = i0 + threadIdx.x; i < i1; i += ORDER_THREADS) atomicAdd(&cnt[cost_bucket(e0[i], e_scale)], 1u);
    __syncthreads();
    for (int q = threadIdx.x; q < ORDER_BUCKETS; q += ORDER_THREADS) {
        base[q] = cnt[q] ? atomicAdd(&cursor[q], cnt[q]) : 0u;
        cnt[q] = 0u;
    }
    __syncthreads();
    for (int i = i0 + threadIdx.x; i < i1; i += ORDER_THREADS) {
        const int b = cost_bucket(e0[i], e_scale);
        const uint32_t pos = base[b] + atomicAdd(&cnt[b], 1u);
        if (pos < (uint32_t)n) order[pos] = i;
    }
}

__global__ void order_clear(uint32_t *hist) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < ORDER_BUCKETS) hist[q] = 0u;
}

int64_t order_scratch_words() { return ORDER_BUCKETS; }

// order[0..n) = a permutation of 0..n-1, most expensive first; hist: ORDER_BUCKETS words
hipError_t launch_cost_order(const float *e0, int n, float e_scale, uint32_t *hist, int32_t *order,
                             int n_cu, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int blocks = std::max(1, std::min((n + ORDER_THREADS - 1) / ORDER_THREADS, n_cu * 4));
    hipLaunchKernelGGL(order_clear, dim3(ORDER_BUCKETS / 256), dim3(256), 0, s, hist);
    hipLaunchKernelGGL(order_hist, dim3(blocks), dim3(ORDER_THREADS), 0, s, e0, n, e_scale, hist);
    hipLaunchKernelGGL(order_scan, dim3(1), dim3(ORDER_BUCKETS), 0, s, hist);
    hipLaunchKernelGGL(order_scatter, dim3((n + ORDER_RUN - 1) / ORDER_RUN), dim3(ORDER_THREADS), 0, s, e0, n,
                       e_scale, hist, order);
    return hipGetLastError();
}

}  // namespace supa
