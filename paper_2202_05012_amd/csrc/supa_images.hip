// supa_images.hip -- per-layer images of the hit clouds (paper, appendix
// "Downsampling": a region of interest per layer, a grid of cells, and per
// cell the sum of the energies of the points that fall in it).
//
// Runs after the scatter kernel, which leaves every shower's hits (with
// their integer, fixed-point energies) in one contiguous segment.  One
// 256-thread workgroup takes one shower at a time: it clears an LDS slab that
// holds several whole layers (or a band of rows of one large layer), adds the
// integer energies of the slab's hits with LDS atomics (integer sums, so
// their order does not matter and the result is exact), and streams the slab
// out as float once.  Each output byte is written exactly once and hits are
// read with coalesced, independent loads.
#include "supa_device.hpp"

namespace supa {

constexpr int IMG_THREADS = 256;
constexpr int IMG_UNROLL = 4;          // hits per thread in flight

__device__ __forceinline__ void write_slab(const ImgParams &Q, const uint32_t *slab, float *dst,
                                           int words) {
    if ((words & 3) == 0 && (((uintptr_t)dst) & 15) == 0) {
        for (int q = 4 * (int)threadIdx.x; q < words; q += 4 * IMG_THREADS) {
            const uint4 v = *(const uint4 *)(slab + q);
            *(float4 *)(dst + q) = make_float4((float)v.x * Q.e_unscale, (float)v.y * Q.e_unscale,
                                               (float)v.z * Q.e_unscale, (float)v.w * Q.e_unscale);
        }
    } else {
        for (int q = (int)threadIdx.x; q < words; q += IMG_THREADS)
            dst[q] = (float)slab[q] * Q.e_unscale;
    }
}

__device__ __forceinline__ void clear_slab(uint32_t *slab, int words) {
    int q = 4 * (int)threadIdx.x;
    for (; q + 3 < words; q += 4 * IMG_THREADS) *(uint4 *)(slab + q) = make_uint4(0u, 0u, 0u, 0u);
    for (int r = (words & ~3) + (int)threadIdx.x; r < words; r += IMG_THREADS) slab[r] = 0u;
}

// Cell of each hit: row = layer * ny + iy (-1 when the hit is outside the
// window or its plane is not read out) and column ix, for IMG_UNROLL hits per
// thread (independent loads, all in flight together).
struct HitCells {
    int row[IMG_UNROLL], col[IMG_UNROLL];
    uint32_t e[IMG_UNROLL];
};

__device__ __forceinline__ HitCells load_cells(const ImgParams &Q, int64_t seg, int nh, int j0) {
    HitCells H;
    float hx[IMG_UNROLL], hy[IMG_UNROLL];
    int hl[IMG_UNROLL];
#pragma unroll
    for (int u = 0; u < IMG_UNROLL; ++u) {
        // only hits j < nh exist: no load at all for the others (the
        // segment start of a shower without handed-over hits may lie
        // outside the arrays)
        const int j = j0 + u * IMG_THREADS;
        hx[u] = hy[u] = 0.0f;
        H.e[u] = 0u;
        hl[u] = -1;
        if (j < nh) {
            const int64_t o = seg + j;
            hx[u] = Q.x[o];
            hy[u] = Q.y[o];
            H.e[u] = Q.e[o];
            hl[u] = Q.layer[o];
        }
    }
#pragma unroll
    for (int u = 0; u < IMG_UNROLL; ++u) {
        const float cx = floorf((hx[u] - Q.x0) * Q.sx);
        const float cy = floorf((hy[u] - Q.y0) * Q.sy);
        const bool in = hl[u] >= 0 && cx >= 0.0f && cx < (float)Q.nx && cy >= 0.0f && cy < (float)Q.ny;
        H.row[u] = in ? hl[u] * Q.ny + (int)cy : -1;
        H.col[u] = in ? (int)cx : 0;
    }
    return H;
}

__device__ __forceinline__ void bin_cells(const ImgParams &Q, uint32_t *slab, const HitCells &H,
                                          int row0, int rows) {
#pragma unroll
    for (int u = 0; u < IMG_UNROLL; ++u) {
        const int r = H.row[u] - row0;
        if (H.row[u] >= 0 && r >= 0 && r < rows) atomicAdd(&slab[r * Q.nx + H.col[u]], H.e[u]);
    }
}

__global__ void __launch_bounds__(IMG_THREADS) supa_images(ImgParams Q) {
    extern __shared__ uint32_t slab[];
    // hits are in place only when the propagation succeeded and they fit
    if (batch_failed(Q.ctr) || (int64_t)Q.ctr[CTR_HITS] > Q.cap) return;
    const int total_rows = Q.L * Q.ny;
    for (int i = blockIdx.x; i < Q.n; i += gridDim.x) {
        const int64_t seg = Q.seg[i];
        int nh = Q.count[(int64_t)Q.count_stride * i];
        if (seg < 0 || seg + nh > Q.cap) nh = 0;     // never read outside the hit arrays
        float *img = Q.images + (int64_t)i * total_rows * Q.nx;
        // up to IMG_THREADS * IMG_UNROLL hits stay in registers for every slab
        const bool cached = nh <= IMG_THREADS * IMG_UNROLL;
        HitCells H;
        if (cached) H = load_cells(Q, seg, nh, (int)threadIdx.x);
        for (int row0 = 0; row0 < total_rows; row0 += Q.slab_rows) {
            const int rows = min(total_rows - row0, Q.slab_rows);
            const int words = rows * Q.nx;
            clear_slab(slab, words);
            __syncthreads();
            if (cached) {
                bin_cells(Q, slab, H, row0, rows);
            } else {
                for (int j0 = (int)threadIdx.x; j0 < nh; j0 += IMG_THREADS * IMG_UNROLL)
                    bin_cells(Q, slab, load_cells(Q, seg, nh, j0), row0, rows);
            }
            __syncthreads();
            write_slab(Q, slab, img + (int64_t)row0 * Q.nx, words);
            __syncthreads();
        }
    }
}

constexpr int IMG_SLAB_WORDS = 8192;      // 32 KB of LDS per workgroup

hipError_t launch_images(const ImgParams &P0, int n_cu, hipStream_t s) {
    if (P0.n <= 0 || P0.L <= 0) return hipSuccess;
    ImgParams P = P0;
    // whole layers per slab when they fit, else bands of rows
    const int64_t lw = (int64_t)P.ny * P.nx;
    P.slab_rows = lw <= IMG_SLAB_WORDS ? (int)(IMG_SLAB_WORDS / lw) * P.ny
                                       : std::max(1, IMG_SLAB_WORDS / P.nx);
    P.slab_layers = 0;
    const int blocks = std::min(P.n, n_cu * 5);
    hipLaunchKernelGGL(supa_images, dim3(blocks), dim3(IMG_THREADS), IMG_SLAB_WORDS * 4, s, P);
    return hipGetLastError();
}

}  // namespace supa
