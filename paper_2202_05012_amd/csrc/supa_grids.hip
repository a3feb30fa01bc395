// supa_grids.hip -- per-layer grid images of hit clouds (include/supa_grids.h;
// paper, appendix "Downsampling").
//
// One workgroup per shower at a time (a grid-stride loop over showers): the
// shower's whole image, every layer's grid one after the other, is a slab of
// 64-bit integers in LDS; the workgroup's threads read the shower's hits
// coalesced, add each hit's fixed-point energy to its cell with an LDS
// atomic (integer sums: the result does not depend on the order), then write
// the slab out as float.  HBM traffic: one read of the hits and one write of
// the images.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <string>

#include "../../include/supa_grids.h"

namespace {

constexpr int THREADS = 512;

struct GridSpec {
    int nx, ny, off;
    float pad;
    double x0, y0, sx_num, sx_den, sy_num, sy_den;  // cell = floor((v - lo) * n / (hi - lo))
};

struct GridArgs {
    int64_t n;
    int L, cells;
    const int64_t *off;
    const int32_t *cnt;
    int cstride;
    int64_t len;
    const float *x, *y, *e;
    const int32_t *layer;
    float *out;
    double escale;   // 2^s
    float oscale;    // 2^-s
    GridSpec g[SUPA_GRID_MAX_LAYERS];
};

// Adds hit i (if it lands in a cell) to the slab.
__device__ inline void add_hit(const GridArgs &A, unsigned long long *slab, int l, float xf, float yf,
                               float ef) {
    if (l < 0 || l >= A.L) return;
    if (!(ef >= 0.0f) || !__builtin_isfinite(ef)) return;
    const GridSpec &G = A.g[l];
    const double fx = __builtin_floor(((double)xf - G.x0) * G.sx_num / G.sx_den);
    const double fy = __builtin_floor(((double)yf - G.y0) * G.sy_num / G.sy_den);
    if (!(fx >= 0.0 && fx < (double)G.nx && fy >= 0.0 && fy < (double)G.ny)) return;
    const double q = __builtin_rint((double)ef * A.escale);
    if (!(q < 9.2e18)) return;
    atomicAdd(&slab[G.off + (int)fy * G.nx + (int)fx], (unsigned long long)q);
}

__global__ void __launch_bounds__(THREADS) grids_kernel(GridArgs A) {
    extern __shared__ unsigned long long slab[];
    const int t = threadIdx.x;
    for (int c = t; c < A.cells; c += THREADS) slab[c] = 0ull;
    __syncthreads();
    // the next shower's segment is requested while the current one is binned
    int64_t s = blockIdx.x;
    int64_t na = 0, nc = 0;
    if (s < A.n) {
        na = A.off[s];
        nc = A.cnt[(size_t)s * A.cstride];
    }
    for (; s < A.n; s += gridDim.x) {
        int64_t a = na, b = na + nc;
        const int64_t sn = s + gridDim.x;
        if (sn < A.n) {
            na = A.off[sn];
            nc = A.cnt[(size_t)sn * A.cstride];
        }
        a = a < 0 ? 0 : a;               // never outside the arrays
        b = b > A.len ? A.len : b;
        // four hits per thread per round, all requested before any is used
        for (int64_t i = a + t; i < b; i += 4 * THREADS) {
            int lv[4];
            float xv[4], yv[4], ev[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int64_t j = i + (int64_t)k * THREADS;
                const bool in = j < b;
                lv[k] = in ? A.layer[j] : -1;
                xv[k] = in ? A.x[j] : 0.0f;
                yv[k] = in ? A.y[j] : 0.0f;
                ev[k] = in ? A.e[j] : 0.0f;
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) add_hit(A, slab, lv[k], xv[k], yv[k], ev[k]);
        }
        __syncthreads();
        // write the image and leave the slab zero for the next shower
        float *o = A.out + (size_t)s * A.cells;
        for (int c = t; c < A.cells; c += THREADS) {
            o[c] = (float)slab[c] * A.oscale;
            slab[c] = 0ull;
        }
        __syncthreads();
    }
}

thread_local std::string t_err;

supa_status bad_arg(const char *msg) {
    t_err = msg;
    return SUPA_ERR_INVALID_ARG;
}

int g_cu = 0;

int cu_count() {
    if (!g_cu) {
        int dev = 0, n = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
            g_cu = n;
        else
            g_cu = 256;
    }
    return g_cu;
}

}  // namespace

extern "C" const char *supa_grids_last_error(void) { return t_err.c_str(); }

extern "C" int64_t supa_grid_cells(const supa_grid *grids, int32_t n_layers) {
    if (!grids || n_layers < 1 || n_layers > SUPA_GRID_MAX_LAYERS) return -1;
    int64_t c = 0;
    for (int l = 0; l < n_layers; ++l) {
        const supa_grid &g = grids[l];
        if (g.nx < 1 || g.ny < 1 || !std::isfinite(g.x0) || !std::isfinite(g.x1) || !std::isfinite(g.y0) ||
            !std::isfinite(g.y1) || !(g.x1 > g.x0) || !(g.y1 > g.y0))
            return -1;
        c += (int64_t)g.nx * g.ny;
        if (c > (int64_t)1 << 40) return -1;
    }
    return c;
}

extern "C" supa_status supa_bin_grids(void *stream, int64_t n, int32_t n_layers, const supa_grid *grids,
                                      int32_t energy_frac_bits, const int64_t *hit_offsets,
                                      const int32_t *hit_counts, int32_t counts_stride, int64_t hit_len,
                                      const float *hit_x, const float *hit_y, const float *hit_e,
                                      const int32_t *hit_layer, float *images) {
    if (n < 0 || n > INT32_MAX) return bad_arg("n out of range");
    const int64_t cells = supa_grid_cells(grids, n_layers);
    if (cells < 0) return bad_arg("bad grids (1..16 layers, nx, ny >= 1, finite x0 < x1, y0 < y1)");
    if (cells > SUPA_GRID_MAX_CELLS) return bad_arg("more than SUPA_GRID_MAX_CELLS cells per shower");
    if (energy_frac_bits < 0 || energy_frac_bits > 31) return bad_arg("energy_frac_bits must be 0..31");
    if (counts_stride < 1) return bad_arg("counts_stride must be >= 1");
    if (hit_len < 0) return bad_arg("hit_len < 0");
    if (n == 0) return SUPA_OK;
    if (!hit_offsets || !hit_counts || !images || (hit_len > 0 && (!hit_x || !hit_y || !hit_e || !hit_layer)))
        return bad_arg("NULL array");
    GridArgs A{};
    A.n = n;
    A.L = n_layers;
    A.cells = (int)cells;
    A.off = hit_offsets;
    A.cnt = hit_counts;
    A.cstride = counts_stride;
    A.len = hit_len;
    A.x = hit_x;
    A.y = hit_y;
    A.e = hit_e;
    A.layer = hit_layer;
    A.out = images;
    A.escale = std::ldexp(1.0, energy_frac_bits);
    A.oscale = std::ldexp(1.0f, -energy_frac_bits);
    int off = 0;
    for (int l = 0; l < n_layers; ++l) {
        const supa_grid &g = grids[l];
        A.g[l] = GridSpec{g.nx, g.ny, off, 0.0f, g.x0, g.y0, (double)g.nx, g.x1 - g.x0, (double)g.ny, g.y1 - g.y0};
        off += g.nx * g.ny;
    }
    int64_t blocks = (int64_t)cu_count() * 4;
    if (blocks > n) blocks = n;
    hipLaunchKernelGGL(grids_kernel, dim3((unsigned)blocks), dim3(THREADS),
                       (size_t)cells * sizeof(unsigned long long), (hipStream_t)stream, A);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        t_err = std::string("grids_kernel: ") + hipGetErrorString(e);
        return SUPA_ERR_DEVICE;
    }
    return SUPA_OK;
}
