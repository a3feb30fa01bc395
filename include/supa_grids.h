/*
 * supa_grids.h -- C ABI of per-layer grid images (gfx950): hit point clouds
 * downsampled to images with a different region of interest and number of
 * cells for every layer (paper, appendix "Downsampling": per layer a
 * rectangular region and a number of cells in each direction, each cell the
 * sum of the energies of the points inside it; the CaloGAN-like read-out of
 * 3 x 96, 12 x 12 and 12 x 6 cells and its 2x and 3x multiples are such grids).
 *
 * Conventions: pointers are device pointers owned by the caller unless marked
 * host; work is enqueued on `hip_stream` (hipStream_t, NULL = default stream)
 * and nothing is synchronised; returns SUPA_OK, SUPA_ERR_INVALID_ARG (nothing
 * launched) or SUPA_ERR_DEVICE; supa_grids_last_error() gives the message of
 * the calling thread's last error.
 */
#ifndef SUPA_GRIDS_H
#define SUPA_GRIDS_H

#include <stdint.h>

#include "supa.h"

#ifdef __cplusplus
extern "C" {
#endif

enum { SUPA_GRID_MAX_LAYERS = 16, SUPA_GRID_MAX_CELLS = 8192 };

/* Grid of one layer: nx cells over [x0, x1) and ny cells over [y0, y1); a
 * point lands in column floor((x - x0) * nx / (x1 - x0)) and row
 * floor((y - y0) * ny / (y1 - y0)) (double precision), when both are inside. */
typedef struct supa_grid {
    int32_t nx, ny;
    double x0, x1, y0, y1;
} supa_grid;

/* Cells per shower: sum over layers of nx * ny (host; -1 on bad grids). */
int64_t supa_grid_cells(const supa_grid *grids, int32_t n_layers);

/*
 * Images of n showers whose hits are stored segment by segment (the hit
 * layout of supa_simulate: the hits of shower s are the entries
 * [hit_offsets[s], hit_offsets[s] + hit_counts[s * counts_stride]) of the
 * hit arrays, which have hit_len entries; entries at or beyond hit_len are
 * never read).
 *   n_layers, grids   1..SUPA_GRID_MAX_LAYERS layers, grids[l] (host) for
 *                     layer l; hits of layer -1 or >= n_layers are dropped,
 *                     and so are hits outside their layer's region
 *   energy_frac_bits  s: every hit adds rint(E * 2^s) as an integer, exact
 *                     for the energies supa_simulate writes (multiples of
 *                     2^-s); hits with a negative or non-finite energy are
 *                     dropped
 *   images            out, float [n][cells] with cells = supa_grid_cells(),
 *                     layer l's image [ny_l][nx_l] (row = y cell) starting at
 *                     the sum of the earlier layers' cells; a cell holds
 *                     float(sum of its integers) * 2^-s, so results do not
 *                     depend on the order of the hits
 * At most SUPA_GRID_MAX_CELLS cells per shower (one shower's image sits in
 * LDS while its hits are binned).
 */
supa_status supa_bin_grids(void *hip_stream, int64_t n, int32_t n_layers, const supa_grid *grids,
                           int32_t energy_frac_bits, const int64_t *hit_offsets,
                           const int32_t *hit_counts, int32_t counts_stride, int64_t hit_len,
                           const float *hit_x, const float *hit_y, const float *hit_e,
                           const int32_t *hit_layer, float *images);

const char *supa_grids_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SUPA_GRIDS_H */
