/*
 * supa_shapes.h -- C ABI of the evaluation kernels (gfx950): shower shape
 * variables of hit point clouds and the normalised Wasserstein-1 distance
 * between two samples of any per-shower or per-point variable.
 *
 * Shower shape variables: paper, section "Shower Shape Variables" (feature
 * means and standard deviations of eta = x, phi = y, r = sqrt(x^2 + y^2) and
 * E; layer energy; total energy) and appendix "More shower shape variables"
 * (layer centroids and lateral widths, energy fraction per layer, energy
 * ratio of the two largest deposits, shower depth and its width).  Distance:
 * section "Performance Analysis of Generative Models" -- Wasserstein-1
 * between histograms of the two samples' marginals, after normalising both
 * by the mean and standard deviation of the reference sample, averaged over
 * groups of marginals ("mean discrepancy").
 *
 * Conventions (all entry points):
 *   - pointers are device pointers owned by the caller unless marked host;
 *   - work is enqueued on `hip_stream` (hipStream_t, NULL = default stream)
 *     and nothing is synchronised;
 *   - return SUPA_OK, SUPA_ERR_INVALID_ARG (bad sizes or NULL pointers,
 *     nothing launched) or SUPA_ERR_DEVICE; supa_shapes_last_error() gives the
 *     message of the calling thread's last error.
 */
#ifndef SUPA_SHAPES_H
#define SUPA_SHAPES_H

#include <stddef.h>
#include <stdint.h>

#include "supa.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Columns of the per-layer record (float [n][n_layers][SUPA_LAYER_VARS]).
 * Layers are numbered from 0; for layer i of one shower, over its points j:
 *   COUNT          number of points
 *   MEAN_v         sum_j v_j / COUNT                       (v = x, y, r, E)
 *   STD_v          sqrt(sum_j v_j^2 / COUNT - MEAN_v^2)     (unweighted)
 *   ENERGY         E_i = sum_j E_j
 *   CENTROID_v     sum_j E_j v_j / E_i                     (v = x, y, r)
 *   WIDTH_v        sqrt(sum_j E_j v_j^2 / E_i - CENTROID_v^2)
 *   FRACTION       E_i / E_tot
 *   ENERGY_RATIO   (E[1] - E[2]) / (E[1] + E[2]), the two largest point
 *                  energies of the layer, E[2] = 0 when it has one point.
 * A layer without points has COUNT 0, ENERGY 0 and NaN means, deviations,
 * centroids, widths and ratio; a variance that rounds below zero counts as 0;
 * FRACTION is NaN when E_tot is 0. */
enum {
    SUPA_LV_COUNT = 0, SUPA_LV_MEAN_X, SUPA_LV_MEAN_Y, SUPA_LV_MEAN_R, SUPA_LV_MEAN_E,
    SUPA_LV_STD_X, SUPA_LV_STD_Y, SUPA_LV_STD_R, SUPA_LV_STD_E, SUPA_LV_ENERGY,
    SUPA_LV_CENTROID_X, SUPA_LV_CENTROID_Y, SUPA_LV_CENTROID_R,
    SUPA_LV_WIDTH_X, SUPA_LV_WIDTH_Y, SUPA_LV_WIDTH_R, SUPA_LV_FRACTION, SUPA_LV_ENERGY_RATIO,
    SUPA_LAYER_VARS = 18
};

/* Columns of the per-shower record (float [n][SUPA_SHOWER_VARS]):
 *   E_TOT     sum_i E_i
 *   DEPTH     deepest layer with E_i > 0 (-1: none)
 *   L_D       sum_i i E_i
 *   S_D       L_D / E_tot (NaN when E_tot is 0)
 *   S_D_WIDTH sqrt(sum_i i^2 E_i / E_tot - S_D^2), over every layer
 *             (NaN when E_tot is 0). */
enum {
    SUPA_SV_E_TOT = 0, SUPA_SV_DEPTH, SUPA_SV_L_D, SUPA_SV_S_D, SUPA_SV_S_D_WIDTH,
    SUPA_SHOWER_VARS = 5
};

/*
 * Shape variables of n showers whose hits are stored segment by segment (the
 * hit layout of supa_simulate): the hits of shower s are the entries
 * [hit_offsets[s], hit_offsets[s] + hit_counts[s * counts_stride]) of
 * hit_x, hit_y, hit_e (float) and hit_layer (int32), arrays of hit_len
 * entries; every segment must lie inside [0, hit_len) (the kernel reads
 * aligned blocks of 32 entries that may reach outside a segment, never
 * outside the arrays; it cannot check the segments).  Hits of layer -1 (planes
 * not read out) are skipped.  Within a segment the hits of one layer must be
 * contiguous (true for supa_simulate's output, which groups each segment by
 * layer, whatever its layer map).
 *   n             showers, 0 <= n <= 2^31 - 1 (0: nothing is launched)
 *   n_layers      L, 1..64; hit layers must be < L
 *   layer_vars    out, float [n][L][SUPA_LAYER_VARS]
 *   shower_vars   out, float [n][SUPA_SHOWER_VARS]
 *   work          device, work_ints >= supa_shapes_work_ints(n) int32 owned
 *                 by the caller, overwritten: after the call work[0] holds
 *                 the number of showers that broke the contiguity rule or
 *                 carried a layer >= L (all their variables are NaN); the
 *                 rest is the kernel's own (a work queue, bucket counts, and
 *                 the order in which showers are taken: longest first, over
 *                 the whole batch when every shower fits in flight at once,
 *                 else within windows of consecutive showers, so that the
 *                 lanes of a wave carry showers of similar length while the
 *                 showers in flight stay close together in memory).  The
 *                 results do not depend on that order.
 * Sums are taken in double precision; results are rounded to float.
 */
supa_status supa_shower_shapes(void *hip_stream, int64_t n, int32_t n_layers,
                               const int64_t *hit_offsets, const int32_t *hit_counts,
                               int32_t counts_stride, int64_t hit_len, const float *hit_x,
                               const float *hit_y,
                               const float *hit_e, const int32_t *hit_layer, float *layer_vars,
                               float *shower_vars, int32_t *work, int64_t work_ints);

/* int32 entries of supa_shower_shapes' work array for n showers (2052 + n;
 * -1 for n < 0). */
int64_t supa_shapes_work_ints(int64_t n);

/* r = sqrt(x^2 + y^2) for n points (float, rounded from double), the radial
 * point feature whose marginal the paper compares besides eta, phi and E. */
supa_status supa_hit_radius(void *hip_stream, int64_t n, const float *x, const float *y, float *r);

/*
 * Normalised Wasserstein-1 distance, column by column, between a reference
 * sample (rows of `ref`, element (i, c) at ref[i * ref_ld + c]) and a sample
 * `smp` (same layout with smp_ld), over n_cols columns; non-finite entries are
 * left out.  For each column: both samples are histogrammed over the same
 * n_bins equal bins spanning [lo, hi], the smallest and largest finite value
 * of the two samples together (bin of v: floor((v - lo) * (n_bins / (hi - lo)))
 * in double precision, the top edge in the last bin); the distance of the two
 * histograms with each bin's mass at its centre is
 *   W = (hi - lo) / n_bins * sum_k |F_ref(k) - F_smp(k)|
 * (F = cumulative fractions) and w1[c] = W / sigma_ref, sigma_ref the
 * population standard deviation of the reference column (normalising both
 * samples by the reference mean and deviation leaves W / sigma_ref).  A
 * column is skipped (w1[c] = NaN) when the reference has fewer than 2 finite
 * values or all of them are equal, or the sample has none.
 *   n_ref, n_smp   rows, 1..2^31 - 1;  ref_ld, smp_ld >= n_cols
 *   n_cols         1..65535;  n_bins 1..4096
 *   w1             out, double [n_cols]
 *   group_of_col   NULL, or int32 [n_cols] with values in [-1, n_groups):
 *                  group_mean[g] (out, double [n_groups]) = mean of the
 *                  non-NaN w1[c] with group_of_col[c] == g (NaN if none) --
 *                  the "mean discrepancy" of a group of marginals
 *   workspace      device, workspace_bytes >= supa_w1_workspace_bytes(...)
 */
size_t supa_w1_workspace_bytes(int32_t n_cols, int32_t n_bins, int64_t n_ref, int64_t n_smp);
supa_status supa_w1_normalized(void *hip_stream, int32_t n_cols, const float *ref, int64_t n_ref,
                               int64_t ref_ld, const float *smp, int64_t n_smp, int64_t smp_ld,
                               int32_t n_bins, const int32_t *group_of_col, int32_t n_groups,
                               double *w1, double *group_mean, void *workspace,
                               size_t workspace_bytes);

const char *supa_shapes_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SUPA_SHAPES_H */
