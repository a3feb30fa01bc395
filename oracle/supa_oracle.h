/*
 * supa_oracle.h -- plain FP64 CPU oracle of the SUPA propagation model.
 *
 * TEST INFRASTRUCTURE. Only the test-suite, the package's smoke check and the
 * benchmark's CPU-baseline leg load this library; the product path never does.
 * It shares no code with the HIP library: its random-number generator, energy
 * arithmetic, kinematics and bookkeeping are written here, separately.
 *
 * What it computes: the particle-splitting process of the paper's section
 * "Propagation Model" and Algorithm 1 ("SUPA - Particle Splitting"), one shower
 * after another, one plane after another, one particle after another in a
 * stable order, in double precision for every coordinate and angle and in
 * unsigned fixed-point integers for every energy (see supa_oracle.c for the
 * step-by-step account and the reading taken where the paper is silent).
 */
#ifndef SUPA_ORACLE_H
#define SUPA_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORACLE_ANGLE_FIXED = 0, ORACLE_ANGLE_UNIFORM = 1, ORACLE_ANGLE_RAYLEIGH = 2 };
enum { ORACLE_KIN_3D = 0, ORACLE_KIN_LITERAL = 1 };
enum { ORACLE_OK = 0, ORACLE_ERR_INVALID_ARG = 1, ORACLE_ERR_RANGE = 2, ORACLE_ERR_NOMEM = 6 };
enum { ORACLE_HIT_STOP = 0, ORACLE_HIT_CUT = 1 };

/* Parameters of the process (Algorithm 1, "Parameters" block; Table 2). */
typedef struct {
    int32_t n_planes;              /* slices z_0..z_{N-1}                          */
    double z_first, dz;            /* z_k = z_first + k*dz                         */
    const int32_t *layer_of_plane; /* n_planes entries, or NULL for identity       */
    const double *p_stop;          /* n_planes entries, or NULL for all 0          */
    const double *p_split;         /* n_planes entries, or NULL for all 1          */
    double e_cut;                  /* energy threshold (energy units)              */
    int32_t angle_mode;            /* ORACLE_ANGLE_*                               */
    double angle_a, angle_b;       /* FIXED(a), UNIFORM(a,b), RAYLEIGH(sigma=a)    */
    double frac_lo, frac_hi;       /* energy fraction f ~ U(frac_lo, frac_hi)      */
    int32_t frac_bits;             /* fixed-point fractional bits of energies      */
    int32_t kinematics;            /* ORACLE_KIN_*                                 */
    int32_t n_regions;             /* 0 or 1: one region; 2..4: lateral rings      */
    const double *region_r;        /* n_regions - 1 ascending radii; with rings,
                                      p_stop / p_split hold n_regions * n_planes
                                      entries, ring-major ([ring][plane])          */
} oracle_geometry;

/* Growable result arrays, all owned by the oracle; free with oracle_free. */
typedef struct {
    int64_t n_hits, cap_hits;
    int32_t *hit_sid, *hit_plane, *hit_layer, *hit_kind;
    double *hit_x, *hit_y;
    uint32_t *hit_e;               /* fixed-point energy units                     */
    uint64_t *hit_key;             /* path id of the particle that deposited       */

    int64_t n_nodes, cap_nodes;
    int32_t *node_sid, *node_parent, *node_gen;   /* parent: shower-local index     */
    double *node_vx, *node_vy, *node_vz;
    uint32_t *node_e;
    uint64_t *node_key;

    int64_t n_showers;
    uint64_t *ledger;              /* per shower: E0, E_stop, E_cut, E_esc          */
    int32_t *counts;               /* per shower: nodes, hits, steps, splits, escaped,
                                      escaped because the direction no longer points to +z */
    int32_t *peak_frontier;        /* per shower: largest frontier over the planes  */
    double *region_margin;         /* per shower: smallest |r - ring radius| over the
                                      three-way choices (infinity without rings)    */
} oracle_result;

/* One Philox4x32-10 block: key (k0,k1), counter (c0..c3) -> out[4]. */
void oracle_philox4x32_10(uint32_t k0, uint32_t k1, uint32_t c0, uint32_t c1,
                          uint32_t c2, uint32_t c3, uint32_t out[4]);

/* Simulate showers i = 0..n-1 with global ids sid_base + i.  x0/y0 may be NULL.
 * Returns ORACLE_OK or an error; on error *res holds what was done so far. */
int oracle_simulate(const oracle_geometry *g, int64_t n, const float *e0,
                    const float *polar, const float *azimuth, const float *x0,
                    const float *y0, uint32_t sid_base, uint64_t seed,
                    oracle_result *res);

void oracle_free(oracle_result *res);

#ifdef __cplusplus
}
#endif
#endif
