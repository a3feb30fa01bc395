/*
 * supa_oracle.c -- plain FP64 CPU oracle of the SUPA propagation model.
 *
 * TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU-baseline timing).  Slow and
 * obvious on purpose: one shower at a time, one plane at a time, one particle at
 * a time, no blocking, no reordering.  Shares no code with the HIP library.
 *
 * The process (paper, section "Propagation Model", Algorithm 1):
 *   A particle starts at the origin with an energy and a velocity; slices
 *   (planes) sit at evenly spaced z.  Each time a particle reaches a plane it
 *   either stops and deposits its energy (a hit, recorded with its energy and
 *   location), splits into two particles whose energies are E*(theta/2 +- eps)/
 *   theta, or passes through unchanged.  After the last plane every deposit is
 *   collected; planes are grouped into layers and z is projected out.
 *
 * Readings taken where the paper is silent or garbled:
 *   - energies are unsigned fixed-point integers with `frac_bits` fractional
 *     bits; the primary is rounded to nearest-even, a split gives
 *     E_a = floor(E*F/2^32) and E_b = E - E_a with F the 32-bit fraction, so the
 *     split of Algorithm 1 conserves energy exactly (f = 1/2 + eps/theta);
 *   - the three-way choice of Algorithm 1 compares the first 32-bit word w0 of
 *     one Philox4x32-10 block against integer thresholds C1 = floor(p_stop*2^32)
 *     and C2 = C1 + floor(p_split*2^32): stop iff w0 < C1, split iff
 *     C1 <= w0 < C2, pass otherwise;
 *   - the block is keyed by the 64-bit seed and counted by (plane k, shower id,
 *     path id low, path id high), the path id being 1 for the primary and
 *     2p, 2p+1 for the two daughters of path p;
 *   - an energy threshold is checked first when a particle arrives at a plane:
 *     below it, the particle deposits its energy there (a "cut" hit);
 *   - regional parameters (section "Extensions": slices divided into regions
 *     with their own parameters) are taken as concentric rings around the
 *     beam axis: the ring of a particle arriving at plane k is the number of
 *     ring radii <= r = sqrt(x^2 + y^2), and its stop / split probabilities are
 *     those of (ring, plane);
 *   - a particle flies in a straight line between planes ("continues with its
 *     original velocity"); it leaves the detector after the last plane or when
 *     its direction no longer points to +z;
 *   - a split turns the parent direction d by angles theta*(1-f) and theta*f to
 *     opposite sides of the plane through d at azimuth omega, so the opening
 *     angle of the two daughters is theta; omega is measured in the frame
 *     obtained by the rotation that takes +z to d (Rodrigues), applied to +x
 *     and +y.
 * With kinematics = ORACLE_KIN_LITERAL the motion is Algorithm 1 as printed
 * instead: a particle has a lateral position only (the primary starts at its
 * impact point and moves along +z, whatever its angles); a pass keeps the
 * position; a split places the daughters at p + dz*(sin(theta/2 + eps),
 * cos(theta/2 + eps)) and p - dz*(same), the first one carrying E(theta/2 +
 * eps)/theta, with eps = (f - 1/2)*theta; omega is drawn and not used.  The
 * daughters are displaced at the split and reach the next plane there.
 */
#include "supa_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw: "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11).  Ten rounds; each round multiplies counter words */
/* 0 and 2 by the two Philox multipliers, xors the high halves with the other */
/* words and the round key, and the key is bumped by the two Weyl constants.  */
/* ------------------------------------------------------------------------ */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void oracle_philox4x32_10(uint32_t k0, uint32_t k1, uint32_t c0, uint32_t c1,
                          uint32_t c2, uint32_t c3, uint32_t out[4])
{
    uint32_t x0 = c0, x1 = c1, x2 = c2, x3 = c3;
    for (int round = 0; round < 10; ++round) {
        uint64_t prod0 = (uint64_t)PHILOX_M0 * (uint64_t)x0;
        uint64_t prod1 = (uint64_t)PHILOX_M1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += PHILOX_W0;
        k1 += PHILOX_W1;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* u(w) = (w + 1/2) / 2^32, strictly inside (0, 1); exact in double. */
static double unit_open(uint32_t w) { return ((double)w + 0.5) * 0x1p-32; }

/* ------------------------------------------------------------------------ */
/* Result storage                                                            */
/* ------------------------------------------------------------------------ */
static int grow(void **p, int64_t cap, size_t elem)
{
    void *q = realloc(*p, (size_t)cap * elem);
    if (!q) return 0;
    *p = q;
    return 1;
}

static int ensure_hits(oracle_result *r, int64_t need)
{
    if (need <= r->cap_hits) return 1;
    int64_t cap = r->cap_hits ? r->cap_hits : 1024;
    while (cap < need) cap *= 2;
    if (!grow((void **)&r->hit_sid, cap, sizeof(int32_t))) return 0;
    if (!grow((void **)&r->hit_plane, cap, sizeof(int32_t))) return 0;
    if (!grow((void **)&r->hit_layer, cap, sizeof(int32_t))) return 0;
    if (!grow((void **)&r->hit_kind, cap, sizeof(int32_t))) return 0;
    if (!grow((void **)&r->hit_x, cap, sizeof(double))) return 0;
    if (!grow((void **)&r->hit_y, cap, sizeof(double))) return 0;
    if (!grow((void **)&r->hit_e, cap, sizeof(uint32_t))) return 0;
    if (!grow((void **)&r->hit_key, cap, sizeof(uint64_t))) return 0;
    r->cap_hits = cap;
    return 1;
}

static int ensure_nodes(oracle_result *r, int64_t need)
{
    if (need <= r->cap_nodes) return 1;
    int64_t cap = r->cap_nodes ? r->cap_nodes : 1024;
    while (cap < need) cap *= 2;
    if (!grow((void **)&r->node_sid, cap, sizeof(int32_t))) return 0;
    if (!grow((void **)&r->node_parent, cap, sizeof(int32_t))) return 0;
    if (!grow((void **)&r->node_gen, cap, sizeof(int32_t))) return 0;
    if (!grow((void **)&r->node_vx, cap, sizeof(double))) return 0;
    if (!grow((void **)&r->node_vy, cap, sizeof(double))) return 0;
    if (!grow((void **)&r->node_vz, cap, sizeof(double))) return 0;
    if (!grow((void **)&r->node_e, cap, sizeof(uint32_t))) return 0;
    if (!grow((void **)&r->node_key, cap, sizeof(uint64_t))) return 0;
    r->cap_nodes = cap;
    return 1;
}

void oracle_free(oracle_result *r)
{
    free(r->hit_sid); free(r->hit_plane); free(r->hit_layer); free(r->hit_kind);
    free(r->hit_x); free(r->hit_y); free(r->hit_e); free(r->hit_key);
    free(r->node_sid); free(r->node_parent); free(r->node_gen);
    free(r->node_vx); free(r->node_vy); free(r->node_vz);
    free(r->node_e); free(r->node_key);
    free(r->ledger); free(r->counts); free(r->peak_frontier); free(r->region_margin);
    memset(r, 0, sizeof(*r));
}

/* ------------------------------------------------------------------------ */
/* One particle of the frontier                                              */
/* ------------------------------------------------------------------------ */
typedef struct {
    double x, y, z;     /* position                                  */
    double dx, dy, dz;  /* unit direction of flight                  */
    uint32_t e;         /* fixed-point energy                        */
    uint64_t path;      /* 1 for the primary; 2p / 2p+1 for daughters */
    int32_t node;       /* shower-local tree node index              */
    int32_t gen;        /* number of splits since the primary        */
} particle;

typedef struct {
    particle *v;
    int64_t n, cap;
} plist;

static int plist_push(plist *l, const particle *p)
{
    if (l->n == l->cap) {
        int64_t cap = l->cap ? 2 * l->cap : 64;
        particle *q = (particle *)realloc(l->v, (size_t)cap * sizeof(particle));
        if (!q) return 0;
        l->v = q;
        l->cap = cap;
    }
    l->v[l->n++] = *p;
    return 1;
}

/* Constants derived once per run from the parameters. */
typedef struct {
    uint64_t t_cut;      /* ceil(e_cut * 2^s)                 */
    uint64_t *c1, *c2;   /* stop / split thresholds per plane */
    uint64_t f_lo, f_w;  /* fraction F = f_lo + floor(w1*f_w/2^32) */
} derived;

static int add_hit(oracle_result *r, uint32_t sid, const particle *p, int32_t plane,
                   int32_t layer, int32_t kind)
{
    if (!ensure_hits(r, r->n_hits + 1)) return 0;
    int64_t h = r->n_hits++;
    r->hit_sid[h] = (int32_t)sid;
    r->hit_plane[h] = plane;
    r->hit_layer[h] = layer;
    r->hit_kind[h] = kind;
    r->hit_x[h] = p->x;
    r->hit_y[h] = p->y;
    r->hit_e[h] = p->e;
    r->hit_key[h] = p->path;
    return 1;
}

static int add_node(oracle_result *r, uint32_t sid, int32_t parent, int32_t gen,
                    double vx, double vy, double vz, uint32_t e, uint64_t key)
{
    if (!ensure_nodes(r, r->n_nodes + 1)) return 0;
    int64_t j = r->n_nodes++;
    r->node_sid[j] = (int32_t)sid;
    r->node_parent[j] = parent;
    r->node_gen[j] = gen;
    r->node_vx[j] = vx;
    r->node_vy[j] = vy;
    r->node_vz[j] = vz;
    r->node_e[j] = e;
    r->node_key[j] = key;
    return 1;
}

/*
 * Split of one particle (Algorithm 1, split branch; section "Propagation
 * Model": two particles generated at the split location).  Words w1..w3 of
 * the particle's Philox block drive the energy fraction, the opening angle and
 * the azimuth.  Writes the two daughters, a then b.
 */
static void split_particle(const oracle_geometry *g, const derived *dv, const particle *p,
                           const uint32_t w[4], particle *a, particle *b)
{
    /* energy fraction and exact fixed-point split (E_{0,1} = E(theta/2 +- eps)/theta) */
    uint64_t F = dv->f_lo + (((uint64_t)w[1] * dv->f_w) >> 32);
    uint32_t ea = (uint32_t)(((uint64_t)p->e * F) >> 32);
    uint32_t eb = p->e - ea;
    double f = (double)F * 0x1p-32;

    /* opening angle theta ~ p_theta */
    double theta;
    if (g->angle_mode == ORACLE_ANGLE_FIXED)
        theta = g->angle_a;
    else if (g->angle_mode == ORACLE_ANGLE_UNIFORM)
        theta = g->angle_a + (g->angle_b - g->angle_a) * unit_open(w[2]);
    else
        theta = g->angle_a * sqrt(-2.0 * log(unit_open(w[2])));

    /* azimuth of the splitting plane, omega ~ U(0, 2 pi) */
    double omega = 2.0 * M_PI * unit_open(w[3]);

    /* deflections of the two daughters, to opposite sides */
    double aa = theta * (1.0 - f);
    double ab = theta * f;

    /* frame (e1, e2) perpendicular to d: Rodrigues rotation +z -> d applied to +x, +y */
    double dx = p->dx, dy = p->dy, dz = p->dz;
    double c = 1.0 / (1.0 + dz);
    double e1x = 1.0 - dx * dx * c, e1y = -dx * dy * c, e1z = -dx;
    double e2x = -dx * dy * c, e2y = 1.0 - dy * dy * c, e2z = -dy;
    double nx = cos(omega) * e1x + sin(omega) * e2x;
    double ny = cos(omega) * e1y + sin(omega) * e2y;
    double nz = cos(omega) * e1z + sin(omega) * e2z;

    *a = *p;
    *b = *p;
    if (g->kinematics == ORACLE_KIN_LITERAL) {
        /* Algorithm 1 as printed: one displacement, + for the first daughter, -
           for the second; directions stay along +z */
        double eps = (f - 0.5) * theta;
        double ux = g->dz * sin(theta / 2.0 + eps), uy = g->dz * cos(theta / 2.0 + eps);
        a->x = p->x + ux;
        a->y = p->y + uy;
        b->x = p->x - ux;
        b->y = p->y - uy;
        a->e = ea;
        b->e = eb;
        a->path = 2 * p->path;
        b->path = 2 * p->path + 1;
        a->gen = b->gen = p->gen + 1;
        return;
    }
    a->dx = cos(aa) * dx + sin(aa) * nx;
    a->dy = cos(aa) * dy + sin(aa) * ny;
    a->dz = cos(aa) * dz + sin(aa) * nz;
    b->dx = cos(ab) * dx - sin(ab) * nx;
    b->dy = cos(ab) * dy - sin(ab) * ny;
    b->dz = cos(ab) * dz - sin(ab) * nz;
    a->e = ea;
    b->e = eb;
    a->path = 2 * p->path;
    b->path = 2 * p->path + 1;
    a->gen = b->gen = p->gen + 1;
}

/* One shower; returns ORACLE_OK or an error code. */
static int simulate_one(const oracle_geometry *g, const derived *dv, int64_t i,
                        uint32_t sid, uint64_t seed, float e0f, float polf, float azf,
                        float x0f, float y0f, oracle_result *r)
{
    uint64_t *ledger = r->ledger + 4 * i;
    int32_t *cnt = r->counts + 6 * i;
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);

    /* primary energy, rounded to nearest-even in fixed point */
    double scaled = ldexp((double)e0f, g->frac_bits);
    if (!(scaled >= 0.0)) return ORACLE_ERR_RANGE;
    double rounded = nearbyint(scaled);
    if (rounded >= 4294967296.0) return ORACLE_ERR_RANGE;
    uint32_t e0 = (uint32_t)rounded;

    /* primary at (x0, y0, 0) moving along polar angle alpha, azimuth beta */
    double alpha = (double)polf, beta = (double)azf;
    particle p;
    p.x = (double)x0f;
    p.y = (double)y0f;
    p.z = 0.0;
    p.dx = sin(alpha) * cos(beta);
    p.dy = sin(alpha) * sin(beta);
    p.dz = cos(alpha);
    if (g->kinematics == ORACLE_KIN_LITERAL) {   /* lateral position only */
        p.dx = 0.0;
        p.dy = 0.0;
        p.dz = 1.0;
    }
    p.e = e0;
    p.path = 1;
    p.gen = 0;
    int32_t n_nodes = 0;
    p.node = n_nodes++;
    if (!add_node(r, sid, -1, 0, p.x, p.y, p.z, p.e, p.path)) return ORACLE_ERR_NOMEM;

    uint64_t e_stop = 0, e_cut = 0, e_esc = 0;
    double margin = INFINITY;
    int32_t n_hits = 0, n_steps = 0, n_splits = 0, n_escaped = 0, n_backward = 0, peak = 1;

    plist cur = {0, 0, 0}, nxt = {0, 0, 0};
    int status = ORACLE_OK;
    if (!plist_push(&cur, &p)) return ORACLE_ERR_NOMEM;

    for (int32_t k = 0; k < g->n_planes && status == ORACLE_OK; ++k) {
        double zk = g->z_first + (double)k * g->dz;
        int32_t layer = g->layer_of_plane ? g->layer_of_plane[k] : k;
        nxt.n = 0;
        for (int64_t j = 0; j < cur.n; ++j) {
            particle q = cur.v[j];
            /* free flight to plane k; a particle not moving towards +z leaves */
            if (!(q.dz > 0.0)) {
                e_esc += q.e;
                ++n_escaped;
                ++n_backward;
                continue;
            }
            double t = (zk - q.z) / q.dz;
            q.x += t * q.dx;
            q.y += t * q.dy;
            q.z = zk;
            ++n_steps;

            /* energy threshold: deposit everything here */
            if ((uint64_t)q.e < dv->t_cut) {
                if (!add_hit(r, sid, &q, k, layer, ORACLE_HIT_CUT)) { status = ORACLE_ERR_NOMEM; break; }
                e_cut += q.e;
                ++n_hits;
                continue;
            }

            /* the particle's ring (regional parameters) */
            int32_t ring = 0;
            if (g->n_regions >= 2) {
                double rr = sqrt(q.x * q.x + q.y * q.y);
                for (int32_t b = 0; b < g->n_regions - 1; ++b) {
                    if (rr >= g->region_r[b]) ++ring;
                    double d = fabs(rr - g->region_r[b]);
                    if (d < margin) margin = d;
                }
            }
            const uint64_t c1 = dv->c1[(int64_t)ring * g->n_planes + k];
            const uint64_t c2 = dv->c2[(int64_t)ring * g->n_planes + k];

            /* three-way choice of Algorithm 1 */
            uint32_t w[4];
            oracle_philox4x32_10(k0, k1, (uint32_t)k, sid, (uint32_t)q.path,
                                 (uint32_t)(q.path >> 32), w);
            if ((uint64_t)w[0] < c1) {                    /* stop: deposit */
                if (!add_hit(r, sid, &q, k, layer, ORACLE_HIT_STOP)) { status = ORACLE_ERR_NOMEM; break; }
                e_stop += q.e;
                ++n_hits;
            } else if ((uint64_t)w[0] < c2) {             /* split in two */
                particle a, b;
                split_particle(g, dv, &q, w, &a, &b);
                a.node = n_nodes++;
                b.node = n_nodes++;
                if (!add_node(r, sid, q.node, a.gen, q.x, q.y, q.z, a.e, a.path) ||
                    !add_node(r, sid, q.node, b.gen, q.x, q.y, q.z, b.e, b.path) ||
                    !plist_push(&nxt, &a) || !plist_push(&nxt, &b)) {
                    status = ORACLE_ERR_NOMEM;
                    break;
                }
                ++n_splits;
            } else {                                      /* pass through */
                if (!plist_push(&nxt, &q)) { status = ORACLE_ERR_NOMEM; break; }
            }
        }
        plist tmp = cur;
        cur = nxt;
        nxt = tmp;
        if (cur.n > peak) peak = (int32_t)cur.n;
    }
    /* everything still moving after the last plane leaks out */
    for (int64_t j = 0; j < cur.n; ++j) {
        e_esc += cur.v[j].e;
        ++n_escaped;
    }
    free(cur.v);
    free(nxt.v);

    ledger[0] = e0;
    ledger[1] = e_stop;
    ledger[2] = e_cut;
    ledger[3] = e_esc;
    cnt[0] = n_nodes;
    cnt[1] = n_hits;
    cnt[2] = n_steps;
    cnt[3] = n_splits;
    cnt[4] = n_escaped;
    cnt[5] = n_backward;
    r->peak_frontier[i] = peak;
    r->region_margin[i] = margin;
    return status;
}

static int validate(const oracle_geometry *g)
{
    if (g->n_planes < 1 || g->n_planes > 63) return ORACLE_ERR_INVALID_ARG;
    if (!(g->dz > 0.0) || !(g->z_first > 0.0) || !isfinite(g->z_first) || !isfinite(g->dz))
        return ORACLE_ERR_INVALID_ARG;
    if (!(g->e_cut >= 0.0) || !isfinite(g->e_cut)) return ORACLE_ERR_INVALID_ARG;
    if (g->frac_bits < 0 || g->frac_bits > 31) return ORACLE_ERR_INVALID_ARG;
    if (!(g->frac_lo >= 0.0 && g->frac_lo <= g->frac_hi && g->frac_hi <= 1.0)) return ORACLE_ERR_INVALID_ARG;
    if (g->angle_mode < ORACLE_ANGLE_FIXED || g->angle_mode > ORACLE_ANGLE_RAYLEIGH) return ORACLE_ERR_INVALID_ARG;
    if (g->kinematics != ORACLE_KIN_3D && g->kinematics != ORACLE_KIN_LITERAL) return ORACLE_ERR_INVALID_ARG;
    if (!isfinite(g->angle_a) || !isfinite(g->angle_b)) return ORACLE_ERR_INVALID_ARG;
    if (g->n_regions < 0 || g->n_regions > 4) return ORACLE_ERR_INVALID_ARG;
    int32_t rings = g->n_regions >= 2 ? g->n_regions : 1;
    if (rings >= 2) {
        if (!g->region_r) return ORACLE_ERR_INVALID_ARG;
        for (int32_t b = 0; b < rings - 1; ++b)
            if (!(g->region_r[b] > 0.0) || !isfinite(g->region_r[b]) ||
                (b > 0 && !(g->region_r[b] > g->region_r[b - 1])))
                return ORACLE_ERR_INVALID_ARG;
    }
    for (int64_t j = 0; j < (int64_t)rings * g->n_planes; ++j) {
        double ps = g->p_stop ? g->p_stop[j] : 0.0;
        double pl = g->p_split ? g->p_split[j] : 1.0;
        if (!(ps >= 0.0 && pl >= 0.0 && ps + pl <= 1.0)) return ORACLE_ERR_INVALID_ARG;
    }
    for (int32_t k = 0; k < g->n_planes; ++k) {
        if (g->layer_of_plane && (g->layer_of_plane[k] < -1 || g->layer_of_plane[k] >= g->n_planes))
            return ORACLE_ERR_INVALID_ARG;
    }
    return ORACLE_OK;
}

int oracle_simulate(const oracle_geometry *g, int64_t n, const float *e0,
                    const float *polar, const float *azimuth, const float *x0,
                    const float *y0, uint32_t sid_base, uint64_t seed,
                    oracle_result *r)
{
    memset(r, 0, sizeof(*r));
    int status = validate(g);
    if (status != ORACLE_OK) return status;
    if (n < 0) return ORACLE_ERR_INVALID_ARG;

    derived dv;
    dv.t_cut = (uint64_t)ceil(ldexp(g->e_cut, g->frac_bits));
    const int64_t nthr = (int64_t)(g->n_regions >= 2 ? g->n_regions : 1) * g->n_planes;
    dv.c1 = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)nthr);
    dv.c2 = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)nthr);
    if (!dv.c1 || !dv.c2) { free(dv.c1); free(dv.c2); return ORACLE_ERR_NOMEM; }
    for (int64_t j = 0; j < nthr; ++j) {
        double ps = g->p_stop ? g->p_stop[j] : 0.0;
        double pl = g->p_split ? g->p_split[j] : 1.0;
        dv.c1[j] = (uint64_t)floor(ldexp(ps, 32));
        dv.c2[j] = dv.c1[j] + (uint64_t)floor(ldexp(pl, 32));
    }
    dv.f_lo = (uint64_t)floor(ldexp(g->frac_lo, 32));
    dv.f_w = (uint64_t)floor(ldexp(g->frac_hi, 32)) - dv.f_lo;

    r->n_showers = n;
    r->ledger = (uint64_t *)calloc((size_t)(n > 0 ? n : 1) * 4, sizeof(uint64_t));
    r->counts = (int32_t *)calloc((size_t)(n > 0 ? n : 1) * 6, sizeof(int32_t));
    r->peak_frontier = (int32_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int32_t));
    r->region_margin = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    if (!r->ledger || !r->counts || !r->peak_frontier || !r->region_margin) status = ORACLE_ERR_NOMEM;

    for (int64_t i = 0; i < n && status == ORACLE_OK; ++i) {
        status = simulate_one(g, &dv, i, sid_base + (uint32_t)i, seed, e0[i], polar[i],
                              azimuth[i], x0 ? x0[i] : 0.0f, y0 ? y0[i] : 0.0f, r);
    }
    free(dv.c1);
    free(dv.c2);
    return status;
}
