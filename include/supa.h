/*
 * supa.h -- C ABI of the MI355X (gfx950) SUPA shower-propagation library.
 *
 * The library runs the particle-splitting process of SUPA (paper: section
 * "Propagation Model" and Algorithm 1 "SUPA - Particle Splitting") for a
 * batch of showers in hand-written HIP kernels and returns, per shower, its
 * hit point cloud (section "Propagation Model": deposits collected after the
 * last slice, z projected out per layer; "Notation": per-layer clouds of
 * (eta, phi, E)), optional per-layer images (appendix "Downsampling"), the
 * optional propagation tree (Algorithm 1's tree T), an exact energy ledger
 * and counts.
 *
 * Conventions for every function below:
 *   - every function returns a supa_status and never throws or aborts;
 *   - "device pointer" means memory on the context's GPU, allocated and owned
 *     by the caller (the library never frees it); "host pointer" means CPU
 *     memory read during the call only;
 *   - work is enqueued on the HIP stream given to supa_init_geometry;
 *     supa_simulate synchronises that stream once, at its end, to read back
 *     totals and error flags;
 *   - a context is not thread-safe; use one per stream;
 *   - after an error, supa_last_error(ctx) describes it.
 *
 * Numerics (identical in every entry point):
 *   - energies are unsigned 32-bit fixed point with `energy_frac_bits` (s)
 *     fractional bits: E_int = round-to-nearest-even(E0 * 2^s); a split gives
 *     E_a = floor(E_int * F / 2^32) and E_b = E_int - E_a, F the 32-bit energy
 *     fraction (Algorithm 1's E(theta/2 +- eps)/theta with f = 1/2 + eps/theta);
 *     float outputs are E_int * 2^-s rounded once to float;
 *   - randomness: one Philox4x32-10 block (Salmon et al., SC'11) per particle
 *     arrival, key = seed, counter = (plane k, shower id, path id low, path id
 *     high); the path id is 1 for the primary and 2p, 2p+1 for the daughters
 *     of path p, so results do not depend on launch order or batch split;
 *   - on arrival at plane k a particle below the energy threshold deposits
 *     (a "cut" hit); otherwise word w0 decides: stop if w0 < C1[k], split if
 *     C1[k] <= w0 < C2[k], pass otherwise, C1 = floor(p_stop*2^32),
 *     C2 = C1 + floor(p_split*2^32) (Algorithm 1's three-way choice);
 *   - a split turns the direction by theta*(1-f) and theta*f to opposite sides
 *     of the plane at azimuth omega = 2*pi*u(w3) (u(w) = (w + 1/2)/2^32), with
 *     theta FIXED, UNIFORM or RAYLEIGH from w2 and F from w1;
 *   - particles fly straight between planes and leave after the last plane or
 *     when their direction stops pointing to +z.
 */
#ifndef SUPA_H
#define SUPA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SUPA_ABI_VERSION 6

typedef enum supa_status {
    SUPA_OK = 0,
    SUPA_ERR_INVALID_ARG = 1, /* bad parameter, NULL where required, bad size   */
    SUPA_ERR_RANGE = 2,       /* an initial energy is < 0, NaN or >= 2^(32-s)    */
    SUPA_ERR_CAPACITY = 3,    /* caller's hit or node arrays too small; totals set */
    SUPA_ERR_DEVICE = 4,      /* a HIP runtime call failed                       */
    SUPA_ERR_STATE = 5,       /* context unusable (NULL or after a device error) */
    SUPA_ERR_NOMEM = 6        /* library could not allocate its device scratch   */
} supa_status;

enum { SUPA_ANGLE_FIXED = 0, SUPA_ANGLE_UNIFORM = 1, SUPA_ANGLE_RAYLEIGH = 2 };

/* Kinematics (supa_geometry.kinematics).
 *   SUPA_KIN_3D       particles fly in straight lines between planes and a
 *                     split turns the two daughters away from the parent's
 *                     direction (the reading of the section "Propagation
 *                     Model" described above);
 *   SUPA_KIN_LITERAL  Algorithm 1 as printed: a particle has a lateral
 *                     position only (the primary starts at its impact point,
 *                     its angles are not used); a pass keeps the position; a
 *                     split places the daughters at p + dz (sin(theta/2 + eps),
 *                     cos(theta/2 + eps)) and p - dz (same), the first one
 *                     carrying the energy fraction f = 1/2 + eps/theta, so
 *                     theta/2 + eps = f theta; the azimuth is not used. */
enum { SUPA_KIN_3D = 0, SUPA_KIN_LITERAL = 1 };

/* Output selection bits for supa_geometry.outputs. */
enum {
    SUPA_OUT_HITS = 1,   /* hit point clouds                                 */
    SUPA_OUT_IMAGES = 2, /* per-layer images (with or without hit clouds)    */
    SUPA_OUT_TREE = 4,   /* propagation tree                                 */
    SUPA_OUT_KEYS = 8    /* path ids of hits and nodes (canonical keys)      */
};

/*
 * Process parameters (Algorithm 1 "Parameters": p_stop, p_split, layer
 * configuration, slice gap, splitting angle, deviation angle; Table 2).
 * Host struct; host arrays are deep-copied by supa_init_geometry.
 */
typedef struct supa_geometry {
    int32_t n_planes;               /* N, 1..63 (path ids must fit in 64 bits)        */
    double z_first, dz;             /* plane k at z_first + k*dz; z_first > 0, dz > 0;
                                       the primary starts at z = 0                     */
    const int32_t *layer_of_plane;  /* host, N entries in [-1, N), or NULL = identity;
                                       -1 = plane not read out (hits keep layer -1 and
                                       are left out of images)                        */
    const double *p_stop;           /* host, N entries (n_regions * N with rings),
                                       or NULL = all 0                                */
    const double *p_split;          /* host, N entries (n_regions * N), or NULL = all 1;
                                       p_stop[k] + p_split[k] <= 1                    */
    double e_cut;                   /* energy threshold >= 0 (energy units)            */
    int32_t angle_mode;             /* SUPA_ANGLE_*                                   */
    double angle_a, angle_b;        /* FIXED: theta = a; UNIFORM: theta ~ U(a, b);
                                       RAYLEIGH: theta = a*sqrt(-2 ln u), sigma = a    */
    double frac_lo, frac_hi;        /* f ~ U(frac_lo, frac_hi), 0 <= lo <= hi <= 1     */
    int32_t energy_frac_bits;       /* s, 0..31 (21: resolution 2^-21, E0 < 2048)      */
    int32_t img_nx, img_ny;         /* image grid (used with SUPA_OUT_IMAGES), >= 1    */
    double img_x0, img_x1;          /* region of interest [x0, x1) x [y0, y1),         */
    double img_y0, img_y1;          /* cells half-open; x1 > x0, y1 > y0               */
    uint32_t outputs;               /* SUPA_OUT_* bitmask                             */
    int32_t kinematics;             /* SUPA_KIN_*                                     */
    /* Regional parameters (section "Extensions": slices divided into regions
       with their own parameters), taken as rings around the beam axis: a
       particle arriving at plane k is in ring j = the number of radii
       region_r[b] <= r = sqrt(x^2 + y^2), and stops / splits with the
       probabilities of (ring j, plane k).  n_regions 0 or 1: one region (the
       arrays above have N entries); 2..4: rings, region_r (host) holds
       n_regions - 1 ascending radii > 0 and p_stop / p_split hold
       n_regions * N entries, ring-major (entry j * N + k).  The ring is decided
       on float coordinates, so a particle within rounding of a radius may
       take either ring; the oracle reports each shower's margin. */
    int32_t n_regions;
    const double *region_r;
} supa_geometry;

/* Opaque context: the parameters, their device copies and library scratch. */
typedef struct supa_ctx supa_ctx;

/* Initial conditions of a batch (section "Using SUPA": energy, angle and
 * position of the incident particle).  Device pointers of n floats each. */
typedef struct supa_batch {
    const float *e0;          /* initial energy (energy units), required          */
    const float *polar;       /* polar angle from +z (radians), required           */
    const float *azimuth;     /* azimuth (radians), required                        */
    const float *x0, *y0;     /* impact point at z = 0, or NULL for 0               */
    int64_t n;                /* showers, 0 <= n <= 2^31 - 1                        */
    uint32_t shower_id_base;  /* shower i has global id shower_id_base + i          */
} supa_batch;

/*
 * Outputs.  All arrays are device pointers owned by the caller.
 * Layout is segmented (CSR): the hits of shower i occupy the contiguous range
 * [hit_offsets[i], hit_offsets[i] + counts[6*i+1]) of every hit array, with
 * hit_offsets the exclusive prefix sums of the hit counts in batch order, so
 * the segments tile [0, total_hits) in shower order.  Within a segment hits
 * are grouped by layer in increasing order (layer -1, planes not read out,
 * first) and within a layer by plane in increasing order, so with a
 * non-decreasing layer map (the identity by default) they are in plane
 * order, and with any map the hits of one layer are contiguous; their order
 * within a plane is unspecified (the path id, SUPA_OUT_KEYS, is a canonical
 * key).  Nodes: same
 * rule with node_offsets and counts[6*i]; within a segment node j is the one
 * node_parent of its children refers to: the primary is node 0 and the two
 * daughters of a split are consecutive (a first), in the order the splits
 * were processed.
 */
typedef struct supa_output {
    /* hit point clouds (SUPA_OUT_HITS); hit_key also needs SUPA_OUT_KEYS */
    int64_t *hit_offsets;            /* n                                        */
    float *hit_x, *hit_y, *hit_e;    /* hit_capacity each                        */
    int32_t *hit_layer;              /* hit_capacity                             */
    uint64_t *hit_key;               /* hit_capacity, or NULL                    */
    int64_t hit_capacity;
    /* images (SUPA_OUT_IMAGES): n * L * img_ny * img_nx floats, L = 1 + the
       largest layer index; pixel [i][l][iy][ix] sums the energies of the
       shower's hits of layer l with floor((x - x0)*nx/(x1 - x0)) == ix and
       floor((y - y0)*ny/(y1 - y0)) == iy (appendix "Downsampling") */
    float *images;
    /* propagation tree (SUPA_OUT_TREE): per node its parent's index within the
       shower (-1 for the primary), generation (splits since the primary),
       vertex (where it was created) and energy */
    int64_t *node_offsets;           /* n                                        */
    int32_t *node_parent, *node_gen; /* node_capacity each                       */
    float *node_vx, *node_vy, *node_vz, *node_e;
    uint64_t *node_key;              /* node_capacity, or NULL                   */
    int64_t node_capacity;
    /* always written: */
    uint64_t *ledger;                /* n * 4: E0, deposited by stops, deposited
                                        below threshold, escaped (fixed point);
                                        E0 == sum of the other three            */
    int32_t *counts;                 /* n * 6: nodes, hits, particle-steps,
                                        splits, escaped particles, escapes
                                        because the direction turned away from +z */
    /* showers that every per-shower array above holds (ledger, counts,
       hit_offsets, node_offsets, images): a call with n > shower_capacity is
       refused with SUPA_ERR_INVALID_ARG before anything is launched, so the
       library never writes past the caller's per-shower rows */
    int64_t shower_capacity;
    /* host outputs, set on SUPA_OK and on SUPA_ERR_CAPACITY: */
    int64_t total_hits, total_nodes, total_steps;
} supa_output;

/* Version of this ABI (SUPA_ABI_VERSION). */
int32_t supa_abi_version(void);

/* Checks parameters on the host only (no device call): SUPA_OK or
 * SUPA_ERR_INVALID_ARG.  Same checks as supa_init_geometry. */
supa_status supa_validate_geometry(const supa_geometry *g);

/*
 * Checks the arguments of a supa_simulate call on the host only (no device
 * call, no context needed): the same checks supa_simulate makes before it
 * launches anything -- parameters (as supa_validate_geometry), 0 <= n <=
 * 2^31 - 1, the input arrays and every output array the selected outputs
 * need are non-NULL, capacities >= 0 and n <= out->shower_capacity.
 * SUPA_OK or SUPA_ERR_INVALID_ARG (supa_last_error(NULL) says why).
 */
supa_status supa_validate_call(const supa_geometry *g, const supa_batch *b, const supa_output *out);

/*
 * Creates a context for device `device` and HIP stream `hip_stream`
 * (hipStream_t, may be NULL for the default stream).  Validates `g` on the
 * host, derives the integer thresholds, copies them to the device and
 * allocates the library's scratch.  *out receives the context (NULL on error).
 */
supa_status supa_init_geometry(const supa_geometry *g, int device, void *hip_stream,
                               supa_ctx **out);

/* Frees the context and its device scratch (after synchronising its stream). */
supa_status supa_destroy(supa_ctx *ctx);

/*
 * Simulates a batch with 64-bit `seed` (Algorithm 1 applied plane by plane to
 * every live particle of every shower).  Fills `out` as described above.
 * Errors: INVALID_ARG (NULL pointers for requested outputs, bad n, n larger
 * than out->shower_capacity),
 * RANGE (an initial energy out of range: nothing else is meaningful),
 * CAPACITY (total hits or nodes exceed the capacities: ledger, counts and the
 * host totals are valid, hit/node arrays and images are not; a retry with
 * larger arrays gives the same per-shower results), DEVICE.
 */
supa_status supa_simulate(supa_ctx *ctx, const supa_batch *b, uint64_t seed,
                          supa_output *out);

/*
 * k calls in one (a workload whose outputs do not fit one call, run slice
 * by slice): the same as supa_simulate(ctx, &b[j], seed, &out[j]) for j = 0
 * .. k-1, with one synchronisation at the end, and the propagation of call
 * j+1 running on the GPU while the hits, images and tree of call j are
 * placed (the library keeps two sets of logs for the two calls in flight).
 * Sharing: the hit, node and image arrays of different calls may be the
 * same memory (placements run in call order, so a later call overwrites an
 * earlier one's), as may hit_offsets and node_offsets; the ledger and counts
 * rows of consecutive calls must not overlap (refused with INVALID_ARG).
 * Returns OK, or the first RANGE / DEVICE error, else CAPACITY if any call's
 * records exceeded its capacities (out[j].total_* are set for every call);
 * scratch that runs out grows and every call is rerun (bit-identical).
 * supa_last_kernel_times sums the kernel times over the calls.
 */
supa_status supa_simulate_batches(supa_ctx *ctx, int32_t k, const supa_batch *b, uint64_t seed,
                                  supa_output *out);

/*
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, outputs, numerics and errors as supa_simulate, but the library's
 * scratch (particle spill, hit and node logs, per-shower log starts, scan
 * partial sums, work order, image buckets) is carved out of one fixed device
 * array of SUPA_FIXED_SCRATCH_BYTES per GPU -- a static array of the library,
 * resolved once per device by supa_init_geometry and held until the process
 * ends -- and the call makes no hipMalloc, hipFree or other allocation, never
 * grows its scratch and never reruns.  Limits: the per-shower part (8 bytes
 * per shower with hits or images, 4 more with the cost order, plus scan
 * sums) must fit, and the particles a batch leaves pending and the hit and
 * node records it writes must fit the rest; otherwise SUPA_ERR_NOMEM, with
 * nothing meaningful in the outputs (a call of fewer showers, or
 * supa_simulate, then runs it).  Every call on one GPU uses that GPU's one
 * array: calls that overlap in time on the same GPU (any context, stream or
 * thread) race on it and give wrong results.  Calls of supa_simulate do not
 * touch it.
 */
#define SUPA_FIXED_SCRATCH_BYTES (256ull << 20)
supa_status supa_simulate_noalloc(supa_ctx *ctx, const supa_batch *b, uint64_t seed, supa_output *out);

/*
 * Launch settings of the propagation kernel (affect speed only, never
 * results; 0 keeps the current value of a setting).
 *   waves_per_cu  waves launched per compute unit, 1..32 (each wave keeps a
 *                 few showers in flight, taken from the work queue);
 *   frontier_cap  pending particles per wave kept in LDS: 128, 256, 512 or
 *                 1024 (more spill to a per-wave global area);
 *   hit_cap, node_cap  sizes (records) of the library's hit and node logs,
 *                 where the propagation kernel leaves hits and nodes before
 *                 they are placed into the output arrays (default: sized
 *                 from the output capacities).
 * The spill area and the logs grow by themselves (and the batch is rerun)
 * when a batch needs more.
 */
supa_status supa_set_launch(supa_ctx *ctx, int32_t waves_per_cu, int32_t frontier_cap,
                            int32_t hit_cap, int32_t node_cap);

/*
 * Scheduling of supa_simulate (affects speed only, never results).
 *   sub_batches  the batch runs as this many consecutive sub-batches, and the
 *                placement of the hits, nodes and images of one (on a second,
 *                library-owned stream) overlaps the propagation of the next.
 *                0 (default) = 1; 1..8 = that many (never more than n).
 *                Counts-only calls use one.
 *   cost_order   1: showers are handed to the propagation kernel most
 *                expensive first (expected cost grows with E0; a device
 *                counting sort on log2 of the fixed-point energy), so the
 *                end of a launch is filled with cheap showers; 0: batch
 *                order; -1 (default): automatic.
 */
supa_status supa_set_schedule(supa_ctx *ctx, int32_t sub_batches, int32_t cost_order);

/*
 * Subtree work items (affect speed only, never results; section "Propagation
 * Model": a particle's further history depends only on its own state, its
 * plane and its path id, not on the rest of its shower, so any wave can
 * finish it).  With phases > 1 a call runs that many propagation launches on
 * its stream.  In every launch but the last, a wave whose pool of pending
 * particles holds export_pool + 64 or more entries takes its 64 oldest, and
 * those of the shower with most of them (at least 16) leave the wave as one
 * item; the next launch hands the items out to all its waves.  The shower
 * then becomes shared: a device record collects the tallies of every party
 * working on it, the last party to finish writes its ledger and counts, its
 * hit records continue one run of the hit log (chunks reserved for it when
 * it is shared), and with a tree its node indices are taken from a shared
 * counter, so node numbering and the order of records within a plane may
 * differ from a call without items (the sets are the same).  Showers of a
 * small batch then spread over all waves instead of the few that started
 * them.  A wave exports only once its claim for new showers has come back
 * empty (while showers remain to be started every wave is busy anyway).
 *   phases       0 (default): automatic -- 2 when the batch's showers all
 *                start at once on at most a quarter of the waves (4 n <= the
 *                waves launched), the kinematics are plain and no sub-batches
 *                are asked for, else 1; 1: no items; 2 .. 4: that many
 *                launches;
 *   export_pool  pending particles beyond one step (64) from which a wave
 *                exports (default 0: every wave with 64 or more).
 * Items need the plain kinematics without regional parameters (INVALID_ARG
 * for phases > 1 otherwise; automatic then means 1).  A call with items runs
 * as one sub-batch; supa_simulate_noalloc decides automatic as 1.  Items and shared
 * showers are bounded per call (16,384 each; 1,024 with
 * supa_simulate_noalloc); beyond that waves keep their particles.  A shared
 * shower whose hits outgrow the reserve is rerun with a larger one
 * (bit-identical sets; SUPA_ERR_NOMEM from supa_simulate_noalloc).
 */
supa_status supa_set_subtrees(supa_ctx *ctx, int32_t phases, int32_t export_pool);

/*
 * Subtree work items of the context's last supa_simulate or
 * supa_simulate_noalloc call (or the last supa_graph_check): counts5 (host,
 * 5 int64) receives the showers that became shared, then the items exported
 * by launches 0 .. 3.  All zero without items.
 */
supa_status supa_last_subtrees(const supa_ctx *ctx, int64_t *counts5);

/*
 * Picks launch settings by measurement: runs the batch under every
 * combination of waves per CU {8, 12, 16}, LDS pool {128, 256} entries,
 * sub-batches {1, 2} and cost order {0, 1} (each twice: warm-up, then timed
 * with the context's events) and keeps the fastest whole call in the
 * context.  Same arguments and errors as supa_simulate; `out` holds the
 * batch's results afterwards.  best (host, 4 int32) receives waves_per_cu,
 * frontier_cap, sub_batches, cost_order; best_ms (host) the fastest time.
 * The choice is kept in the context (whose geometry and device are fixed)
 * per batch size: a later supa_autotune of a batch of the same size applies
 * it and makes one call, without searching again.  supa_autotune_forget
 * clears what the context keeps.
 */
supa_status supa_autotune(supa_ctx *ctx, const supa_batch *b, uint64_t seed, supa_output *out,
                          int32_t *best, float *best_ms);
supa_status supa_autotune_forget(supa_ctx *ctx);

/*
 * Captured calls (HIP graphs).  supa_graph_create runs supa_simulate once on
 * the batch (sizing the library's scratch and checking the capacities), then
 * captures the launch sequence of that call -- counters cleared, work order,
 * propagation, offsets, placement, images, tree -- as one HIP graph with no
 * host work, no allocation and no memset nodes.  The graph keeps the batch and
 * output pointers of `b` and `out`; replays recompute the outputs from the
 * current contents of the input arrays (so new initial conditions of the same
 * count can be written in place between replays).
 *   supa_graph_launch  enqueues one replay on hip_stream (NULL = the
 *                      context's stream); nothing is synchronised.
 *   supa_graph_check   synchronises hip_stream and reads the replay's
 *                      counters: OK, RANGE, CAPACITY (outputs or library
 *                      scratch too small for this replay: its results are not
 *                      valid), DEVICE; totals3 (host, may be NULL) receives
 *                      total hits, nodes, steps.
 *   supa_graph_destroy frees the graph.
 * A graph shares the context's counters and scratch: replays and other calls
 * on one context must not overlap in time.  A later call on the context that
 * needs more scratch than the capture's (a larger batch, more hits or nodes,
 * other launch settings) reallocates it; the graph is then stale, and
 * supa_graph_launch and supa_graph_check return SUPA_ERR_STATE without
 * launching anything: capture it again.
 */
typedef struct supa_graph supa_graph;
supa_status supa_graph_create(supa_ctx *ctx, const supa_batch *b, uint64_t seed, supa_output *out,
                              supa_graph **graph);
supa_status supa_graph_launch(supa_graph *graph, void *hip_stream);
supa_status supa_graph_check(supa_graph *graph, void *hip_stream, int64_t *totals3);
supa_status supa_graph_destroy(supa_graph *graph);

/*
 * Device time of the last supa_simulate, in milliseconds, measured with HIP
 * events: [0] propagation kernels (summed over sub-batches), [1] placement
 * of hits, images and nodes (summed; with sub-batches they overlap [0]),
 * [2] whole call (including work ordering and segment offsets).  Host
 * pointer to 3 floats.
 */
supa_status supa_last_timing(const supa_ctx *ctx, float *ms3);

/*
 * The same device times split by kernel: ms[0] propagation, [1] placement
 * and node scatter, [2] whole call, [3] hit / image placement kernel alone,
 * [4] node scatter kernel alone (each summed over sub-batches; 0 for parts
 * the call does not run).  Host pointer to `count` floats; entries past the
 * fifth are set to 0.
 */
supa_status supa_last_kernel_times(const supa_ctx *ctx, float *ms, int32_t count);

/*
 * How evenly the last propagation launch of the context kept its waves busy:
 * ms[q] (host, up to `capacity` entries) = the time wave q spent from its
 * start to its exit, on the device's constant-rate clock; *count (host) =
 * the waves that launch had.  The launch is that of the last supa_simulate,
 * supa_simulate_noalloc, graph replay, or the last call of
 * supa_simulate_batches (the last sub-batch with sub-batches).  Synchronises
 * the context's stream.
 */
supa_status supa_last_wave_times(supa_ctx *ctx, float *ms, int32_t capacity, int32_t *count);

/*
 * One Philox4x32-10 block per counter, on the device: ctr and out are device
 * arrays of 4*n uint32 (counter words c0..c3 / output words w0..w3).  For
 * checking the device generator against independent implementations.
 */
supa_status supa_philox(supa_ctx *ctx, const uint32_t *ctr, int64_t n, uint64_t key,
                        uint32_t *out);

/*
 * The sine and cosine of a split's azimuth omega = 2 pi u(w3), u(w) =
 * (w + 1/2) / 2^32 (Algorithm 1's uniform angle of the split plane), as the
 * propagation kernel evaluates them, for n words: w device uint32 [n],
 * sin_out and cos_out device float [n].  For checking them against the
 * definition.  INVALID_ARG for n < 0 or NULL arrays with n > 0.
 */
supa_status supa_azimuth(supa_ctx *ctx, const uint32_t *w, int64_t n, float *sin_out, float *cos_out);

/* Description of the last error of ctx (or of the last failed
 * supa_init_geometry when ctx is NULL); owned by the library. */
const char *supa_last_error(const supa_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
