// supa_api.hip -- host side of the C ABI declared in include/supa.h.
//
// Validates parameters on the host, derives the integer thresholds of the
// three-way choice and of the energy split, keeps their device copies and the
// per-wave scratch of the propagation kernel, and launches it on the caller's
// stream.  Scratch grows (and the batch is rerun, which the counter-based
// randomness makes bit-identical) when a shower needs more than it holds.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/supa.h"
#include "supa_device.hpp"

namespace supa {
hipError_t launch_zero_counters(unsigned long long *ctr, hipStream_t s);
hipError_t launch_note_chunks(const unsigned long long *ctr, unsigned long long *sub, hipStream_t s);
hipError_t launch_propagate(const Params &P, bool literal, bool rings, int blocks, hipStream_t s);
hipError_t launch_philox(const uint32_t *ctr, int64_t n, uint32_t k0, uint32_t k1, uint32_t *out,
                         hipStream_t s);
hipError_t launch_azimuth(const uint32_t *w, int64_t n, float *sn, float *cs, hipStream_t s);
size_t propagate_lds_bytes(int pool_cap, bool rings);
hipError_t launch_place(const PlaceParams &P, int n_cu, hipStream_t s);
void place_bucket_size(int L, int nx, int ny, bool keys, int n_cu, int64_t *per_block, int64_t *blocks);
int64_t scan_partial_words(int64_t n);
hipError_t launch_scan(const ScanParams &S, hipStream_t s);
hipError_t launch_scatter_nodes(const ScatterParams &Q, int32_t n, int n_cu, hipStream_t s);
int64_t order_scratch_words();
hipError_t launch_cost_order(const float *e0, int n, float e_scale, uint32_t *hist, int32_t *order,
                             int n_cu, hipStream_t s);
}  // namespace supa

// A device buffer that only grows (its contents are scratch).  Every
// reallocation advances *gen, so that a captured graph holding the old
// address can tell that it is stale.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    bool ensure(size_t need, uint64_t *gen) {
        if (need <= bytes) return true;
        ++*gen;
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
        if (hipMalloc(&p, need) != hipSuccess) {
            (void)hipGetLastError();
            return false;
        }
        bytes = need;
        return true;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
};

static constexpr int kMaxImageWidth = 1024;
// subtree work items: items per launch phase and shared showers per call
// (context scratch; the fixed array holds fewer).  When they run out, waves
// stop exporting and finish their showers themselves.
static constexpr int kItemCap = 16384, kShareCap = 16384;
static constexpr int kFixedItemCap = 1024, kFixedShareCap = 1024;
static constexpr int64_t kAutoOrderMin = 65536;     // automatic cost order: from this batch size

// Scratch of supa_simulate_noalloc: one fixed array per GPU, held from the
// library's first use of a device until the process ends.  Host code never
// passes `scratch` itself to a kernel (on the host it is only a stand-in for
// the symbol): it uses the device address resolved once per device below.
static constexpr size_t kFixedBytes = SUPA_FIXED_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kFixedBytes];
static constexpr int kMaxDevices = 64;
static std::mutex g_fixed_mu;
static void *g_fixed[kMaxDevices];

// The device address of `device`'s copy of the fixed array; the device must
// be current.  Resolved on the first call for a device, then reused.
static hipError_t fixed_scratch(int device, void **ptr) {
    *ptr = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_fixed_mu);
    if (!g_fixed[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_fixed[device] = p;
    }
    *ptr = g_fixed[device];
    return hipSuccess;
}

// threshold table: 4 rings x 64 planes (the propagation kernel's layout)
constexpr int THR_ENTRIES = 4 * 64;

struct supa_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    supa_geometry g{};                 // host copy (array pointers cleared)
    std::vector<int32_t> layer;        // host copies
    std::vector<double> p_stop, p_split;
    float ring_r[4] = {0.f, 0.f, 0.f, 0.f};   // ring radii, +inf past the last
    int32_t n_layers = 0;
    // derived constants
    uint64_t t_cut = 0;
    uint32_t f_lo = 0;
    uint64_t f_w = 0;
    // device copies
    int32_t *d_layer = nullptr;
    int32_t *d_layer_plane_start = nullptr, *d_layer_planes = nullptr;
    uint64_t *d_c1 = nullptr, *d_c2 = nullptr;
    unsigned long long *d_ctr = nullptr;
    unsigned long long *h_ctr = nullptr;   // pinned
    supa::Cold *d_cold = nullptr;          // per-sub-batch inputs/outputs blocks (device)
    supa::Cold *h_cold = nullptr;          // their pinned host staging copy
    // launch settings and scratch
    int n_cu = 0;
    int waves_per_cu = 16;
    int pool_cap = 128;                  // particle-pool entries kept in LDS
    int spill_cap = 4096;                // per-wave spill entries
    int64_t h_chunks = 0, n_chunks = 0;  // log chunks (grow on demand)
    int sub_batches = 0;                 // 0: chosen from the batch size
    int cost_order = -1;                 // hand out expensive showers first: 1 on, 0 off, -1 auto
    // subtree work items: propagation launches per call (1: none), the pool
    // size beyond one step from which a wave exports, the reserve of hit-log
    // chunks per shared shower relative to its expected hits
    int phases = 0;                      // 0: automatic
    int export_top = 0;
    float share_margin = 1.5f;
    DevBuf items, shares;
    int64_t last_item_cap = 0, last_share_cap = 0;   // of the last prepared call
    int last_sub_batches = 0;
    DevBuf spill, hlog, nlog, shower, bucket;
    // second set of the buffers that the propagation of one call writes while
    // the placement of the previous call reads them (supa_simulate_batches)
    DevBuf hlog2, nlog2, hstart2;
    DevBuf snap;                         // per-call copies of the counters (batches)
    unsigned long long *h_snap = nullptr;    // pinned host copy of snap
    size_t h_snap_bytes = 0;
    supa::Cold *h_calls = nullptr;       // pinned per-call input/output blocks (batches)
    size_t h_calls_n = 0;
    DevBuf d_calls;
    std::vector<hipEvent_t> call_ev;     // 5 per call: propagation start/end, scan done,
                                         // placement end, node scatter end (batches)
    hipEvent_t ev_set_free[2] = {};      // second stream done with a set of buffers
    uint64_t scratch_gen = 0;            // advanced by every scratch reallocation
    char *fixed = nullptr;               // this device's fixed scratch array (device address)
    unsigned long long *d_wclk = nullptr;   // per wave of the last propagation launch: start, end
    int64_t last_waves = 0;
    // launch settings picked by supa_autotune, per batch size
    struct Tuned {
        int64_t n;
        int32_t best[4];
        float ms;
    };
    std::vector<Tuned> tuned;
    // the placement of a sub-batch runs on a second stream, overlapping the
    // propagation of the next one
    hipStream_t aux = nullptr;
    hipEvent_t ev_begin = nullptr, ev_end = nullptr, ev_joined = nullptr;
    hipEvent_t ev_prop[supa::MAX_SUB][2] = {};    // propagation start / end (stream)
    hipEvent_t ev_post[supa::MAX_SUB][2] = {};    // placement start / end (aux)
    hipEvent_t ev_place[supa::MAX_SUB] = {};      // end of the hit / image placement (aux)
    // propagation, placement + node scatter, whole call, placement alone,
    // node scatter alone (ms, summed over sub-batches)
    float timing[5] = {0, 0, 0, 0, 0};
    std::string err;
    bool broken = false;
};

static std::string g_init_error;

static supa_status fail(supa_ctx *c, supa_status s, const std::string &msg) {
    if (c) c->err = msg; else g_init_error = msg;
    return s;
}

static supa_status hip_fail(supa_ctx *c, hipError_t e, const char *what) {
    if (c) c->broken = true;
    return fail(c, SUPA_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(c, call)                                 \
    do {                                                 \
        hipError_t e_ = (call);                          \
        if (e_ != hipSuccess) return hip_fail(c, e_, #call); \
    } while (0)

extern "C" int32_t supa_abi_version(void) { return SUPA_ABI_VERSION; }

static bool is_fin(double v) { return std::isfinite(v); }

static supa_status validate(const supa_geometry *g, std::string &why) {
    if (!g) { why = "geometry is NULL"; return SUPA_ERR_INVALID_ARG; }
    if (g->n_planes < 1 || g->n_planes > 63) { why = "n_planes must be in [1, 63]"; return SUPA_ERR_INVALID_ARG; }
    if (!is_fin(g->z_first) || !is_fin(g->dz) || !(g->dz > 0) || !(g->z_first > 0)) {
        why = "z_first and dz must be finite and > 0";
        return SUPA_ERR_INVALID_ARG;
    }
    if (!is_fin(g->e_cut) || !(g->e_cut >= 0)) { why = "e_cut must be finite and >= 0"; return SUPA_ERR_INVALID_ARG; }
    if (g->angle_mode < SUPA_ANGLE_FIXED || g->angle_mode > SUPA_ANGLE_RAYLEIGH) {
        why = "unknown angle_mode";
        return SUPA_ERR_INVALID_ARG;
    }
    if (!is_fin(g->angle_a) || !is_fin(g->angle_b)) { why = "angles must be finite"; return SUPA_ERR_INVALID_ARG; }
    if (g->kinematics != SUPA_KIN_3D && g->kinematics != SUPA_KIN_LITERAL) {
        why = "unknown kinematics";
        return SUPA_ERR_INVALID_ARG;
    }
    if (!(g->frac_lo >= 0 && g->frac_lo <= g->frac_hi && g->frac_hi <= 1)) {
        why = "need 0 <= frac_lo <= frac_hi <= 1";
        return SUPA_ERR_INVALID_ARG;
    }
    if (g->energy_frac_bits < 0 || g->energy_frac_bits > 31) {
        why = "energy_frac_bits must be in [0, 31]";
        return SUPA_ERR_INVALID_ARG;
    }
    if (g->n_regions < 0 || g->n_regions > 4) { why = "n_regions must be in [0, 4]"; return SUPA_ERR_INVALID_ARG; }
    const int rings = g->n_regions >= 2 ? g->n_regions : 1;
    if (rings >= 2) {
        if (!g->region_r) { why = "region_r is NULL"; return SUPA_ERR_INVALID_ARG; }
        for (int b = 0; b < rings - 1; ++b)
            if (!is_fin(g->region_r[b]) || !(g->region_r[b] > 0) || (b > 0 && !(g->region_r[b] > g->region_r[b - 1]))) {
                why = "region_r must be finite, > 0 and ascending";
                return SUPA_ERR_INVALID_ARG;
            }
    }
    for (int j = 0; j < rings * g->n_planes; ++j) {
        const double ps = g->p_stop ? g->p_stop[j] : 0.0;
        const double pl = g->p_split ? g->p_split[j] : 1.0;
        if (!(ps >= 0 && pl >= 0 && ps + pl <= 1)) {
            why = "need p_stop, p_split >= 0 and p_stop + p_split <= 1 on every plane";
            return SUPA_ERR_INVALID_ARG;
        }
    }
    for (int k = 0; k < g->n_planes; ++k) {
        if (g->layer_of_plane && (g->layer_of_plane[k] < -1 || g->layer_of_plane[k] >= g->n_planes)) {
            why = "layer_of_plane entries must be in [-1, n_planes)";
            return SUPA_ERR_INVALID_ARG;
        }
    }
    if (g->outputs & ~15u) { why = "unknown output bits"; return SUPA_ERR_INVALID_ARG; }
    if (g->outputs & SUPA_OUT_IMAGES) {
        if (g->img_nx < 1 || g->img_ny < 1 || g->img_nx > kMaxImageWidth) {
            why = "image grid must have 1 <= nx <= 1024 and ny >= 1";
            return SUPA_ERR_INVALID_ARG;
        }
        if (!is_fin(g->img_x0) || !is_fin(g->img_x1) || !is_fin(g->img_y0) || !is_fin(g->img_y1) ||
            !(g->img_x1 > g->img_x0) || !(g->img_y1 > g->img_y0)) {
            why = "image window must be finite with x1 > x0 and y1 > y0";
            return SUPA_ERR_INVALID_ARG;
        }
    }
    return SUPA_OK;
}

extern "C" supa_status supa_validate_geometry(const supa_geometry *g) {
    std::string why;
    supa_status s = validate(g, why);
    if (s != SUPA_OK) g_init_error = why;
    return s;
}

// hit-log chunks that hold `records` records for `waves` waves: full chunks,
// plus the partly filled chunk every shower slot may leave at the end
static int64_t hit_chunks_for(int64_t records, int64_t waves) {
    return (records + supa::HIT_CHUNK - 1) / supa::HIT_CHUNK + waves * supa::SLOTS + 8;
}

// node-log chunks: a closed chunk may leave up to 127 records unused (a
// phase appends at most 2 per lane), plus one open chunk per wave
static int64_t node_chunks_for(int64_t records, int64_t waves) {
    const int64_t per = supa::LOG_CHUNK - 127;
    return (records + per - 1) / per + waves + 8;
}

static supa_status nomem(supa_ctx *c, const char *what, size_t bytes) {
    return fail(c, SUPA_ERR_NOMEM, std::string("cannot allocate ") + std::to_string(bytes) +
                                       " bytes of " + what);
}

extern "C" supa_status supa_init_geometry(const supa_geometry *g, int device, void *hip_stream,
                                          supa_ctx **out) {
    if (!out) return fail(nullptr, SUPA_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    std::string why;
    supa_status s = validate(g, why);
    if (s != SUPA_OK) return fail(nullptr, s, why);

    supa_ctx *c = new supa_ctx();
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    c->g = *g;
    const int N = g->n_planes;
    const int rings = g->n_regions >= 2 ? g->n_regions : 1;
    c->layer.resize(N);
    c->p_stop.resize((size_t)rings * N);
    c->p_split.resize((size_t)rings * N);
    int32_t max_layer = -1;
    for (int k = 0; k < N; ++k) {
        c->layer[k] = g->layer_of_plane ? g->layer_of_plane[k] : k;
        max_layer = std::max(max_layer, c->layer[k]);
    }
    for (int j = 0; j < rings * N; ++j) {
        c->p_stop[j] = g->p_stop ? g->p_stop[j] : 0.0;
        c->p_split[j] = g->p_split ? g->p_split[j] : 1.0;
    }
    for (int b = 0; b < 4; ++b)
        c->ring_r[b] = b < rings - 1 ? (float)g->region_r[b] : __builtin_inff();
    c->n_layers = max_layer + 1;
    // planes of each layer, as a CSR list (layers need not be contiguous)
    std::vector<int32_t> lps(c->n_layers + 1, 0), lp;
    for (int l = 0; l < c->n_layers; ++l) {
        for (int k = 0; k < N; ++k)
            if (c->layer[k] == l) lp.push_back(k);
        lps[l + 1] = (int32_t)lp.size();
    }
    if (lp.empty()) lp.push_back(0);
    c->g.layer_of_plane = nullptr;
    c->g.p_stop = nullptr;
    c->g.p_split = nullptr;
    c->g.region_r = nullptr;

    // integer thresholds: stop iff w0 < C1, split iff C1 <= w0 < C2; entry
    // ring * 64 + plane (4 rings of 64 planes, unused entries 0)
    std::vector<uint64_t> c1(THR_ENTRIES, 0), c2(THR_ENTRIES, 0);
    for (int j = 0; j < rings; ++j)
        for (int k = 0; k < N; ++k) {
            c1[j * 64 + k] = (uint64_t)std::floor(std::ldexp(c->p_stop[j * N + k], 32));
            c2[j * 64 + k] = c1[j * 64 + k] + (uint64_t)std::floor(std::ldexp(c->p_split[j * N + k], 32));
        }
    const double tc = std::ceil(std::ldexp(g->e_cut, g->energy_frac_bits));
    c->t_cut = tc >= 18446744073709551615.0 ? ~0ull : (uint64_t)tc;
    c->f_lo = (uint32_t)std::min(std::floor(std::ldexp(g->frac_lo, 32)), 4294967295.0);
    c->f_w = (uint64_t)std::floor(std::ldexp(g->frac_hi, 32)) - (uint64_t)std::floor(std::ldexp(g->frac_lo, 32));

    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) { delete c; return hip_fail(nullptr, e, "hipSetDevice"); }
    if (hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
        c->n_cu <= 0) {
        delete c;
        return fail(nullptr, SUPA_ERR_DEVICE, "cannot query compute units");
    }
    void *fx = nullptr;
    e = fixed_scratch(device, &fx);
    if (e != hipSuccess) {
        delete c;
        return hip_fail(nullptr, e, "hipGetSymbolAddress of the fixed scratch array");
    }
    c->fixed = (char *)fx;
    bool ok = hipMalloc(&c->d_layer, N * sizeof(int32_t)) == hipSuccess &&
              hipMalloc(&c->d_c1, THR_ENTRIES * sizeof(uint64_t)) == hipSuccess &&
              hipMalloc(&c->d_layer_plane_start, lps.size() * sizeof(int32_t)) == hipSuccess &&
              hipMalloc(&c->d_layer_planes, lp.size() * sizeof(int32_t)) == hipSuccess &&
              hipMemcpy(c->d_layer_plane_start, lps.data(), lps.size() * sizeof(int32_t),
                        hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(c->d_layer_planes, lp.data(), lp.size() * sizeof(int32_t),
                        hipMemcpyHostToDevice) == hipSuccess &&
              hipMalloc(&c->d_c2, THR_ENTRIES * sizeof(uint64_t)) == hipSuccess &&
              hipMalloc(&c->d_ctr, 2 * supa::CTR_WORDS * sizeof(unsigned long long)) == hipSuccess &&
              hipHostMalloc(&c->h_ctr, supa::CTR_WORDS * sizeof(unsigned long long), 0) == hipSuccess &&
              hipMalloc(&c->d_cold, supa::MAX_SUB * sizeof(supa::Cold)) == hipSuccess &&
              hipMalloc(&c->d_wclk, (size_t)2 * 32 * c->n_cu * sizeof(unsigned long long)) == hipSuccess &&
              hipHostMalloc(&c->h_cold, supa::MAX_SUB * sizeof(supa::Cold), 0) == hipSuccess &&
              hipMemcpy(c->d_layer, c->layer.data(), N * sizeof(int32_t), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(c->d_c1, c1.data(), THR_ENTRIES * sizeof(uint64_t), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(c->d_c2, c2.data(), THR_ENTRIES * sizeof(uint64_t), hipMemcpyHostToDevice) == hipSuccess;
    // default priority, and no implicit synchronisation with the null stream
    ok = ok && hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking) == hipSuccess;
    for (hipEvent_t *e : {&c->ev_begin, &c->ev_end, &c->ev_joined})
        ok = ok && hipEventCreate(e) == hipSuccess;
    for (int b = 0; b < supa::MAX_SUB && ok; ++b)
        for (int q = 0; q < 2 && ok; ++q)
            ok = hipEventCreate(&c->ev_prop[b][q]) == hipSuccess && hipEventCreate(&c->ev_post[b][q]) == hipSuccess;
    for (int b = 0; b < supa::MAX_SUB && ok; ++b) ok = hipEventCreate(&c->ev_place[b]) == hipSuccess;
    for (int q = 0; q < 2 && ok; ++q) ok = hipEventCreate(&c->ev_set_free[q]) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        supa_destroy(c);
        return fail(nullptr, SUPA_ERR_DEVICE, "device allocation or copy failed in init");
    }
    *out = c;
    return SUPA_OK;
}

extern "C" supa_status supa_destroy(supa_ctx *c) {
    if (!c) return SUPA_ERR_STATE;
    (void)hipSetDevice(c->device);
    // both streams drain before their scratch is freed (a null stream is
    // the default stream, also synchronised)
    (void)hipStreamSynchronize(c->stream);
    if (c->aux) (void)hipStreamSynchronize(c->aux);
    for (DevBuf *d : {&c->spill, &c->hlog, &c->nlog, &c->shower, &c->bucket, &c->hlog2, &c->nlog2, &c->hstart2,
                      &c->snap, &c->d_calls, &c->items, &c->shares})
        d->release();
    if (c->h_snap) (void)hipHostFree(c->h_snap);
    if (c->h_calls) (void)hipHostFree(c->h_calls);
    for (hipEvent_t e : c->call_ev)
        if (e) (void)hipEventDestroy(e);
    for (int q = 0; q < 2; ++q)
        if (c->ev_set_free[q]) (void)hipEventDestroy(c->ev_set_free[q]);
    if (c->d_layer) (void)hipFree(c->d_layer);
    if (c->d_layer_plane_start) (void)hipFree(c->d_layer_plane_start);
    if (c->d_layer_planes) (void)hipFree(c->d_layer_planes);
    if (c->d_c1) (void)hipFree(c->d_c1);
    if (c->d_c2) (void)hipFree(c->d_c2);
    if (c->d_ctr) (void)hipFree(c->d_ctr);
    if (c->h_ctr) (void)hipHostFree(c->h_ctr);
    if (c->d_cold) (void)hipFree(c->d_cold);
    if (c->d_wclk) (void)hipFree(c->d_wclk);
    if (c->h_cold) (void)hipHostFree(c->h_cold);
    for (hipEvent_t e : {c->ev_begin, c->ev_end, c->ev_joined})
        if (e) (void)hipEventDestroy(e);
    for (int b = 0; b < supa::MAX_SUB; ++b)
        for (int q = 0; q < 2; ++q) {
            if (c->ev_prop[b][q]) (void)hipEventDestroy(c->ev_prop[b][q]);
            if (c->ev_post[b][q]) (void)hipEventDestroy(c->ev_post[b][q]);
        }
    for (int b = 0; b < supa::MAX_SUB; ++b)
        if (c->ev_place[b]) (void)hipEventDestroy(c->ev_place[b]);
    if (c->aux) (void)hipStreamDestroy(c->aux);
    delete c;
    return SUPA_OK;
}

extern "C" supa_status supa_set_launch(supa_ctx *c, int32_t waves_per_cu, int32_t frontier_cap,
                                       int32_t hit_cap, int32_t node_cap) {
    if (!c) return SUPA_ERR_STATE;
    const bool pow2 = frontier_cap == 0 || (frontier_cap & (frontier_cap - 1)) == 0;
    if (waves_per_cu < 0 || waves_per_cu > 32 || frontier_cap < 0 || frontier_cap > 1024 ||
        (frontier_cap != 0 && frontier_cap < 128) || !pow2 || hit_cap < 0 || node_cap < 0)
        return fail(c, SUPA_ERR_INVALID_ARG, "launch settings out of range");
    if (waves_per_cu) c->waves_per_cu = waves_per_cu;
    if (frontier_cap) c->pool_cap = frontier_cap;
    // initial log sizes in records (the logs grow by themselves when a batch
    // needs more; small values exercise that path)
    if (hit_cap) c->h_chunks = std::max<int64_t>(1, (hit_cap + supa::HIT_CHUNK - 1) / supa::HIT_CHUNK);
    if (node_cap) c->n_chunks = std::max<int64_t>(1, (node_cap + supa::LOG_CHUNK - 1) / supa::LOG_CHUNK);
    return SUPA_OK;
}

extern "C" supa_status supa_set_schedule(supa_ctx *c, int32_t sub_batches, int32_t cost_order) {
    if (!c) return SUPA_ERR_STATE;
    if (sub_batches < 0 || sub_batches > supa::MAX_SUB)
        return fail(c, SUPA_ERR_INVALID_ARG, "sub_batches must be in [0, 8]");
    if (cost_order < -1 || cost_order > 1) return fail(c, SUPA_ERR_INVALID_ARG, "cost_order must be -1, 0 or 1");
    c->sub_batches = sub_batches;
    c->cost_order = cost_order;
    return SUPA_OK;
}

extern "C" supa_status supa_set_subtrees(supa_ctx *c, int32_t phases, int32_t export_pool) {
    if (!c) return SUPA_ERR_STATE;
    if (phases < 0 || phases > supa::MAX_PHASES)
        return fail(c, SUPA_ERR_INVALID_ARG, "phases must be in [0, " + std::to_string(supa::MAX_PHASES) + "]");
    if (export_pool < 0 || export_pool > 1 << 20)
        return fail(c, SUPA_ERR_INVALID_ARG, "export_pool must be in [0, 2^20]");
    if (phases > 1 && (c->g.kinematics == SUPA_KIN_LITERAL || c->g.n_regions >= 2))
        return fail(c, SUPA_ERR_INVALID_ARG, "subtree work items need the plain kinematics without regional parameters");
    c->phases = phases;
    c->export_top = export_pool;
    return SUPA_OK;
}

extern "C" supa_status supa_last_subtrees(const supa_ctx *c, int64_t *counts5) {
    if (!c) return SUPA_ERR_STATE;
    if (!counts5) return SUPA_ERR_INVALID_ARG;
    counts5[0] = std::min<int64_t>((int64_t)c->h_ctr[supa::CTR_ST_SHARES], c->last_share_cap);
    for (int p = 0; p < supa::MAX_PHASES; ++p)
        counts5[1 + p] = std::min<int64_t>((int64_t)c->h_ctr[supa::ctr_st_out(p)], c->last_item_cap);
    return SUPA_OK;
}

extern "C" supa_status supa_last_timing(const supa_ctx *c, float *ms3) {
    if (!c) return SUPA_ERR_STATE;
    if (!ms3) return SUPA_ERR_INVALID_ARG;
    std::memcpy(ms3, c->timing, 3 * sizeof(float));
    return SUPA_OK;
}

extern "C" supa_status supa_last_kernel_times(const supa_ctx *c, float *ms, int32_t count) {
    if (!c) return SUPA_ERR_STATE;
    if (!ms || count < 0) return SUPA_ERR_INVALID_ARG;
    const int m = std::min<int>(count, 5);
    std::memcpy(ms, c->timing, (size_t)m * sizeof(float));
    for (int q = m; q < count; ++q) ms[q] = 0.0f;
    return SUPA_OK;
}

extern "C" supa_status supa_last_wave_times(supa_ctx *c, float *ms, int32_t capacity, int32_t *count) {
    if (!c) return SUPA_ERR_STATE;
    if (!count || capacity < 0 || (capacity > 0 && !ms)) return fail(c, SUPA_ERR_INVALID_ARG, "bad wave-time arguments");
    const int64_t w = std::min<int64_t>(c->last_waves, (int64_t)32 * c->n_cu);
    *count = (int32_t)w;
    if (w == 0 || capacity == 0) return SUPA_OK;
    std::vector<unsigned long long> t((size_t)2 * w);
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    HIP_TRY(c, hipMemcpy(t.data(), c->d_wclk, t.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost));
    int rate_khz = 0;
    HIP_TRY(c, hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, c->device));
    const double to_ms = rate_khz > 0 ? 1.0 / rate_khz : 0.0;
    for (int64_t q = 0; q < std::min<int64_t>(w, capacity); ++q)
        ms[q] = (float)((double)(t[2 * q + 1] - t[2 * q]) * to_ms);
    return SUPA_OK;
}

extern "C" const char *supa_last_error(const supa_ctx *c) {
    return c ? c->err.c_str() : g_init_error.c_str();
}

extern "C" supa_status supa_philox(supa_ctx *c, const uint32_t *ctr, int64_t n, uint64_t key,
                                   uint32_t *out) {
    if (!c) return SUPA_ERR_STATE;
    if (n < 0 || (n > 0 && (!ctr || !out))) return fail(c, SUPA_ERR_INVALID_ARG, "bad philox arguments");
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, supa::launch_philox(ctr, n, (uint32_t)key, (uint32_t)(key >> 32), out, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return SUPA_OK;
}

extern "C" supa_status supa_azimuth(supa_ctx *c, const uint32_t *w, int64_t n, float *sin_out,
                                    float *cos_out) {
    if (!c) return SUPA_ERR_STATE;
    if (n < 0 || (n > 0 && (!w || !sin_out || !cos_out)))
        return fail(c, SUPA_ERR_INVALID_ARG, "bad azimuth arguments");
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, supa::launch_azimuth(w, n, sin_out, cos_out, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return SUPA_OK;
}

static int64_t round_up_pow2(int64_t v) {
    int64_t p = 64;
    while (p < v) p <<= 1;
    return p;
}

// Argument checks of a simulate call against the selected outputs (host
// only): SUPA_OK or SUPA_ERR_INVALID_ARG with the reason in `why`.
static supa_status check_args(uint32_t outs, const supa_batch *b, const supa_output *out, std::string &why) {
    if (!b || !out) { why = "batch or output is NULL"; return SUPA_ERR_INVALID_ARG; }
    if (b->n < 0 || b->n > 2147483647LL) { why = "n out of range"; return SUPA_ERR_INVALID_ARG; }
    const int64_t n = b->n;
    if (n == 0) return SUPA_OK;
    // every per-shower row the call writes must lie inside the caller's arrays
    if (out->shower_capacity < n) {
        why = "outputs hold " + std::to_string(out->shower_capacity) + " showers (shower_capacity), the batch has " +
              std::to_string(n);
        return SUPA_ERR_INVALID_ARG;
    }
    if (!b->e0 || !b->polar || !b->azimuth) { why = "e0, polar and azimuth are required"; return SUPA_ERR_INVALID_ARG; }
    if (!out->ledger || !out->counts) { why = "ledger and counts are required"; return SUPA_ERR_INVALID_ARG; }
    if ((outs & SUPA_OUT_HITS) &&
        (!out->hit_offsets || ((!out->hit_x || !out->hit_y || !out->hit_e || !out->hit_layer) && out->hit_capacity > 0) ||
         out->hit_capacity < 0 || ((outs & SUPA_OUT_KEYS) && out->hit_capacity > 0 && !out->hit_key))) {
        why = "hit outputs missing";
        return SUPA_ERR_INVALID_ARG;
    }
    if ((outs & SUPA_OUT_IMAGES) && !out->images) { why = "images missing"; return SUPA_ERR_INVALID_ARG; }
    if ((outs & SUPA_OUT_TREE) &&
        (!out->node_offsets || out->node_capacity < 0 ||
         ((!out->node_parent || !out->node_gen || !out->node_vx || !out->node_vy || !out->node_vz || !out->node_e) &&
          out->node_capacity > 0) ||
         ((outs & SUPA_OUT_KEYS) && out->node_capacity > 0 && !out->node_key))) {
        why = "tree outputs missing";
        return SUPA_ERR_INVALID_ARG;
    }
    return SUPA_OK;
}

extern "C" supa_status supa_validate_call(const supa_geometry *g, const supa_batch *b, const supa_output *out) {
    std::string why;
    supa_status s = validate(g, why);
    if (s == SUPA_OK) s = check_args(g->outputs, b, out, why);
    if (s != SUPA_OK) g_init_error = why;
    return s;
}

// Argument checks of a simulate call on a context (host only).
static supa_status check_call(supa_ctx *c, const supa_batch *b, supa_output *out) {
    if (!c) return SUPA_ERR_STATE;
    if (c->broken) return fail(c, SUPA_ERR_STATE, "context unusable after a device error");
    c->err.clear();
    std::string why;
    const supa_status s = check_args(c->g.outputs, b, out, why);
    if (s != SUPA_OK) return fail(c, s, why);
    out->total_hits = out->total_nodes = out->total_steps = 0;
    return SUPA_OK;
}

// Everything one call launches: parameters and scratch pointers.
struct Plan {
    bool tree, hits_out, images, recs, post;
    int N, nsub, phases;
    int64_t n, waves, img_words;
    supa::Params P;
    float e_unscale;
    int64_t *d_hstart, *d_part;
    int32_t *d_order;
    uint32_t *d_ohist;
    bool place_keys;                 // placement writes path ids
    uint2 *d_bucket;                 // placement's per-workgroup hit buckets, or null
    int32_t bucket_cap;
    unsigned long long *ctr;         // the call's counters (set 0 or 1)
    int64_t off(int j) const { return n * j / nsub; }
};

static constexpr size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

// Sizes the scratch for the call and fills the plan.  fixed == nullptr: the
// context's buffers, grown when needed; otherwise every piece is carved out
// of the fixed array at `fixed` (kFixedBytes), nothing is allocated, and the
// pieces are sized to fit it (a batch that needs more fails, see finish).
static supa_status prepare(supa_ctx *c, const supa_batch *b, uint64_t seed, supa_output *out, Plan &L,
                           int force_nsub, char *fixed = nullptr, int set = 0) {
    const uint32_t outs = c->g.outputs;
    const int64_t n = b->n;
    L.n = n;
    L.tree = (outs & SUPA_OUT_TREE) != 0;
    L.hits_out = (outs & SUPA_OUT_HITS) != 0;
    L.images = (outs & SUPA_OUT_IMAGES) != 0;
    L.recs = L.hits_out || L.images;
    L.post = L.recs || L.tree;
    L.N = c->g.n_planes;
    L.waves = std::max(1, c->n_cu * c->waves_per_cu);
    L.img_words = L.images ? (int64_t)c->n_layers * c->g.img_ny * c->g.img_nx : 0;
    // sub-batches: the placement of sub-batch j (aux stream) overlaps the
    // propagation of sub-batch j+1 (the context's stream); one by default
    int nsub = force_nsub > 0 ? force_nsub : (c->sub_batches > 0 ? c->sub_batches : 1);
    // subtree work items: automatic (0) = one export round when every shower
    // of the batch starts at once on at most a quarter of the waves (the
    // rest would idle behind the largest showers) and nothing else asks for
    // the single-launch path; measured to cost more than it saves once the
    // showers fill the waves
    const bool plain = c->g.kinematics != SUPA_KIN_LITERAL && c->g.n_regions < 2;
    int phases = c->phases;
    if (phases == 0)
        phases = (plain && !fixed && nsub <= 1 && force_nsub <= 1 && (int64_t)supa::SLOTS * n <= L.waves) ? 2 : 1;
    L.phases = plain ? phases : 1;
    if (!L.post || L.phases > 1) nsub = 1;
    L.nsub = (int)std::min<int64_t>(std::min(nsub, supa::MAX_SUB), n);
    // the placement kernel's variant (with path ids): sizes and launch must agree
    L.place_keys = L.hits_out && (outs & SUPA_OUT_KEYS) && out->hit_key != nullptr;

    // scratch: per-shower log starts, scan tile sums, work order; per-wave
    // spill; image buckets; hit and node logs
    const size_t hstart_b = L.recs ? al256((size_t)n * 8) : 0;
    const size_t part_b = al256((size_t)supa::scan_partial_words(n) * 8);
    const bool ordered = c->cost_order > 0 || (c->cost_order < 0 && n >= kAutoOrderMin);
    const size_t order_b = ordered ? al256((size_t)n * 4) + al256((size_t)supa::order_scratch_words() * 4) : 0;
    const size_t shower_b = hstart_b + part_b + order_b;
    int64_t bucket_per = 0, bucket_blocks = 0;
    if (L.images)
        supa::place_bucket_size(c->n_layers, c->g.img_nx, c->g.img_ny, L.place_keys, c->n_cu, &bucket_per,
                                &bucket_blocks);
    const size_t hit_chunk_b = (size_t)supa::HIT_CHUNK_WORDS * 4, node_chunk_b = (size_t)supa::NL_FIELDS * supa::LOG_CHUNK * 4;
    char *sh = nullptr, *spill_p = nullptr, *hlog_p = nullptr, *nlog_p = nullptr;
    char *items_p = nullptr, *shares_p = nullptr;
    int item_cap = 0, share_cap = 0;
    const bool subtrees = L.phases > 1;
    uint2 *bucket_p = nullptr;
    int32_t bucket_cap = 0;
    int spill_cap = c->spill_cap;
    int64_t h_chunks = c->h_chunks, n_chunks = c->n_chunks;
    if (!fixed) {
        const size_t spill_b = al256((size_t)L.waves * supa::POOL_FIELDS * c->spill_cap * 4);
        if (!c->spill.ensure(spill_b, &c->scratch_gen)) return nomem(c, "spill area", spill_b);
        // set 1 (the second call in flight of supa_simulate_batches) has logs
        // and log starts of its own; the rest is used by one call at a time
        DevBuf &hl = set ? c->hlog2 : c->hlog, &nl = set ? c->nlog2 : c->nlog;
        const size_t hlog_b = L.recs ? al256((size_t)h_chunks * 4) + (size_t)h_chunks * hit_chunk_b : 0;
        if (L.recs && !hl.ensure(hlog_b, &c->scratch_gen)) return nomem(c, "hit log", hlog_b);
        const size_t nlog_b = L.tree ? al256((size_t)n_chunks * 4) + (size_t)n_chunks * node_chunk_b : 0;
        if (L.tree && !nl.ensure(nlog_b, &c->scratch_gen)) return nomem(c, "node log", nlog_b);
        if (!c->shower.ensure(shower_b, &c->scratch_gen)) return nomem(c, "per-shower scratch", shower_b);
        if (set && hstart_b && !c->hstart2.ensure(hstart_b, &c->scratch_gen))
            return nomem(c, "per-shower log starts", hstart_b);
        if (bucket_per > 0) {
            const size_t bb = (size_t)bucket_per * bucket_blocks * sizeof(uint2);
            if (!c->bucket.ensure(bb, &c->scratch_gen)) return nomem(c, "image buckets", bb);
            bucket_p = (uint2 *)c->bucket.p;
            bucket_cap = (int32_t)bucket_per;
        }
        if (subtrees) {
            const size_t items_b = (size_t)2 * kItemCap * supa::ITEM_WORDS * 4;
            const size_t shares_b = (size_t)kShareCap * supa::SHARE_WORDS * 4;
            if (!c->items.ensure(items_b, &c->scratch_gen)) return nomem(c, "subtree items", items_b);
            if (!c->shares.ensure(shares_b, &c->scratch_gen)) return nomem(c, "share records", shares_b);
            items_p = (char *)c->items.p;
            shares_p = (char *)c->shares.p;
            item_cap = kItemCap;
            share_cap = kShareCap;
        }
        sh = (char *)c->shower.p;
        spill_p = (char *)c->spill.p;
        hlog_p = (char *)hl.p;
        nlog_p = (char *)nl.p;
    } else {
        size_t used = 0;
        auto take = [&](size_t bytes) -> char * {
            bytes = al256(bytes);
            if (bytes > kFixedBytes - used) return nullptr;
            char *p = fixed + used;
            used += bytes;
            return p;
        };
        sh = take(shower_b);
        if (!sh)
            return fail(c, SUPA_ERR_NOMEM, "a batch of " + std::to_string(n) + " showers needs " +
                                               std::to_string(shower_b) + " bytes of per-shower scratch; the fixed array holds " +
                                               std::to_string(kFixedBytes));
        // a wave takes SLOTS showers at a time: more waves than that would
        // idle (speed only), and each launched wave owns a spill area
        L.waves = std::min<int64_t>(L.waves, (n + supa::SLOTS - 1) / supa::SLOTS);
        const int64_t per_entry = L.waves * supa::POOL_FIELDS * 4;
        spill_cap = (int)std::min<int64_t>(c->spill_cap, (int64_t)(kFixedBytes / 8) / per_entry);
        // with exports the spill area is a ring indexed modulo its size
        if (subtrees)
            while (spill_cap & (spill_cap - 1)) spill_cap &= spill_cap - 1;
        spill_p = take((size_t)per_entry * spill_cap);
        if (!spill_p) return fail(c, SUPA_ERR_NOMEM, "no room left for the particle spill area in the fixed scratch array");
        if (bucket_per > 0) {
            bucket_cap = (int32_t)std::min<int64_t>(bucket_per, (int64_t)(kFixedBytes / 8) / (bucket_blocks * 8));
            bucket_p = bucket_cap > 0 ? (uint2 *)take((size_t)bucket_cap * bucket_blocks * 8) : nullptr;
            if (!bucket_p) bucket_cap = 0;
        }
        if (subtrees) {
            items_p = take((size_t)2 * kFixedItemCap * supa::ITEM_WORDS * 4);
            shares_p = take((size_t)kFixedShareCap * supa::SHARE_WORDS * 4);
            if (!items_p || !shares_p) return fail(c, SUPA_ERR_NOMEM, "no room left for subtree items in the fixed scratch array");
            item_cap = kFixedItemCap;
            share_cap = kFixedShareCap;
        }
        // the logs share what is left, in proportion to what the caller's
        // capacities suggest they need
        const size_t rest = kFixedBytes - used;
        const int64_t hint_h = (outs & SUPA_OUT_HITS) ? out->hit_capacity : 64 * n;
        const double need_h = L.recs ? (double)hit_chunks_for(std::min<int64_t>(hint_h, (int64_t)1 << 28), L.waves) * hit_chunk_b : 0.0;
        const double need_n = L.tree ? (double)node_chunks_for(std::min<int64_t>(out->node_capacity, (int64_t)1 << 28), L.waves) * node_chunk_b : 0.0;
        const size_t room_h = (need_h + need_n) > 0 ? (size_t)((double)rest * need_h / (need_h + need_n)) : 0;
        const size_t room_n = rest - room_h;
        h_chunks = L.recs ? (int64_t)((room_h > 512 ? room_h - 512 : 0) / (hit_chunk_b + 4)) : 0;
        n_chunks = L.tree ? (int64_t)((room_n > 512 ? room_n - 512 : 0) / (node_chunk_b + 4)) : 0;
        if ((L.recs && h_chunks < 1) || (L.tree && n_chunks < 1))
            return fail(c, SUPA_ERR_NOMEM, "no room left for the hit and node logs in the fixed scratch array");
        hlog_p = L.recs ? take(al256((size_t)h_chunks * 4) + (size_t)h_chunks * hit_chunk_b) : nullptr;
        nlog_p = L.tree ? take(al256((size_t)n_chunks * 4) + (size_t)n_chunks * node_chunk_b) : nullptr;
        if ((L.recs && !hlog_p) || (L.tree && !nlog_p))
            return fail(c, SUPA_ERR_NOMEM, "fixed scratch layout does not fit");
    }
    L.d_hstart = L.recs ? (int64_t *)(set ? (char *)c->hstart2.p : sh) : nullptr;
    L.d_part = (int64_t *)(sh + hstart_b);
    L.d_order = ordered ? (int32_t *)(sh + hstart_b + part_b) : nullptr;
    L.d_ohist = ordered ? (uint32_t *)(sh + hstart_b + part_b + al256((size_t)n * 4)) : nullptr;
    // images of many slabs: per-workgroup buckets sorting a shower's hits by slab
    L.d_bucket = bucket_p;
    L.bucket_cap = bucket_cap;
    const size_t hnext_b = al256((size_t)h_chunks * 4), nfill_b = al256((size_t)n_chunks * 4);

    supa::Params &P = L.P;
    P = supa::Params{};
    P.n_planes = L.N;
    P.z_first = (float)c->g.z_first;
    P.dz = (float)c->g.dz;
    P.c1 = c->d_c1;
    P.c2 = c->d_c2;
    P.t_cut = c->t_cut;
    P.f_lo = c->f_lo;
    P.f_w = c->f_w;
    P.angle_mode = c->g.angle_mode;
    P.angle_a = (float)c->g.angle_a;
    P.angle_b = (float)c->g.angle_b;
    P.e_scale = std::ldexp(1.0f, c->g.energy_frac_bits);
    P.seed_lo = (uint32_t)seed;
    P.seed_hi = (uint32_t)(seed >> 32);
    P.n = (int32_t)n;
    P.sid_base = b->shower_id_base;
    P.outputs = outs;
    P.keys = (outs & SUPA_OUT_KEYS) != 0;
    P.pool_cap = c->pool_cap;
    P.spill_cap = spill_cap;
    P.spill = (uint32_t *)spill_p;
    P.hnext = L.recs ? (uint32_t *)hlog_p : nullptr;
    P.hlog = L.recs ? (uint32_t *)(hlog_p + hnext_b) : nullptr;
    P.h_chunks = L.recs ? (int32_t)h_chunks : 0;
    P.nfill = L.tree ? (uint32_t *)nlog_p : nullptr;
    P.nlog = L.tree ? (uint32_t *)(nlog_p + nfill_b) : nullptr;
    P.n_chunks = L.tree ? (int32_t)n_chunks : 0;
    L.ctr = c->d_ctr + (set ? supa::CTR_WORDS : 0);
    P.ctr = L.ctr;
    P.sub = nullptr;
    P.phase = 0;
    P.last_phase = subtrees ? L.phases - 1 : 0;
    P.export_top = c->export_top;
    P.items = (uint32_t *)items_p;
    P.item_cap = item_cap;
    P.shares = (uint32_t *)shares_p;
    P.share_cap = share_cap;
    P.share_margin = c->share_margin;
    c->last_item_cap = item_cap;
    c->last_share_cap = share_cap;
    L.e_unscale = std::ldexp(1.0f, -c->g.energy_frac_bits);

    // the per-sub-batch input/output blocks, staged on the host
    for (int j = 0; j < L.nsub; ++j) {
        const int64_t o = L.off(j);
        supa::Cold &K = c->h_cold[j];
        std::memset(&K, 0, sizeof(K));
        K.e0 = b->e0 + o;
        K.polar = b->polar + o;
        K.azimuth = b->azimuth + o;
        K.x0 = b->x0 ? b->x0 + o : nullptr;
        K.y0 = b->y0 ? b->y0 + o : nullptr;
        K.order = L.d_order ? L.d_order + o : nullptr;
        K.ledger = out->ledger + 4 * o;
        K.counts = out->counts + 6 * o;
        K.hstart = L.d_hstart ? L.d_hstart + o : nullptr;
        for (int q = 0; q < 4; ++q) K.ring_r[q] = c->ring_r[q];
        K.wave_clk = c->d_wclk;
    }
    c->last_waves = L.waves;
    return SUPA_OK;
}

// Launches the call: counters cleared, then per sub-batch the work order,
// the propagation (main stream) and the scan, placement and node scatter
// (second stream, after the propagation of the same sub-batch).  d_cold
// holds the per-sub-batch blocks.  With timed, events bracket the parts.
// ev_prop[j], ev_post[j], ev_place[j]: the events of sub-batch j (the
// context's, or a call's own in supa_simulate_batches).  join: the main
// stream waits for the second stream at the end.
static supa_status enqueue(supa_ctx *c, const supa_batch *b, supa_output *out, const Plan &L,
                           supa::Cold *d_cold, hipStream_t s_main, hipStream_t s_aux, bool timed,
                           hipEvent_t (*ev_prop)[2], hipEvent_t (*ev_post)[2], hipEvent_t *ev_place,
                           bool join = true) {
    auto sub_ctr = [&](int j) { return L.ctr + supa::CTR_BLOCK * (1 + j); };
    const supa::Params &P = L.P;
    HIP_TRY(c, supa::launch_zero_counters(L.ctr, s_main));
    for (int j = 0; j < L.nsub; ++j) {
        const int64_t o = L.off(j), nj = L.off(j + 1) - o;
        supa::Params Pj = P;
        Pj.n = (int32_t)nj;
        Pj.sid_base = b->shower_id_base + (uint32_t)o;
        Pj.cold = d_cold + j;
        Pj.sub = sub_ctr(j);
        if (L.d_order)
            HIP_TRY(c, supa::launch_cost_order(b->e0 + o, (int)nj, P.e_scale, L.d_ohist, L.d_order + o,
                                               c->n_cu, s_main));
        if (timed) HIP_TRY(c, hipEventRecord(ev_prop[j][0], s_main));
        HIP_TRY(c, supa::launch_propagate(Pj, c->g.kinematics == SUPA_KIN_LITERAL, c->g.n_regions >= 2, (int)L.waves, s_main));
        // later launches finish the subtree items the previous one exported
        for (int ph = 1; ph <= P.last_phase; ++ph) {
            supa::Params Pp = Pj;
            Pp.phase = ph;
            HIP_TRY(c, supa::launch_propagate(Pp, false, false, (int)L.waves, s_main));
        }
        if (L.tree) HIP_TRY(c, supa::launch_note_chunks(L.ctr, sub_ctr(j), s_main));
        // the second stream waits on this event (none inside a capture, where
        // both are one stream)
        const bool two = s_aux != s_main;
        if (timed || two) HIP_TRY(c, hipEventRecord(ev_prop[j][1], s_main));
        if (!L.post) continue;

        supa::ScanParams SP{};
        SP.n = (int32_t)nj;
        SP.counts = out->counts + 6 * o;
        SP.hoff = L.hits_out ? out->hit_offsets + o : nullptr;
        SP.noff = L.tree ? out->node_offsets + o : nullptr;
        SP.partial = L.d_part;
        SP.sub = sub_ctr(j);
        SP.prev = j > 0 ? sub_ctr(j - 1) : nullptr;

        supa::PlaceParams H{};
        H.n = (int32_t)nj;
        H.n_planes = L.N;
        H.L = c->n_layers;
        H.nx = c->g.img_nx;
        H.ny = c->g.img_ny;
        H.x0 = (float)c->g.img_x0;
        H.y0 = (float)c->g.img_y0;
        H.sx = L.images ? (float)(c->g.img_nx / (c->g.img_x1 - c->g.img_x0)) : 0.0f;
        H.sy = L.images ? (float)(c->g.img_ny / (c->g.img_y1 - c->g.img_y0)) : 0.0f;
        H.e_unscale = L.e_unscale;
        H.ctr = L.ctr;
        H.sub = sub_ctr(j);
        H.counts = SP.counts;
        H.hstart = L.d_hstart ? L.d_hstart + o : nullptr;
        H.hlog = P.hlog;
        H.hnext = P.hnext;
        H.h_chunks = P.h_chunks;
        H.layer = c->d_layer;
        H.hoff = SP.hoff;
        H.hcap = L.hits_out ? out->hit_capacity : 0;
        H.hx = L.hits_out ? out->hit_x : nullptr;
        H.hy = L.hits_out ? out->hit_y : nullptr;
        H.he = L.hits_out ? out->hit_e : nullptr;
        H.hl = L.hits_out ? out->hit_layer : nullptr;
        H.hk = L.place_keys ? out->hit_key : nullptr;
        H.images = L.images ? out->images + L.img_words * o : nullptr;
        H.bucket = L.d_bucket;
        H.bucket_cap = L.bucket_cap;

        supa::ScatterParams Q{};
        Q.z_first = P.z_first;
        Q.dz = P.dz;
        Q.e_unscale = L.e_unscale;
        Q.ctr = L.ctr;
        Q.sub = sub_ctr(j);
        Q.prev = SP.prev;
        Q.nlog = P.nlog;
        Q.nfill = P.nfill;
        Q.n_chunks = P.n_chunks;
        Q.noff = SP.noff;
        Q.ncap = L.tree ? out->node_capacity : 0;
        Q.np = out->node_parent;
        Q.ng = out->node_gen;
        Q.nvx = out->node_vx;
        Q.nvy = out->node_vy;
        Q.nvz = out->node_vz;
        Q.ne = out->node_e;
        Q.nk = (L.tree && P.keys) ? out->node_key : nullptr;

        if (two) HIP_TRY(c, hipStreamWaitEvent(s_aux, ev_prop[j][1], 0));
        HIP_TRY(c, supa::launch_scan(SP, s_aux));
        if (timed) HIP_TRY(c, hipEventRecord(ev_post[j][0], s_aux));
        if (L.recs) HIP_TRY(c, supa::launch_place(H, c->n_cu, s_aux));
        if (timed) HIP_TRY(c, hipEventRecord(ev_place[j], s_aux));
        if (L.tree) HIP_TRY(c, supa::launch_scatter_nodes(Q, (int32_t)nj, c->n_cu, s_aux));
        if (timed || two) HIP_TRY(c, hipEventRecord(ev_post[j][1], s_aux));
    }
    if (join && L.post && s_aux != s_main) HIP_TRY(c, hipStreamWaitEvent(s_main, ev_post[L.nsub - 1][1], 0));
    return SUPA_OK;
}

// Outcome of a call from the counters it left (host copy in c->h_ctr):
// OK, CAPACITY, RANGE, DEVICE, or -1 when scratch ran out (grown here; rerun).
static int finish(supa_ctx *c, const Plan &L, supa_output *out, bool fixed = false,
                  const unsigned long long *h = nullptr) {
    if (!h) h = c->h_ctr;
    const unsigned long long flags = h[supa::CTR_FLAGS];
    if (flags & supa::FLAG_RANGE)
        return fail(c, SUPA_ERR_RANGE, "an initial energy is negative, NaN or too large for the fixed-point format");
    const unsigned long long *last = h + supa::CTR_BLOCK * L.nsub;    // running totals
    const int64_t total_hits = (int64_t)last[supa::SUB_HITS], total_nodes = (int64_t)last[supa::SUB_NODES];
    if ((flags & (supa::FLAG_OVERFLOW | supa::FLAG_SHARE)) && fixed)
        return fail(c, SUPA_ERR_NOMEM, "the batch needs more scratch (particle spill, hit or node log) than the "
                                       "fixed array of " + std::to_string(kFixedBytes) + " bytes holds: run it in "
                                       "smaller calls, or with supa_simulate");
    if (flags & supa::FLAG_SHARE) {
        // a shared shower outgrew the hit-log chunks reserved for it (the
        // records that did not fit were dropped): rerun with a larger reserve
        if (c->share_margin >= 64.0f)
            return fail(c, SUPA_ERR_DEVICE, "shared showers' hit reserves did not converge");
        c->share_margin *= 2.0f;
        if (!(flags & supa::FLAG_OVERFLOW)) return -1;
    }
    if (flags & supa::FLAG_OVERFLOW) {
        // grow what ran out: the spill area to the largest pool seen, a log
        // to the totals (exact unless the spill overflowed too)
        const int64_t nf = std::max<int64_t>(0, (int64_t)h[supa::CTR_NEED_F] - c->pool_cap);
        c->spill_cap = (int)std::min<int64_t>((int64_t)1 << 30,
                                              std::max<int64_t>(c->spill_cap, round_up_pow2(nf + 1)));
        if (L.recs && (int64_t)h[supa::CTR_HCHUNK] > c->h_chunks)
            c->h_chunks = std::max(2 * c->h_chunks, hit_chunks_for(total_hits, L.waves));
        if (L.tree && (int64_t)h[supa::CTR_NCHUNK] > c->n_chunks)
            c->n_chunks = std::max(2 * c->n_chunks, node_chunks_for(total_nodes, L.waves));
        return -1;
    }
    // only meaningful when nothing overflowed (a lost spill entry breaks
    // the particle accounting of its wave, and the batch is rerun anyway)
    if (flags & supa::FLAG_INTERNAL) {
        c->broken = true;
        return fail(c, SUPA_ERR_DEVICE, "internal particle accounting error in the propagation kernel");
    }
    out->total_steps = (int64_t)h[supa::CTR_STEPS];
    out->total_hits = L.hits_out ? total_hits : 0;
    out->total_nodes = L.tree ? total_nodes : 0;
    if (L.hits_out && total_hits > out->hit_capacity)
        return fail(c, SUPA_ERR_CAPACITY, "hit arrays too small: need " + std::to_string(total_hits));
    if (L.tree && total_nodes > out->node_capacity)
        return fail(c, SUPA_ERR_CAPACITY, "node arrays too small: need " + std::to_string(total_nodes));
    return SUPA_OK;
}

// first sizes of the logs: the caller's capacities (or 64 hits per shower
// for images only), unless earlier batches needed more
static void size_logs(supa_ctx *c, const supa_batch *b, const supa_output *out) {
    const uint32_t outs = c->g.outputs;
    const int64_t waves = std::max(1, c->n_cu * c->waves_per_cu);
    if (outs & (SUPA_OUT_HITS | SUPA_OUT_IMAGES)) {
        const int64_t hint = (outs & SUPA_OUT_HITS) ? out->hit_capacity : 64 * b->n;
        c->h_chunks = std::max(c->h_chunks, hit_chunks_for(std::min<int64_t>(hint, (int64_t)1 << 28), waves));
    }
    if (outs & SUPA_OUT_TREE)
        c->n_chunks = std::max(c->n_chunks,
                               node_chunks_for(std::min<int64_t>(out->node_capacity, (int64_t)1 << 28), waves));
}

// Runs a prepared call once: launches it, reads back its counters (one
// synchronisation) and records the kernel times.
static supa_status run_once(supa_ctx *c, const supa_batch *b, supa_output *out, const Plan &L) {
    HIP_TRY(c, hipMemcpyAsync(c->d_cold, c->h_cold, L.nsub * sizeof(supa::Cold), hipMemcpyHostToDevice,
                              c->stream));
    HIP_TRY(c, hipEventRecord(c->ev_begin, c->stream));
    supa_status st = enqueue(c, b, out, L, c->d_cold, c->stream, c->aux, true, c->ev_prop, c->ev_post, c->ev_place);
    if (st != SUPA_OK) return st;
    HIP_TRY(c, hipMemcpyAsync(c->h_ctr, L.ctr, supa::CTR_WORDS * sizeof(unsigned long long),
                              hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipEventRecord(c->ev_end, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    float t_prop = 0, t_post = 0, t_all = 0, t_place = 0, t_scatter = 0, t = 0;
    for (int j = 0; j < L.nsub; ++j) {
        if (hipEventElapsedTime(&t, c->ev_prop[j][0], c->ev_prop[j][1]) == hipSuccess) t_prop += t;
        if (L.post && hipEventElapsedTime(&t, c->ev_post[j][0], c->ev_post[j][1]) == hipSuccess) t_post += t;
        if (L.recs && hipEventElapsedTime(&t, c->ev_post[j][0], c->ev_place[j]) == hipSuccess) t_place += t;
        if (L.tree && hipEventElapsedTime(&t, c->ev_place[j], c->ev_post[j][1]) == hipSuccess) t_scatter += t;
    }
    (void)hipEventElapsedTime(&t_all, c->ev_begin, c->ev_end);
    (void)hipGetLastError();
    c->timing[0] = t_prop;
    c->timing[1] = t_post;
    c->timing[2] = t_all;
    c->timing[3] = t_place;
    c->timing[4] = t_scatter;
    c->last_sub_batches = L.nsub;
    return SUPA_OK;
}

extern "C" supa_status supa_simulate(supa_ctx *c, const supa_batch *b, uint64_t seed,
                                     supa_output *out) {
    supa_status st = check_call(c, b, out);
    if (st != SUPA_OK || b->n == 0) return st;
    HIP_TRY(c, hipSetDevice(c->device));
    size_logs(c, b, out);
    for (int attempt = 0; attempt < 8; ++attempt) {
        Plan L{};
        st = prepare(c, b, seed, out, L, 0);
        if (st != SUPA_OK) return st;
        st = run_once(c, b, out, L);
        if (st != SUPA_OK) return st;
        const int r = finish(c, L, out);
        if (r >= 0) return (supa_status)r;
    }
    return fail(c, SUPA_ERR_NOMEM, "scratch sizes did not converge");
}

// supa_simulate with the library's scratch carved out of this device's fixed
// array: no allocation, no growth, one attempt.
extern "C" supa_status supa_simulate_noalloc(supa_ctx *c, const supa_batch *b, uint64_t seed,
                                             supa_output *out) {
    supa_status st = check_call(c, b, out);
    if (st != SUPA_OK || b->n == 0) return st;
    if (!c->fixed) return fail(c, SUPA_ERR_STATE, "the fixed scratch array of this device is not resolved");
    HIP_TRY(c, hipSetDevice(c->device));
    Plan L{};
    st = prepare(c, b, seed, out, L, 0, c->fixed);
    if (st != SUPA_OK) return st;
    st = run_once(c, b, out, L);
    if (st != SUPA_OK) return st;
    return (supa_status)finish(c, L, out, true);
}

// ---------------------------------------------------------------------------
// Several calls in one: the propagation of call j+1 (main stream) overlaps
// the scan, placement and node scatter of call j (second stream).  The logs,
// log starts and counters that a propagation writes and the next steps read
// come in two sets, used by alternate calls; a call reuses a set once the
// second stream is done with the call before the previous one.  Each call's
// counters are copied aside when its second-stream work ends and read back
// together with one synchronisation at the end.
// ---------------------------------------------------------------------------
static bool ensure_pinned(void **p, size_t *have, size_t need) {
    if (need <= *have) return true;
    if (*p) (void)hipHostFree(*p);
    *p = nullptr;
    *have = 0;
    if (hipHostMalloc(p, need, 0) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    *have = need;
    return true;
}

extern "C" supa_status supa_simulate_batches(supa_ctx *c, int32_t k, const supa_batch *b, uint64_t seed,
                                             supa_output *out) {
    if (!c) return SUPA_ERR_STATE;
    if (k < 0 || (k > 0 && (!b || !out))) return fail(c, SUPA_ERR_INVALID_ARG, "bad call list");
    for (int32_t j = 0; j < k; ++j) {
        const supa_status st = check_call(c, &b[j], &out[j]);
        if (st != SUPA_OK) {
            c->err = "call " + std::to_string(j) + ": " + c->err;
            return st;
        }
    }
    if (k == 0) return SUPA_OK;
    HIP_TRY(c, hipSetDevice(c->device));
    for (int32_t j = 0; j < k; ++j) size_logs(c, &b[j], &out[j]);
    // pinned per-call staging, device per-call blocks, counters and events
    size_t calls_n = c->h_calls_n;
    if (!ensure_pinned((void **)&c->h_calls, &calls_n, (size_t)k * sizeof(supa::Cold)))
        return nomem(c, "pinned per-call blocks", (size_t)k * sizeof(supa::Cold));
    c->h_calls_n = calls_n;
    const size_t snap_b = (size_t)k * supa::CTR_WORDS * sizeof(unsigned long long);
    if (!ensure_pinned((void **)&c->h_snap, &c->h_snap_bytes, snap_b)) return nomem(c, "pinned counters", snap_b);
    if (!c->snap.ensure(snap_b, &c->scratch_gen)) return nomem(c, "per-call counters", snap_b);
    if (!c->d_calls.ensure((size_t)k * sizeof(supa::Cold), &c->scratch_gen))
        return nomem(c, "per-call blocks", (size_t)k * sizeof(supa::Cold));
    while (c->call_ev.size() < (size_t)k * 5) {
        hipEvent_t e = nullptr;
        HIP_TRY(c, hipEventCreate(&e));
        c->call_ev.push_back(e);
    }
    // consecutive calls are in flight together: the per-shower rows that one
    // call's propagation writes (ledger, counts) must not be read by the
    // other's placement
    for (int32_t j = 0; j + 1 < k; ++j) {
        auto span = [](const void *p, int64_t bytes) { return std::make_pair((uintptr_t)p, (uintptr_t)p + bytes); };
        const auto la = span(out[j].ledger, b[j].n * 32), lb = span(out[j + 1].ledger, b[j + 1].n * 32);
        const auto ca = span(out[j].counts, b[j].n * 24), cb = span(out[j + 1].counts, b[j + 1].n * 24);
        auto meet = [](std::pair<uintptr_t, uintptr_t> x, std::pair<uintptr_t, uintptr_t> y) {
            return x.first < x.second && y.first < y.second && x.first < y.second && y.first < x.second;
        };
        if (meet(la, lb) || meet(ca, cb) || meet(la, cb) || meet(ca, lb))
            return fail(c, SUPA_ERR_INVALID_ARG, "calls " + std::to_string(j) + " and " + std::to_string(j + 1) +
                                                     " share ledger or counts rows (consecutive calls run at once)");
    }
    std::vector<Plan> plans((size_t)k);
    for (int attempt = 0; attempt < 8; ++attempt) {
        // sizes first (buffers may grow: nothing is in flight), then the
        // plans, whose pointers no later preparation moves
        supa_status st = SUPA_OK;
        for (int pass = 0; pass < 2 && st == SUPA_OK; ++pass)
            for (int32_t j = 0; j < k && st == SUPA_OK; ++j) {
                st = prepare(c, &b[j], seed, &out[j], plans[j], 1, nullptr, j & 1);
                if (pass == 1) c->h_calls[j] = c->h_cold[0];
            }
        if (st != SUPA_OK) return st;
        supa::Cold *d_calls = (supa::Cold *)c->d_calls.p;
        HIP_TRY(c, hipEventRecord(c->ev_begin, c->stream));
        HIP_TRY(c, hipMemcpyAsync(d_calls, c->h_calls, (size_t)k * sizeof(supa::Cold), hipMemcpyHostToDevice,
                                  c->stream));
        unsigned long long *snap = (unsigned long long *)c->snap.p;
        for (int32_t j = 0; j < k; ++j) {
            const int q = j & 1;
            // the set's buffers are free once the second stream is done with call j - 2
            if (j >= 2) HIP_TRY(c, hipStreamWaitEvent(c->stream, c->ev_set_free[q], 0));
            hipEvent_t *e = &c->call_ev[(size_t)j * 5];
            hipEvent_t ev_prop[1][2] = {{e[0], e[1]}}, ev_post[1][2] = {{e[2], e[4]}}, ev_place[1] = {e[3]};
            st = enqueue(c, &b[j], &out[j], plans[j], d_calls + j, c->stream, c->aux, true, ev_prop, ev_post,
                         ev_place, false);
            if (st != SUPA_OK) return st;
            // counters-only calls have no second-stream part: order after the propagation
            if (!plans[j].post) HIP_TRY(c, hipStreamWaitEvent(c->aux, e[1], 0));
            HIP_TRY(c, hipMemcpyAsync(snap + (size_t)j * supa::CTR_WORDS, plans[j].ctr,
                                      supa::CTR_WORDS * sizeof(unsigned long long), hipMemcpyDeviceToDevice,
                                      c->aux));
            HIP_TRY(c, hipEventRecord(c->ev_set_free[q], c->aux));
        }
        HIP_TRY(c, hipEventRecord(c->ev_joined, c->aux));
        HIP_TRY(c, hipStreamWaitEvent(c->stream, c->ev_joined, 0));
        HIP_TRY(c, hipMemcpyAsync(c->h_snap, snap, snap_b, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipEventRecord(c->ev_end, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        float t_prop = 0, t_post = 0, t_all = 0, t_place = 0, t_scatter = 0, t = 0;
        for (int32_t j = 0; j < k; ++j) {
            const hipEvent_t *e = &c->call_ev[(size_t)j * 5];
            if (hipEventElapsedTime(&t, e[0], e[1]) == hipSuccess) t_prop += t;
            if (plans[j].post && hipEventElapsedTime(&t, e[2], e[4]) == hipSuccess) t_post += t;
            if (plans[j].recs && hipEventElapsedTime(&t, e[2], e[3]) == hipSuccess) t_place += t;
            if (plans[j].tree && hipEventElapsedTime(&t, e[3], e[4]) == hipSuccess) t_scatter += t;
        }
        (void)hipEventElapsedTime(&t_all, c->ev_begin, c->ev_end);
        (void)hipGetLastError();
        c->timing[0] = t_prop;
        c->timing[1] = t_post;
        c->timing[2] = t_all;
        c->timing[3] = t_place;
        c->timing[4] = t_scatter;
        c->last_sub_batches = 1;
        // outcome: a range error anywhere wins, then a capacity error; an
        // overflow of library scratch grows it and reruns every call
        bool rerun = false, cap = false;
        int first_cap = -1;
        for (int32_t j = 0; j < k; ++j) {
            const int r = finish(c, plans[j], &out[j], false, c->h_snap + (size_t)j * supa::CTR_WORDS);
            if (r < 0) {
                rerun = true;
            } else if (r == SUPA_ERR_RANGE || r == SUPA_ERR_DEVICE) {
                c->err = "call " + std::to_string(j) + ": " + c->err;
                return (supa_status)r;
            } else if (r == SUPA_ERR_CAPACITY) {
                if (!cap) first_cap = j;
                cap = true;
            }
        }
        if (rerun) continue;
        if (cap) {
            // finish() of later calls cleared the message: restate the first
            return fail(c, SUPA_ERR_CAPACITY, "call " + std::to_string(first_cap) + ": hit or node arrays too small "
                                              "(need " + std::to_string(out[first_cap].total_hits) + " hits, " +
                                              std::to_string(out[first_cap].total_nodes) + " nodes)");
        }
        c->err.clear();
        return SUPA_OK;
    }
    return fail(c, SUPA_ERR_NOMEM, "scratch sizes did not converge");
}

// A captured call: the launch sequence of one supa_simulate (one sub-batch,
// no host work) as an instantiated HIP graph, with its own copy of the
// per-call input/output block so that replays do not depend on later calls.
struct supa_graph {
    supa_ctx *ctx = nullptr;
    uint64_t gen = 0;                    // the context's scratch generation at capture
    hipGraphExec_t exec = nullptr;
    supa::Cold *d_cold = nullptr;
    Plan plan{};
    supa_output out{};
};

extern "C" supa_status supa_graph_create(supa_ctx *c, const supa_batch *b, uint64_t seed,
                                         supa_output *out, supa_graph **gout) {
    if (!c) return SUPA_ERR_STATE;
    if (!gout) return fail(c, SUPA_ERR_INVALID_ARG, "graph out pointer is NULL");
    *gout = nullptr;
    supa_status st = check_call(c, b, out);
    if (st != SUPA_OK) return st;
    if (b->n == 0) return fail(c, SUPA_ERR_INVALID_ARG, "an empty batch has no graph");
    // one eager call sizes every scratch buffer and checks the capacities
    const int saved_sub = c->sub_batches;
    c->sub_batches = 1;
    st = supa_simulate(c, b, seed, out);
    c->sub_batches = saved_sub;
    if (st != SUPA_OK) return st;
    supa_graph *g = new supa_graph();
    g->ctx = c;
    g->out = *out;
    st = prepare(c, b, seed, out, g->plan, 1);         // sizes suffice: allocates nothing
    if (st != SUPA_OK) {
        delete g;
        return st;
    }
    g->gen = c->scratch_gen;
    hipGraph_t graph = nullptr;
    hipError_t e = hipMalloc(&g->d_cold, sizeof(supa::Cold));
    if (e == hipSuccess) e = hipMemcpy(g->d_cold, c->h_cold, sizeof(supa::Cold), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipStreamBeginCapture(c->aux, hipStreamCaptureModeRelaxed);
    if (e == hipSuccess) {
        st = enqueue(c, b, out, g->plan, g->d_cold, c->aux, c->aux, false, c->ev_prop, c->ev_post, c->ev_place);
        const hipError_t e2 = hipStreamEndCapture(c->aux, &graph);
        if (st == SUPA_OK && e2 != hipSuccess) e = e2;
    }
    if (e == hipSuccess && st == SUPA_OK) e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (e != hipSuccess || st != SUPA_OK) {
        if (g->d_cold) (void)hipFree(g->d_cold);
        delete g;
        (void)hipGetLastError();
        return st != SUPA_OK ? st : fail(c, SUPA_ERR_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    }
    *gout = g;
    return SUPA_OK;
}

// the graph's kernels hold the scratch addresses of the capture: after a
// reallocation they would read and write freed memory
static supa_status graph_current(supa_graph *g) {
    if (g->gen == g->ctx->scratch_gen) return SUPA_OK;
    return fail(g->ctx, SUPA_ERR_STATE,
                "the context's scratch was reallocated after this graph was captured: create the graph again");
}

extern "C" supa_status supa_graph_launch(supa_graph *g, void *hip_stream) {
    if (!g || !g->ctx) return SUPA_ERR_STATE;
    supa_ctx *c = g->ctx;
    const supa_status cur = graph_current(g);
    if (cur != SUPA_OK) return cur;
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipGraphLaunch(g->exec, hip_stream ? (hipStream_t)hip_stream : c->stream));
    return SUPA_OK;
}

extern "C" supa_status supa_graph_check(supa_graph *g, void *hip_stream, int64_t *totals3) {
    if (!g || !g->ctx) return SUPA_ERR_STATE;
    supa_ctx *c = g->ctx;
    const supa_status cur = graph_current(g);
    if (cur != SUPA_OK) return cur;
    const hipStream_t s = hip_stream ? (hipStream_t)hip_stream : c->stream;
    HIP_TRY(c, hipMemcpyAsync(c->h_ctr, g->plan.ctr, supa::CTR_WORDS * sizeof(unsigned long long),
                              hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    supa_output o = g->out;
    int r = finish(c, g->plan, &o);
    if (r < 0) r = fail(c, SUPA_ERR_CAPACITY, "library scratch too small for this replay: create the graph again");
    if (totals3) {
        totals3[0] = o.total_hits;
        totals3[1] = o.total_nodes;
        totals3[2] = o.total_steps;
    }
    return (supa_status)r;
}

extern "C" supa_status supa_graph_destroy(supa_graph *g) {
    if (!g) return SUPA_ERR_STATE;
    if (g->ctx) (void)hipSetDevice(g->ctx->device);
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->d_cold) (void)hipFree(g->d_cold);
    delete g;
    return SUPA_OK;
}

// Launch-setting search: every combination of waves per CU, LDS pool size,
// sub-batches and cost order is run on the caller's batch (the first call
// of each setting warms up and sizes scratch; the second is timed with the
// context's events), and the fastest whole-call time wins.  Results are
// identical under every setting, so `out` holds the batch's results after
// the search, from the winning setting.
extern "C" supa_status supa_autotune(supa_ctx *c, const supa_batch *b, uint64_t seed, supa_output *out,
                                     int32_t *best, float *best_ms) {
    if (!c) return SUPA_ERR_STATE;
    if (!best || !best_ms) return fail(c, SUPA_ERR_INVALID_ARG, "best and best_ms are required");
    // a batch size searched before on this context (its geometry and
    // device): the same settings, one call
    for (const supa_ctx::Tuned &t : c->tuned)
        if (t.n == (b ? b->n : -1)) {
            c->waves_per_cu = t.best[0];
            c->pool_cap = t.best[1];
            c->sub_batches = t.best[2];
            c->cost_order = t.best[3];
            std::memcpy(best, t.best, sizeof(t.best));
            *best_ms = t.ms;
            return supa_simulate(c, b, seed, out);
        }
    static const int waves[] = {8, 12, 16};
    static const int pools[] = {128, 256};
    static const int subs[] = {1, 2};
    static const int orders[] = {0, 1};
    const int saved[4] = {c->waves_per_cu, c->pool_cap, c->sub_batches, c->cost_order};
    float bms = 1e30f;
    int bw = saved[0], bp = saved[1], bs = saved[2], bo = saved[3];
    for (int w : waves)
        for (int p : pools)
            for (int sb : subs)
                for (int o : orders) {
                    c->waves_per_cu = w;
                    c->pool_cap = p;
                    c->sub_batches = sb;
                    c->cost_order = o;
                    supa_status st = supa_simulate(c, b, seed, out);
                    if (st == SUPA_OK) st = supa_simulate(c, b, seed, out);
                    if (st != SUPA_OK) {
                        c->waves_per_cu = saved[0];
                        c->pool_cap = saved[1];
                        c->sub_batches = saved[2];
                        c->cost_order = saved[3];
                        return st;
                    }
                    if (c->timing[2] < bms) {
                        bms = c->timing[2];
                        bw = w;
                        bp = p;
                        bs = sb;
                        bo = o;
                    }
                }
    c->waves_per_cu = bw;
    c->pool_cap = bp;
    c->sub_batches = bs;
    c->cost_order = bo;
    const supa_status st = supa_simulate(c, b, seed, out);
    best[0] = bw;
    best[1] = bp;
    best[2] = bs;
    best[3] = bo;
    *best_ms = bms;
    if (st == SUPA_OK) c->tuned.push_back(supa_ctx::Tuned{b->n, {bw, bp, bs, bo}, bms});
    return st;
}

extern "C" supa_status supa_autotune_forget(supa_ctx *c) {
    if (!c) return SUPA_ERR_STATE;
    c->tuned.clear();
    return SUPA_OK;
}
