// supa_propagate.hip -- the SUPA propagation kernel for gfx950.
//
// One wave (64 lanes) owns one shower at a time and pulls the next one from a
// device work queue, so a single launch of a few waves per compute unit runs a
// whole batch however uneven its showers are.  Within a shower the wave walks
// the planes in order (section "Propagation Model": at each slice every live
// particle stops, splits or passes, Algorithm 1), 64 particles per step:
//   free flight to plane k  ->  threshold test  ->  one Philox block  ->
//   three-way choice  ->  split kinematics  ->  ballot/prefix compaction of
//   the next plane's particles, of the new tree nodes and of the hits.
// Compaction is a wave ballot plus a popcount of the lanes below, so the
// order of particles, nodes and hits is the creation order a sequential
// implementation produces, with no atomics.  Particles live in a per-wave
// structure-of-arrays double buffer; hits and nodes are journaled per wave and
// copied once per shower into the caller's arrays at a segment reserved with a
// single atomic.  Per-layer images are binned from the hit journal into an LDS
// tile (integer sums, order independent) and written once.
#include "supa_device.hpp"

namespace supa {

constexpr int WAVE = 64;
constexpr int WAVES_PER_BLOCK = 4;
constexpr int TILE_WORDS = 2048;          // 8 KB LDS image tile per wave

struct Daughters {
    float txa, tya, txb, tyb;
    uint32_t ea, eb;
    bool fwd_a, fwd_b;
};

// Split of one particle (section "Propagation Model", split bullet; Algorithm 1,
// split branch): exact fixed-point energy split by the 32-bit fraction F drawn
// from w1, opening angle theta from w2, azimuth omega from w3; the daughters
// turn by theta*(1-f) and theta*f to opposite sides of the plane through the
// parent direction at azimuth omega (frame: rotation taking +z to d).
__device__ __forceinline__ Daughters split_particle(const Params &P, float tx, float ty,
                                                    uint32_t e, uint4 w) {
    Daughters D;
    const uint32_t F = P.f_lo + (uint32_t)(((uint64_t)w.y * P.f_w) >> 32);
    D.ea = (uint32_t)(((uint64_t)e * F) >> 32);
    D.eb = e - D.ea;
    const float f = (float)F * 0x1p-32f;     // fraction carried by daughter a
    const float g = 1.0f - f;

    float theta;
    if (P.angle_mode == 0) {
        theta = P.angle_a;
    } else if (P.angle_mode == 1) {
        theta = fmaf(P.angle_b - P.angle_a, ((float)w.z + 0.5f) * 0x1p-32f, P.angle_a);
    } else {
        // Rayleigh(sigma): sigma*sqrt(-2 ln u); ln u through log1p(-(1-u)) when
        // u >= 1/2 so that the argument is exact in single precision
        float lnu;
        if (w.z < 0x80000000u)
            lnu = logf(((float)w.z + 0.5f) * 0x1p-32f);
        else
            lnu = log1pf(-(((float)(~w.z) + 0.5f) * 0x1p-32f));
        theta = P.angle_a * sqrtf(-2.0f * lnu);
    }
    // omega = 2 pi u(w3), taken as pi*(signed w3 + 1/2)/2^31 (same angle mod 2 pi)
    float so, co;
    sincospif(((float)(int32_t)w.w + 0.5f) * 0x1p-31f, &so, &co);

    // unit direction from the slopes
    const float dz = 1.0f / sqrtf(1.0f + fmaf(tx, tx, ty * ty));
    const float dx = tx * dz, dy = ty * dz;
    const float c = 1.0f / (1.0f + dz);
    const float e1x = fmaf(-dx * dx, c, 1.0f), e1y = -dx * dy * c, e1z = -dx;
    const float e2x = e1y, e2y = fmaf(-dy * dy, c, 1.0f), e2z = -dy;
    const float nx = co * e1x + so * e2x;
    const float ny = co * e1y + so * e2y;
    const float nz = co * e1z + so * e2z;

    float sa, ca, sb, cb;
    sincosf(theta * g, &sa, &ca);
    sincosf(theta * f, &sb, &cb);
    const float ax = ca * dx + sa * nx, ay = ca * dy + sa * ny, az = ca * dz + sa * nz;
    const float bx = cb * dx - sb * nx, by = cb * dy - sb * ny, bz = cb * dz - sb * nz;
    D.fwd_a = az > 0.0f;
    D.fwd_b = bz > 0.0f;
    const float ia = 1.0f / az, ib = 1.0f / bz;
    D.txa = ax * ia;
    D.tya = ay * ia;
    D.txb = bx * ib;
    D.tyb = by * ib;
    return D;
}

__global__ void __launch_bounds__(WAVE *WAVES_PER_BLOCK) supa_propagate(Params P) {
    __shared__ uint32_t lds_tile[WAVES_PER_BLOCK][TILE_WORDS];
    const uint32_t lane = lane_id();
    const int wib = threadIdx.x / WAVE;
    const int64_t wave = (int64_t)blockIdx.x * WAVES_PER_BLOCK + wib;
    uint32_t *tile = lds_tile[wib];

    const int64_t cap_f = P.cap_f, cap_h = P.cap_h, cap_n = P.cap_n;
    float *const fx = P.fx + wave * 2 * cap_f;
    float *const fy = P.fy + wave * 2 * cap_f;
    float *const ftx = P.ftx + wave * 2 * cap_f;
    float *const fty = P.fty + wave * 2 * cap_f;
    uint32_t *const fe = P.fe + wave * 2 * cap_f;
    uint32_t *const fplo = P.fplo + wave * 2 * cap_f;
    uint32_t *const fphi = P.fphi + wave * 2 * cap_f;
    int32_t *const fnode = P.fnode + wave * 2 * cap_f;

    const bool want_hits = (P.outputs & 3u) != 0;   // hit clouds or images
    const bool want_tree = (P.outputs & 4u) != 0;
    float *const jhx = want_hits ? P.jhx + wave * cap_h : nullptr;
    float *const jhy = want_hits ? P.jhy + wave * cap_h : nullptr;
    uint32_t *const jhe = want_hits ? P.jhe + wave * cap_h : nullptr;
    int32_t *const jhl = want_hits ? P.jhl + wave * cap_h : nullptr;
    uint32_t *const jhplo = want_hits ? P.jhplo + wave * cap_h : nullptr;
    uint32_t *const jhphi = want_hits ? P.jhphi + wave * cap_h : nullptr;
    int32_t *const jnp = want_tree ? P.jnp + wave * cap_n : nullptr;
    int32_t *const jng = want_tree ? P.jng + wave * cap_n : nullptr;
    float *const jnx = want_tree ? P.jnx + wave * cap_n : nullptr;
    float *const jny = want_tree ? P.jny + wave * cap_n : nullptr;
    float *const jnz = want_tree ? P.jnz + wave * cap_n : nullptr;
    uint32_t *const jne = want_tree ? P.jne + wave * cap_n : nullptr;
    uint32_t *const jnplo = want_tree ? P.jnplo + wave * cap_n : nullptr;
    uint32_t *const jnphi = want_tree ? P.jnphi + wave * cap_n : nullptr;

    const int N = P.n_planes;
    for (;;) {
        int item = 0;
        if (lane == 0) item = (int)atomicAdd(&P.ctr[CTR_WORK], 1ull);
        item = wave_uniform(__shfl(item, 0, WAVE));
        if (item >= P.n) break;
        const int i = P.order ? wave_uniform(P.order[item]) : item;
        const uint32_t sid = P.sid_base + (uint32_t)i;

        // ---- initial condition (section "Using SUPA": energy, angle, impact point)
        const float sc = P.e0[i] * P.e_scale;
        if (!(sc >= 0.0f) || !(sc < 4294967296.0f)) {
            if (lane == 0) {
                atomicOr(&P.ctr[CTR_FLAGS], (unsigned long long)FLAG_RANGE);
                for (int q = 0; q < 4; ++q) P.ledger[4 * (int64_t)i + q] = 0;
                for (int q = 0; q < 6; ++q) P.counts[6 * (int64_t)i + q] = 0;
            }
            continue;
        }
        const uint32_t e_first = (uint32_t)rintf(sc);
        float sp, cp, sa, ca;
        sincosf(P.polar[i], &sp, &cp);
        sincosf(P.azimuth[i], &sa, &ca);
        const bool fwd0 = cp > 0.0f;
        const float tpol = sp / cp;
        const float x_first = P.x0 ? P.x0[i] : 0.0f;
        const float y_first = P.y0 ? P.y0[i] : 0.0f;

        if (lane == 0 && fwd0) {
            fx[0] = x_first;
            fy[0] = y_first;
            ftx[0] = tpol * ca;
            fty[0] = tpol * sa;
            fe[0] = e_first;
            fplo[0] = 1u;
            fphi[0] = 0u;
            fnode[0] = 0;
        }
        if (lane == 0 && want_tree) {
            jnp[0] = -1;
            jng[0] = 0;
            jnx[0] = x_first;
            jny[0] = y_first;
            jnz[0] = 0.0f;
            jne[0] = e_first;
            jnplo[0] = 1u;
            jnphi[0] = 0u;
        }
        int n_cur = fwd0 ? 1 : 0;
        int n_hits = 0, n_nodes = 1, n_splits = 0, max_front = n_cur;
        uint64_t e_stop = 0, e_cut = 0, e_esc = 0;
        int steps = 0, escaped = 0, backward = 0;
        if (!fwd0 && lane == 0) {
            e_esc = e_first;
            escaped = 1;
            backward = 1;
        }
        bool overflow = false;
        int plane_start = 0;     // lane k: first journal hit of plane k
        int cur = 0;
        __threadfence_block();

        for (int k = 0; k < N; ++k) {
            if ((int)lane == k) plane_start = n_hits;
            const float h = (k == 0) ? P.z_first : P.dz;
            const int layer = P.layer[k];
            const uint64_t c1 = P.c1[k], c2 = P.c2[k];
            const bool last = (k == N - 1);
            const int64_t rb = (int64_t)cur * cap_f, wb = (int64_t)(cur ^ 1) * cap_f;
            const int n_read = n_cur < (int)cap_f ? n_cur : (int)cap_f;
            int n_next = 0;
            for (int base = 0; base < n_read; base += WAVE) {
                const int j = base + (int)lane;
                const bool valid = j < n_read;
                float x = 0.f, y = 0.f, tx = 0.f, ty = 0.f;
                uint32_t e = 0, plo = 0, phi = 0;
                int node = 0;
                if (valid) {
                    x = fx[rb + j];
                    y = fy[rb + j];
                    tx = ftx[rb + j];
                    ty = fty[rb + j];
                    e = fe[rb + j];
                    plo = fplo[rb + j];
                    phi = fphi[rb + j];
                    node = fnode[rb + j];
                }
                // free flight to plane k
                x = fmaf(h, tx, x);
                y = fmaf(h, ty, y);
                steps += valid ? 1 : 0;

                // threshold, then the three-way choice on one Philox block
                const bool is_cut = valid && (uint64_t)e < P.t_cut;
                uint4 w = make_uint4(0u, 0u, 0u, 0u);
                const bool draw = valid && !is_cut;
                if (draw) w = philox4x32_10((uint32_t)k, sid, plo, phi, P.seed_lo, P.seed_hi);
                const bool is_stop = draw && (uint64_t)w.x < c1;
                const bool is_split = draw && !is_stop && (uint64_t)w.x < c2;
                const bool is_pass = draw && !is_stop && !is_split;

                // hits: journal in creation order
                const bool is_hit = is_cut || is_stop;
                const uint64_t mh = wave_ballot(is_hit);
                if (is_hit) {
                    if (is_cut) e_cut += e; else e_stop += e;
                    if (want_hits) {
                        const int pos = n_hits + (int)lanes_below(mh);
                        if (pos < (int)cap_h) {
                            jhx[pos] = x;
                            jhy[pos] = y;
                            jhe[pos] = e;
                            jhl[pos] = layer;
                            jhplo[pos] = plo;
                            jhphi[pos] = phi;
                        } else {
                            overflow = true;
                        }
                    }
                }
                n_hits += (int)__popcll(mh);

                // splits: two daughters, two tree nodes
                Daughters D;
                D.fwd_a = D.fwd_b = false;
                D.ea = D.eb = 0;
                D.txa = D.tya = D.txb = D.tyb = 0.f;
                if (is_split) D = split_particle(P, tx, ty, e, w);
                const uint64_t ms = wave_ballot(is_split);
                const int node_a = n_nodes + 2 * (int)lanes_below(ms);
                if (is_split && want_tree) {
                    if (node_a + 1 < (int)cap_n) {
                        const float zk = P.z_first + (float)k * P.dz;
                        jnp[node_a] = node;
                        jnp[node_a + 1] = node;
                        const int gen = 63 - __clzll(((uint64_t)phi << 32) | plo);
                        jng[node_a] = gen + 1;
                        jng[node_a + 1] = gen + 1;
                        jnx[node_a] = x;
                        jnx[node_a + 1] = x;
                        jny[node_a] = y;
                        jny[node_a + 1] = y;
                        jnz[node_a] = zk;
                        jnz[node_a + 1] = zk;
                        jne[node_a] = D.ea;
                        jne[node_a + 1] = D.eb;
                        const uint64_t pa = (((uint64_t)phi << 32) | plo) << 1;
                        jnplo[node_a] = (uint32_t)pa;
                        jnphi[node_a] = (uint32_t)(pa >> 32);
                        jnplo[node_a + 1] = (uint32_t)pa | 1u;
                        jnphi[node_a + 1] = (uint32_t)(pa >> 32);
                    } else {
                        overflow = true;
                    }
                }
                n_nodes += 2 * (int)__popcll(ms);
                n_splits += (int)__popcll(ms);

                // particles for plane k+1 (or leaking out after the last plane)
                const bool out_a = !last && ((is_split && D.fwd_a) || is_pass);
                const bool out_b = !last && is_split && D.fwd_b;
                if (last) {
                    if (is_pass) { e_esc += e; escaped += 1; }
                    if (is_split) { e_esc += (uint64_t)D.ea + D.eb; escaped += 2; }
                } else if (is_split) {
                    if (!D.fwd_a) { e_esc += D.ea; escaped += 1; backward += 1; }
                    if (!D.fwd_b) { e_esc += D.eb; escaped += 1; backward += 1; }
                }
                const uint64_t m1 = wave_ballot(out_a), m2 = wave_ballot(out_b);
                const int pos = n_next + (int)lanes_below(m1) + (int)lanes_below(m2);
                if (out_a || out_b) {
                    const uint64_t path = ((uint64_t)phi << 32) | plo;
                    const int pa = pos, pb = pos + (out_a ? 1 : 0);
                    if (out_a) {
                        if (pa < (int)cap_f) {
                            fx[wb + pa] = x;
                            fy[wb + pa] = y;
                            if (is_split) {
                                ftx[wb + pa] = D.txa;
                                fty[wb + pa] = D.tya;
                                fe[wb + pa] = D.ea;
                                fplo[wb + pa] = (uint32_t)(path << 1);
                                fphi[wb + pa] = (uint32_t)(path >> 31);
                                fnode[wb + pa] = node_a;
                            } else {
                                ftx[wb + pa] = tx;
                                fty[wb + pa] = ty;
                                fe[wb + pa] = e;
                                fplo[wb + pa] = plo;
                                fphi[wb + pa] = phi;
                                fnode[wb + pa] = node;
                            }
                        } else {
                            overflow = true;
                        }
                    }
                    if (out_b) {
                        if (pb < (int)cap_f) {
                            fx[wb + pb] = x;
                            fy[wb + pb] = y;
                            ftx[wb + pb] = D.txb;
                            fty[wb + pb] = D.tyb;
                            fe[wb + pb] = D.eb;
                            fplo[wb + pb] = (uint32_t)(path << 1) | 1u;
                            fphi[wb + pb] = (uint32_t)(path >> 31);
                            fnode[wb + pb] = node_a + 1;
                        } else {
                            overflow = true;
                        }
                    }
                }
                n_next += (int)__popcll(m1) + (int)__popcll(m2);
            }
            // the next plane reads what other lanes of this wave just wrote
            __threadfence_block();
            n_cur = n_next;
            max_front = max_front > n_cur ? max_front : n_cur;
            cur ^= 1;
        }
        if ((int)lane == N) plane_start = n_hits;
        if (n_cur > (int)cap_f) overflow = true;
        const bool wave_overflow = wave_ballot(overflow) != 0;

        // ---- per-shower ledger and counts
        e_stop = wave_sum_u64(e_stop);
        e_cut = wave_sum_u64(e_cut);
        e_esc = wave_sum_u64(e_esc);
        steps = wave_sum_i32(steps);
        escaped = wave_sum_i32(escaped);
        backward = wave_sum_i32(backward);

        long long hit_start = 0, node_start = 0;
        if (lane == 0) {
            P.ledger[4 * (int64_t)i + 0] = e_first;
            P.ledger[4 * (int64_t)i + 1] = e_stop;
            P.ledger[4 * (int64_t)i + 2] = e_cut;
            P.ledger[4 * (int64_t)i + 3] = e_esc;
            int32_t *cnt = P.counts + 6 * (int64_t)i;
            cnt[0] = n_nodes;
            cnt[1] = n_hits;
            cnt[2] = steps;
            cnt[3] = n_splits;
            cnt[4] = escaped;
            cnt[5] = backward;
            atomicAdd(&P.ctr[CTR_STEPS], (unsigned long long)steps);
            if (P.outputs & 1u)
                hit_start = (long long)atomicAdd(&P.ctr[CTR_HITS], (unsigned long long)n_hits);
            if (want_tree)
                node_start = (long long)atomicAdd(&P.ctr[CTR_NODES], (unsigned long long)n_nodes);
            atomicMax(&P.ctr[CTR_NEED_F], (unsigned long long)max_front);
            atomicMax(&P.ctr[CTR_NEED_H], (unsigned long long)n_hits);
            atomicMax(&P.ctr[CTR_NEED_N], (unsigned long long)n_nodes);
            if (wave_overflow) atomicOr(&P.ctr[CTR_FLAGS], (unsigned long long)FLAG_OVERFLOW);
        }
        if (wave_overflow) continue;
        hit_start = __shfl(hit_start, 0, WAVE);
        node_start = __shfl(node_start, 0, WAVE);

        // ---- hit point cloud: copy the journal into the reserved segment
        if (P.outputs & 1u) {
            if (lane == 0) P.hit_offsets[i] = hit_start;
            if (hit_start + n_hits <= P.hit_capacity) {
                for (int j = (int)lane; j < n_hits; j += WAVE) {
                    const int64_t o = hit_start + j;
                    P.hit_x[o] = jhx[j];
                    P.hit_y[o] = jhy[j];
                    P.hit_e[o] = (float)jhe[j] * P.e_unscale;
                    P.hit_layer[o] = jhl[j];
                    if (P.hit_key) P.hit_key[o] = ((uint64_t)jhphi[j] << 32) | jhplo[j];
                }
            }
        }
        // ---- propagation tree
        if (want_tree) {
            if (lane == 0) P.node_offsets[i] = node_start;
            if (node_start + n_nodes <= P.node_capacity) {
                for (int j = (int)lane; j < n_nodes; j += WAVE) {
                    const int64_t o = node_start + j;
                    P.node_parent[o] = jnp[j];
                    P.node_gen[o] = jng[j];
                    P.node_vx[o] = jnx[j];
                    P.node_vy[o] = jny[j];
                    P.node_vz[o] = jnz[j];
                    P.node_e[o] = (float)jne[j] * P.e_unscale;
                    if (P.node_key) P.node_key[o] = ((uint64_t)jnphi[j] << 32) | jnplo[j];
                }
            }
        }
        // ---- per-layer images (appendix "Downsampling"): integer sums per cell
        if (P.outputs & 2u) {
            const int nx = P.img_nx, ny = P.img_ny, rows = P.img_rows;
            const int64_t img_layer = (int64_t)ny * nx;
            for (int l = 0; l < P.n_layers; ++l) {
                float *img = P.images + ((int64_t)i * P.n_layers + l) * img_layer;
                for (int r0 = 0; r0 < ny; r0 += rows) {
                    const int nr = (ny - r0) < rows ? (ny - r0) : rows;
                    const int words = nr * nx;
                    for (int q = (int)lane; q < words; q += WAVE) tile[q] = 0u;
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    for (int k = 0; k < N; ++k) {
                        if (P.layer[k] != l) continue;
                        const int hs = __shfl(plane_start, k, WAVE);
                        const int he = __shfl(plane_start, k + 1, WAVE);
                        for (int j = hs + (int)lane; j < he; j += WAVE) {
                            const float cx = floorf((jhx[j] - P.img_x0) * P.img_sx);
                            const float cy = floorf((jhy[j] - P.img_y0) * P.img_sy);
                            if (cx >= 0.0f && cx < (float)nx && cy >= (float)r0 &&
                                cy < (float)(r0 + nr)) {
                                atomicAdd(&tile[((int)cy - r0) * nx + (int)cx], jhe[j]);
                            }
                        }
                    }
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    for (int q = (int)lane; q < words; q += WAVE)
                        img[(int64_t)r0 * nx + q] = (float)tile[q] * P.e_unscale;
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                }
            }
        }
    }
}

__global__ void supa_zero_counters(unsigned long long *ctr) {
    if (threadIdx.x < CTR_COUNT) ctr[threadIdx.x] = 0ull;
}

__global__ void supa_philox_kernel(const uint32_t *ctr, int64_t n, uint32_t k0, uint32_t k1,
                                   uint32_t *out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const uint4 w = philox4x32_10(ctr[4 * t], ctr[4 * t + 1], ctr[4 * t + 2], ctr[4 * t + 3], k0, k1);
    out[4 * t] = w.x;
    out[4 * t + 1] = w.y;
    out[4 * t + 2] = w.z;
    out[4 * t + 3] = w.w;
}

// ---------------------------------------------------------------------------
// host-side launchers (called by the C ABI in supa_api.cpp)
// ---------------------------------------------------------------------------
hipError_t launch_zero_counters(unsigned long long *ctr, hipStream_t s) {
    hipLaunchKernelGGL(supa_zero_counters, dim3(1), dim3(64), 0, s, ctr);
    return hipGetLastError();
}

hipError_t launch_propagate(const Params &P, int blocks, hipStream_t s) {
    hipLaunchKernelGGL(supa_propagate, dim3(blocks), dim3(WAVE * WAVES_PER_BLOCK), 0, s, P);
    return hipGetLastError();
}

hipError_t launch_philox(const uint32_t *ctr, int64_t n, uint32_t k0, uint32_t k1, uint32_t *out,
                         hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int threads = 256;
    const int64_t blocks = (n + threads - 1) / threads;
    hipLaunchKernelGGL(supa_philox_kernel, dim3((unsigned)blocks), dim3(threads), 0, s, ctr, n, k0,
                       k1, out);
    return hipGetLastError();
}

int waves_per_block() { return WAVES_PER_BLOCK; }
int tile_words() { return TILE_WORDS; }

}  // namespace supa
