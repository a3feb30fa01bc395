"""Throughput of the SUPA propagation path on one MI355X.

One step = every shower of the named workload simulated once (initial
conditions resident in HBM before timing): every particle propagated plane by
plane, hit clouds, per-layer images and (50-plane workload) the propagation
tree written.  The default workload is the largest: 1,000,000 showers, E0
log-uniform on [10, 1000], 50 planes, hits + tree + 50 x 256x256 images, run
in calls of 10,000 showers (its 13 TB of images do not fit one call).
Prints one JSON line (see the keys below).  The CPU oracle is timed on a
random sample of the workload's showers on the host's cores and reported
beside it.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
CU, LANES, CLOCK_GHZ = 256, 64, 2.4
PEAK_ALU_TOPS = CU * LANES * CLOCK_GHZ * 1e9 / 1e12      # 39.3 T lane-ops/s (one op/lane/clock)

# algorithmic lane-operations per unit of work (counted from the method's
# arithmetic, not from compiled code):
OPS_PER_ARRIVAL = 3       # flight (2 fma) + threshold compare
OPS_PER_DRAW = 82         # Philox4x32-10: 10 rounds x (2 mul_hi + 2 mul_lo + 4 xor) + 2 compares
OPS_PER_SPLIT = 65        # energy split, angles, frame, two rotations, two slope divisions
BYTES_PER_HIT = 16        # x, y, E (f32) + layer (i32)
BYTES_PER_NODE = 24       # parent, generation (i32) + vertex x, y, z, E (f32)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=None,
                    help="workload name (default: the 1M-shower 50-plane workload; the 100K "
                         "20-plane one for --shapes, --grids, --kinematics literal and --rings)")
    ap.add_argument("--waves-per-cu", type=int, default=0)
    ap.add_argument("--lds-cap", type=int, default=0,
                    help="frontier entries per buffer kept in LDS (0 = library default)")
    ap.add_argument("--outputs", default="",
                    help="override the workload's outputs: comma list of hits,images,tree")
    ap.add_argument("--sub-batches", type=int, default=0,
                    help="sub-batches whose placement overlaps the next propagation (0: automatic)")
    ap.add_argument("--cost-order", type=int, default=-1, choices=(-1, 0, 1),
                    help="hand out expensive showers first (1), batch order (0), automatic (-1)")
    ap.add_argument("--graph", action="store_true",
                    help="time replays of a captured HIP graph of the call")
    ap.add_argument("--chunk", type=int, default=0,
                    help="showers per call for the workload whose outputs do not fit one call "
                         "(0: 10000)")
    ap.add_argument("--serial-calls", action="store_true",
                    help="run that workload's calls one supa_simulate at a time instead of "
                         "supa_simulate_batches (propagation of call j+1 beside the placement of j)")
    ap.add_argument("--subtrees", type=int, default=None,
                    help="propagation launches per call with subtree work items (0 automatic, the "
                         "library default; 1 none; 2..4)")
    ap.add_argument("--autotune", action="store_true",
                    help="pick launch settings by measurement before timing")
    ap.add_argument("--kinematics", default="3d", choices=("3d", "literal"),
                    help="3-D flight (default) or Algorithm 1's literal displacement kinematics")
    ap.add_argument("--rings", type=int, default=0,
                    help="regional parameters: this many rings (2..4) at radii 0.05, 0.15, 0.4, "
                         "every ring with the workload's probabilities (measures the ring lookup)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="wall time of the oracle's host-CPU baseline (all cores)")
    ap.add_argument("--cpu-seconds-1t", type=float, default=4.0,
                    help="wall time of the oracle's one-thread leg")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 1 GiB device copy (reference for HBM counters)")
    ap.add_argument("--surrogate", action="store_true",
                    help="train the surrogate online, then time surrogate + fallback against "
                         "the plain simulator at the W1 <= 2%% target")
    ap.add_argument("--shapes", action="store_true",
                    help="time the shower-shape-variable kernel (and the normalised W1 between "
                         "two simulated samples) on the workload's hit clouds")
    ap.add_argument("--bins", type=int, default=100, help="histogram bins of the W1 (--shapes)")
    ap.add_argument("--grids", action="store_true",
                    help="time per-layer grid images (CaloGAN-like 3x96 / 12x12 / 12x6 at 1x, 2x, 3x) "
                         "of the workload's hit clouds read out as three layers")
    ap.add_argument("--scale", type=int, default=3, help="grid resolution timed for the line (--grids)")
    ap.add_argument("--train-showers", type=int, default=10_000_000)
    ap.add_argument("--eval-showers", type=int, default=1_000_000)
    ap.add_argument("--batch", type=int, default=8192)
    a = ap.parse_args()
    if a.workload is None:
        side = a.shapes or a.grids or a.kinematics != "3d" or a.rings >= 2
        a.workload = "e1to100_20planes_img32_100k" if side else "loge10to1000_50planes_tree_img256_1m"
    return a


def host_cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads() -> int:
    """Threads for the oracle's all-core leg: the CPUs this process may run
    on, capped by OMP_NUM_THREADS when set (the host's share for one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    cap = os.environ.get("OMP_NUM_THREADS")
    if cap and cap.isdigit() and int(cap) > 0:
        n = min(n, int(cap))
    return max(1, n)


def _oracle_showers(wname, geom, ids, seconds: float, images: bool):
    """One host process: the oracle on the showers `ids` of workload wname in
    order (each its own call, with its global shower id; the list is taken
    again from the start if it runs out) until `seconds` have passed:
    simulation with the tree, plus the per-layer images when asked.  Returns
    (showers done, particle-steps, elapsed s)."""
    from oracle import supa_oracle as O
    from paper_2202_05012_amd import workloads
    w = workloads.WORKLOADS[wname]
    e0, pol, az = workloads.initial_conditions(w)
    L = int(max(geom["layer_of_plane"])) + 1 if geom.get("layer_of_plane") else int(geom["n_planes"])
    showers = steps = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        i = int(ids[showers % len(ids)])
        r = O.simulate(geom, e0[i:i + 1], pol[i:i + 1], az[i:i + 1], w.seed, shower_id_base=i)
        if images:
            O.images(r, L, geom["img_nx"], geom["img_ny"], geom["img_x0"], geom["img_x1"],
                     geom["img_y0"], geom["img_y1"])
        showers += 1
        steps += int(r["counts"][:, 2].sum())
    return showers, steps, time.perf_counter() - t0


def _oracle_showers_star(args):
    return _oracle_showers(*args)


def oracle_sample_rate(w, geom, ids, procs: int, seconds: float, images: bool):
    """The oracle on the showers `ids` of workload w for `seconds` of wall
    time, in this process (procs = 1) or in `procs` host processes started
    for it, each taking every procs-th shower of `ids` (processes, not
    threads: the oracle's Python parts hold the interpreter lock, and threads
    of one process ran slower together than one alone).  Returns (showers
    done, particle-steps, elapsed s of the slowest process)."""
    if procs <= 1:
        return _oracle_showers(w.name, geom, ids, seconds, images)
    import multiprocessing as mp
    parts = [(w.name, geom, ids[q::procs], seconds, images) for q in range(procs)]
    with mp.get_context("spawn").Pool(procs) as pool:
        res = pool.map(_oracle_showers_star, parts)
    return sum(r[0] for r in res), sum(r[1] for r in res), max(r[2] for r in res)


def cpu_baseline_sampled(w, geom, seconds: float, seconds_1t: float, images: bool):
    """The oracle timed on a random subset of the workload's showers (drawn
    uniformly over all of them, so the per-shower mean of the subset
    estimates the workload's), once in one host process per host core and
    once in this process alone; the showers/s of the whole workload is
    extrapolated from the subset's per-shower rate."""
    ids = np.random.default_rng(20260).permutation(w.n)
    threads = host_threads()        # host processes of the all-core leg
    n1, s1, t1 = oracle_sample_rate(w, geom, ids, 1, seconds_1t, images)
    # the all-thread leg takes showers the one-thread leg did not (a small
    # workload it exhausted is taken again from the start)
    rest = ids[n1:] if n1 < len(ids) else ids
    n, steps, dt = oracle_sample_rate(w, geom, rest, threads, seconds, images)
    what = "simulation + tree" + (" + per-layer images" if images else "")
    return {"value": round(n / dt, 2), "unit": "showers/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} showers drawn at random from the {w.n:,}" +
                      (" in repeated passes" if n > len(rest) else "") +
                      f" ({what}, one oracle call per shower) in {threads} host processes for {dt:.1f} s; "
                      f"rate extrapolated per shower to the whole workload",
            "extrapolated": True, "seconds": round(dt, 2),
            "particle_steps_per_s": round(steps / dt, 1),
            "one_thread": {"value": round(n1 / t1, 2), "unit": "showers/s", "showers": n1,
                           "seconds": round(t1, 2), "particle_steps_per_s": round(s1 / t1, 1)},
            "workload_seconds_all_threads": round(w.n / (n / dt), 1),
            "cpu_model": host_cpu_model(), "host_cpus": os.cpu_count()}


def bench_surrogate(args):
    """Surrogate + fallback against the plain simulator (per-layer energies
    of the 20-plane workload's distribution, over a 10 x 10 window): two
    networks are trained online on the same simulated showers -- the image
    model (mean and log-variance of each cell of 20 x 16 x 16 images) and the
    per-layer head (of each of the 20 per-layer energies) -- then on held-out
    initial conditions the showers whose predicted uncertainty is above a
    threshold are simulated instead.  The judge (on the GPU) is the W1 of the
    per-layer energies (and, for the image model, of the occupied cells)
    against the simulator's on the same initial conditions.  Each pipeline is
    compared with the simulator producing what it produces: 16 x 16 images
    (energies and occupied cells) for the image model, one cell per layer
    (the energies alone) for the head.  The line's value is the fastest
    surrogate + fallback rate that meets W1 <= 2% of the mean per-layer
    energy; roofline: the fused final layer + gate of the image model (the
    largest matrix-core product); cpu_baseline: the oracle's forward pass."""
    import torch
    from paper_2202_05012_amd import surrogate as S, surrogate_pipeline as SP
    dev = torch.device("cuda", 0)
    sim = SP.ImageSimulator()
    sim1 = SP.ImageSimulator(grid=1)
    model = S.MLP(S.surrogate_dims(), device=dev, seed=1)
    head = S.MLP(SP.layer_head_dims(), device=dev, seed=2)
    steps = max(1, args.train_showers // args.batch)
    losses, head_losses, t_train = SP.train(model, steps, args.batch, seed=7, lr=1e-3,
                                            log_every=max(1, steps // 10), sim=sim, head=head)
    print(f"trained: {steps} steps of {args.batch} showers in {t_train:.1f} s", file=sys.stderr, flush=True)
    rho = SP.calibrate_rho(model, sim, 8192, seed=11)
    n = args.eval_showers
    e0, pol, az = SP.draw_ics(n, 12345, dev)

    def timed(fn, reps=1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            r = fn()
        torch.cuda.synchronize()
        return r, (time.perf_counter() - t0) / reps

    # warm-up at full size: the simulators' logs and the caching allocator
    # reach their sizes before anything is timed
    SP.simulated_layer_energies(e0, pol, az, 3, sim, counts=True)
    SP.simulated_layer_energies(e0, pol, az, 3, sim1)
    SP.surrogate_layer_energies(model, e0, pol, az, 5, rho=rho, counts=True)
    SP.head_layer_energies(head, e0, pol, az, 5)
    (ref_e, ref_c), t_sim = timed(lambda: SP.simulated_layer_energies(e0, pol, az, 3, sim, counts=True), 3)
    _, t_sim1 = timed(lambda: SP.simulated_layer_energies(e0, pol, az, 3, sim1), 3)
    (sur_e, unc, sur_c), t_sur = timed(lambda: SP.surrogate_layer_energies(model, e0, pol, az, 5, rho=rho,
                                                                           counts=True), 3)
    (_, hunc), t_head = timed(lambda: SP.head_layer_energies(head, e0, pol, az, 5), 3)

    def tau_of(u, frac):
        return float(np.quantile(u, 1.0 - frac)) if 0 < frac < 1 else (np.inf if frac == 0 else -np.inf)

    rows, hrows = [], []
    unc_h = unc.cpu().numpy()
    for frac in (0.0, 0.1, 0.3, 0.5, 0.6, 0.7, 0.75, 0.8, 0.85, 0.9, 0.95, 1.0):
        tau = tau_of(unc_h, frac)
        (le, lc, m), t = timed(lambda: SP.surrogate_with_fallback(model, e0, pol, az, 5, tau, sim, rho=rho))
        w, wc, _, _ = SP.judge(le, lc, ref_e, ref_c)
        rows.append({"model": "image", "fallback_frac": m / n, "tau": tau, "seconds": t,
                     "showers_per_s": n / t, "w1_energy_max_rel": w, "w1_occupied_max_rel": wc})
    hunc_h = hunc.cpu().numpy()
    for frac in (0.0, 0.1, 0.3, 0.5, 0.8, 1.0):
        tau = tau_of(hunc_h, frac)
        SP.head_with_fallback(head, e0, pol, az, 5, tau, sim1)
        (le, m), t = timed(lambda: SP.head_with_fallback(head, e0, pol, az, 5, tau, sim1), 3)
        w = SP.judge(le, ref_c, ref_e, ref_c)[0]
        hrows.append({"model": "layer_head", "fallback_frac": m / n, "tau": tau, "seconds": t,
                      "showers_per_s": n / t, "w1_energy_max_rel": w})
    print("fallback sweeps done", file=sys.stderr, flush=True)
    ok = [r for r in rows + hrows if r["w1_energy_max_rel"] <= 0.02]
    best = max(ok, key=lambda r: r["showers_per_s"]) if ok else None
    plain = {"image": n / t_sim, "layer_head": n / t_sim1}

    if args.copy_calibration:
        # one device copy of exactly 1 GiB: what the HBM counters read for it
        # calibrates them (see prof_summary)
        ca = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        cb = torch.empty_like(ca)
        cb.copy_(ca)
        torch.cuda.synchronize()
        del ca, cb
    # roofline of the dominant kernel: the final layer's product fused into
    # the gate (gate_fused_k256_kernel, two launches per call: the mean tiles
    # then the log-variance tiles, 2 B K D flops each), timed with the HIP
    # events the library records on the launch stream
    from paper_2202_05012_amd import prof_summary
    B = 65536
    x = S.features(e0[:B], pol[:B], az[:B], 5, stream_id=2)
    h = model.hidden(x)
    wt = model.final_weights_t()
    K, D2 = h.shape[1], wt.shape[0]
    for _ in range(3):
        S.gate_fused(h, wt, model.b[-1], e0[:B], SP.N_LAYERS, rho=rho)
    S.timing(True)
    times = []
    for _ in range(20):
        S.gate_fused(h, wt, model.b[-1], e0[:B], SP.N_LAYERS, rho=rho)
        times.append(S.last_times())
    S.timing(False)
    t_mean = float(np.mean([t[0] for t in times]))
    t_var = float(np.mean([t[1] for t in times]))
    t_gate = float(np.mean([t[2] for t in times]))
    k_ms = (t_mean + t_var) / 2
    flops = 2.0 * B * K * (D2 // 2)
    tf = flops / (k_ms / 1e3) / 1e12
    workload_name = "surrogate_20layers_16x16"
    traffic = prof_summary.traffic_if_current(os.path.join(ROOT, "profiles"), "gate_fused_k256_kernel", workload_name)
    # the per-layer head's whole forward pass in one kernel (mlp_fused_kernel)
    # over 2^20 rows, timed with events on the stream it is launched on
    # (torch's current stream); algorithmic flops from the network's own
    # widths (19 inputs, not the zero-padded 32)
    Bh = 1 << 20
    eh, ph, ah = SP.draw_ics(Bh, 54321, dev)
    xh_in = S.features(eh, ph, ah, 5, stream_id=2)
    for _ in range(3):
        head.forward_fused(xh_in)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    h_times = []
    for _ in range(20):
        ev0.record()
        head.forward_fused(xh_in)
        ev1.record()
        ev1.synchronize()
        h_times.append(ev0.elapsed_time(ev1))
    h_ms = float(np.mean(h_times))
    hdims = [S.IN_FEATURES + S.N_NOISE] + SP.layer_head_dims()[1:]
    h_flops = 2.0 * Bh * sum(hdims[i] * hdims[i + 1] for i in range(len(hdims) - 1))
    h_tf = h_flops / (h_ms / 1e3) / 1e12
    h_workload = "surrogate_layer_head_1m_rows"
    h_traffic = prof_summary.traffic_if_current(os.path.join(ROOT, "profiles"), "mlp_fused_kernel", h_workload)
    del eh, ph, ah, xh_in
    line = {
        "metric": "surrogate+fallback showers/s at W1 <= 2% of the mean per-layer energy",
        "value": round(best["showers_per_s"], 1) if best else None,
        "unit": "showers/s", "n_gpus": 1, "higher_is_better": True, "vs_baseline": None,
        "dtype": "bf16 mfma (f32 accumulate) + f32/u32 simulation", "data": "synthetic",
        "config": {"workload": workload_name, "eval_showers": n,
                   "train_showers": steps * args.batch, "batch": args.batch,
                   "mlp": "19 -> 4x256 GELU -> 10240", "layer_head": "19 -> 4x256 GELU -> 40",
                   "occupied_cell_threshold": SP.OCC_THR},
        "plain_simulator_showers_per_s": {"images_16x16": round(n / t_sim, 1),
                                          "layer_energies": round(n / t_sim1, 1)},
        "surrogate_only_showers_per_s": {"image": round(n / t_sur, 1), "layer_head": round(n / t_head, 1)},
        "beats_plain_simulator": bool(best and best["showers_per_s"] > plain[best["model"]]),
        "speedup_over_plain_simulator": round(best["showers_per_s"] / plain[best["model"]], 2) if best else None,
        "roofline": {"bound": "mfma", "achieved": round(tf, 2), "peak": 2500.0, "unit": "TFLOP/s",
                     "frac": round(tf / 2500.0, 4), "traffic": traffic,
                     "kernel": "gate_fused_k256_kernel (final layer product + tile sums; per launch half the "
                               "columns: means, then log-variances)",
                     "kernel_ms": round(k_ms, 4), "launch_ms": {"means": round(t_mean, 4), "log_variances":
                                                                 round(t_var, 4), "gate_rows": round(t_gate, 4)},
                     "alg_flops": flops, "rows": B},
        "roofline_head": {"bound": "mfma", "achieved": round(h_tf, 2), "peak": 2500.0, "unit": "TFLOP/s",
                          "frac": round(h_tf / 2500.0, 4), "traffic": h_traffic,
                          "kernel": "mlp_fused_kernel (the per-layer head's forward pass, "
                                    "19 -> 4x256 GELU -> 40, in one launch)",
                          "kernel_ms": round(h_ms, 4), "alg_flops": h_flops, "rows": Bh,
                          "profile_workload": h_workload},
        "train_seconds": round(t_train, 2), "loss_curve": losses, "head_loss_curve": head_losses,
        "rho": rho, "chosen": best, "sweep": rows, "sweep_layer_head": hrows,
    }
    if not args.no_cpu_baseline:
        # the oracle's forward pass (FP64) of the same network on a sample of
        # the held-out rows, for about --cpu-seconds
        from oracle import surrogate_oracle as SO
        Wf = [S.bf16_to_float(w).cpu().numpy().astype(np.float64) for w in model.Wb]
        bf = [b.cpu().numpy().astype(np.float64) for b in model.b]
        params = [[W, b] for W, b in zip(Wf, bf)]
        xh = S.bf16_to_float(x).cpu().numpy().astype(np.float64)
        done, t_cpu, blk = 0, 0.0, 1024
        while t_cpu < args.cpu_seconds:
            c0 = time.perf_counter()
            SO.forward(params, xh[(done % B):(done % B) + blk])
            t_cpu += time.perf_counter() - c0
            done += blk
        line["cpu_baseline"] = {"value": round(done / t_cpu, 1), "unit": "showers/s",
                                "cores": host_threads(), "kind": "oracle",
                                "sample": f"oracle forward pass (FP64 numpy) of {done} held-out rows in blocks of "
                                          f"{blk}, {t_cpu:.1f} s; numpy's BLAS threads",
                                "cpu_model": host_cpu_model()}
    print(json.dumps(line), flush=True)


def bench_shapes(args):
    """Shower shape variables (supa_shower_shapes) of one simulated sample of
    the workload, and the normalised W1 of every variable between it and a
    second sample (supa_w1_normalized).  The hits are simulated once, before
    anything is timed; a step is one shape-variable call over the batch."""
    import torch
    from paper_2202_05012_amd import prof_summary, shapes as SH, supa, workloads
    from oracle import shape_oracle

    w = workloads.WORKLOADS[args.workload]
    geom = workloads.geometry(w)
    L = supa.n_layers(geom)
    dev = torch.device("cuda", 0)
    sim = supa.Simulator(geom, supa.OUT_HITS)
    samples = []
    for k, seed in enumerate((w.seed, w.seed + 1)):
        e0, pol, az = workloads.initial_conditions(w, seed=seed)
        t = [torch.from_numpy(a).to(dev) for a in (e0, pol, az)]
        samples.append(sim.simulate(*t, seed=seed, shower_id_base=k * w.n))
    del sim
    out = samples[0]
    n = w.n
    hits = int(out["total_hits"])
    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    # the second sample's variables (W1 below), then the timed sample checked
    # once for the layer rule: dispatches 0 and 1 of the shape kernel
    lv1, sv1 = SH.simulator_shapes(samples[1], L, check=True)
    SH.simulator_shapes(out, L, check=True)
    for _ in range(args.warmup):
        SH.simulator_shapes(out, L, check=False)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        lv, sv = SH.simulator_shapes(out, L, check=False)
    ev1.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    k_ms = ev0.elapsed_time(ev1) / args.steps
    cols = L * len(SH.LAYER_VARS) + len(SH.SHOWER_VARS)
    alg = BYTES_PER_HIT * hits + n * (8 + 4 + cols * 4)
    prof_dir = os.path.join(ROOT, "profiles")
    wl = "shapes_" + w.name
    gbs = alg / (k_ms / 1e3) / 1e9
    roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(gbs / PEAK_HBM_GBS, 4),
            "traffic": prof_summary.traffic_if_current(prof_dir, "shapes_kernel", wl),
            "kernel": "shapes_kernel", "kernel_ms": round(k_ms, 4), "alg_bytes": alg}

    # normalised W1 of every variable, sample 1 against sample 0 (reference)
    mats = [torch.cat([a.view(n, -1), b], dim=1).contiguous() for a, b in ((lv, sv), (lv1, sv1))]
    groups = torch.cat([torch.arange(len(SH.LAYER_VARS)).repeat(L),
                        len(SH.LAYER_VARS) + torch.arange(len(SH.SHOWER_VARS))]).int().to(dev)
    ws = SH.W1Workspace(dev)
    n_groups = len(SH.LAYER_VARS) + len(SH.SHOWER_VARS)
    for _ in range(max(1, args.warmup)):
        SH.w1_columns(mats[0], mats[1], args.bins, groups, n_groups, ws)
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(args.steps):
        d, gm = SH.w1_columns(mats[0], mats[1], args.bins, groups, n_groups, ws)
    ev1.record()
    torch.cuda.synchronize()
    w1_ms = ev0.elapsed_time(ev1) / args.steps
    w1_bytes = 2 * 2 * n * cols * 4                   # two passes (range, histogram) over both
    tr = [prof_summary.traffic_if_current(prof_dir, k, wl) for k in ("w1_stats", "w1_hist")]
    w1_traffic = None if None in tr else 2 * (tr[0] + tr[1])   # each kernel runs once per sample
    gm_h = gm.cpu().numpy()
    # the groups of marginals of the paper's performance table (untimed): the
    # per-layer variables grouped across layers, and the point-level marginals
    # of eta = x, phi = y, r and E over every hit of each sample
    table = {"feature means <eta>,<phi>,<r>": ("mean_x", "mean_y", "mean_r"), "feature mean <E>": ("mean_e",),
             "deviations of eta, phi, r": ("std_x", "std_y", "std_r"), "deviation of E": ("std_e",),
             "layer energy": ("energy",), "layer centroids": ("centroid_x", "centroid_y", "centroid_r"),
             "layer widths": ("width_x", "width_y", "width_r"),
             "point counts": ("count",), "fraction, energy ratio": ("fraction", "energy_ratio"),
             "shower variables": SH.SHOWER_VARS}
    gidx = {v: g for g, vs in enumerate(table.values()) for v in vs}
    tgroups = torch.tensor([gidx.get(v, -1) for v in SH.LAYER_VARS * L + SH.SHOWER_VARS], dtype=torch.int32, device=dev)
    _, tg = SH.w1_columns(mats[0], mats[1], args.bins, tgroups, len(table), ws)
    md = {k: round(float(v), 5) for k, v in zip(table, tg.cpu().numpy())}
    pts = {}
    for name, key in (("eta", "hit_x"), ("phi", "hit_y"), ("E", "hit_e")):
        pts[name] = float(SH.w1_columns(samples[0][key], samples[1][key], args.bins, workspace=ws)[0].item())
    r0 = SH.hit_radius(samples[0]["hit_x"], samples[0]["hit_y"])
    r1 = SH.hit_radius(samples[1]["hit_x"], samples[1]["hit_y"])
    pts["r"] = float(SH.w1_columns(r0, r1, args.bins, workspace=ws)[0].item())
    md["point features eta, phi, r"] = round((pts["eta"] + pts["phi"] + pts["r"]) / 3, 5)
    md["point feature E"] = round(pts["E"], 5)
    line = {
        "metric": "shower-shape-variable showers/s (1 MI355X)",
        "value": round(n / (ms_per_step / 1e3), 1),
        "unit": "showers/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64 sums, f32 out", "data": "synthetic",
        "config": {"workload": wl, "showers": n, "layers": L, "hits": hits,
                   "variables_per_shower": cols},
        "roofline": roof,
        "roofline_other": {"bound": "hbm", "kernel": "w1 (stats + histograms + distance)",
                           "achieved": round(w1_bytes / (w1_ms / 1e3) / 1e9, 1),
                           "peak": PEAK_HBM_GBS, "unit": "GB/s",
                           "frac": round(w1_bytes / (w1_ms / 1e3) / 1e9 / PEAK_HBM_GBS, 4),
                           "traffic": w1_traffic, "ms": round(w1_ms, 4), "alg_bytes": w1_bytes,
                           "bins": args.bins, "columns": cols},
        "mean_discrepancy_by_variable": {k: round(float(v), 5) for k, v in
                                         zip(SH.LAYER_VARS + SH.SHOWER_VARS, gm_h)},
        "mean_discrepancy_by_group": md,
    }
    if not args.no_cpu_baseline:
        # the oracle's shape variables of the first showers, for about
        # --cpu-seconds of one host core
        off = out["hit_offsets"].cpu().numpy()
        cnt = out["counts"][:, 1].cpu().numpy().astype(np.int64)
        m = 1
        done, t_cpu = 0, 0.0
        while t_cpu < args.cpu_seconds and done < n:
            m = min(2 * m, n - done)
            a, b = int(off[done]), int(off[done + m - 1] + cnt[done + m - 1])
            hx, hy, he, hl = (out[k][a:b].cpu().numpy() for k in ("hit_x", "hit_y", "hit_e", "hit_layer"))
            sid = np.repeat(np.arange(m), cnt[done:done + m])
            keep = hl >= 0
            c0 = time.perf_counter()
            shape_oracle.shapes(m, L, sid[keep], hl[keep], hx[keep].astype(np.float64),
                                hy[keep].astype(np.float64), he[keep].astype(np.float64))
            t_cpu += time.perf_counter() - c0
            done += m
        line["cpu_baseline"] = {"value": round(done / t_cpu, 1), "unit": "showers/s", "cores": 1,
                                "kind": "oracle",
                                "sample": f"shape variables of the first {done} showers "
                                          f"({t_cpu:.1f} s, one thread)"}
    print(json.dumps(line), flush=True)


def bench_grids(args):
    """Per-layer grid images (supa_bin_grids) of one simulated sample of the
    workload read out as three layers (sub-layers 2-5, 6-13, 14-19; 0-1 dead),
    on the CaloGAN-like grids over [-5, 5)^2.  The hits are simulated once,
    before anything is timed; a step is one binning call over the batch."""
    import torch
    from paper_2202_05012_amd import grids as GR, presets, prof_summary, supa, workloads
    from oracle import supa_oracle

    w = workloads.WORKLOADS[args.workload]
    geom = dict(workloads.geometry(w), layer_of_plane=[-1] * 2 + [0] * 4 + [1] * 8 + [2] * 6)
    if w.n_planes != 20:
        sys.exit("--grids reads out the 20-plane workloads as three layers")
    dev = torch.device("cuda", 0)
    e0, pol, az = workloads.initial_conditions(w)
    sim = supa.Simulator(geom, supa.OUT_HITS)
    out = sim.simulate(*[torch.from_numpy(a).to(dev) for a in (e0, pol, az)], seed=w.seed)
    del sim
    n, hits = w.n, int(out["total_hits"])
    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        torch.empty_like(a).copy_(a)
        torch.cuda.synchronize()
        del a
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    per_scale = {}
    for scale in sorted({1, 2, 3, args.scale}, key=lambda k: k == args.scale):  # timed scale last
        gr = presets.calogan_grids(scale, half_width=5.0)
        for _ in range(max(1, args.warmup)):
            GR.simulator_grids(out, gr)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev0.record()
        for _ in range(args.steps):
            img = GR.simulator_grids(out, gr)
        ev1.record()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        cells = GR.cells(gr)
        alg = BYTES_PER_HIT * hits + n * (12 + 4 * cells)
        k_ms = ev0.elapsed_time(ev1) / args.steps
        per_scale[scale] = {"cells": cells, "ms": round(k_ms, 4), "alg_bytes": alg,
                            "GBps": round(alg / (k_ms / 1e3) / 1e9, 1),
                            "ms_per_step": (t1 - t0) * 1e3 / args.steps}
    r = per_scale[args.scale]
    wl = f"grids{args.scale}x_" + w.name
    prof_dir = os.path.join(ROOT, "profiles")
    line = {
        "metric": f"per-layer grid images showers/s ({args.scale}x CaloGAN-like, 1 MI355X)",
        "value": round(n / (r["ms_per_step"] / 1e3), 1), "unit": "showers/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(r["ms_per_step"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64 sums, f32 out",
        "data": "synthetic",
        "config": {"workload": wl, "showers": n, "hits": hits, "layers": 3, "cells": r["cells"]},
        "roofline": {"bound": "hbm", "achieved": r["GBps"], "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(r["GBps"] / PEAK_HBM_GBS, 4),
                     "traffic": prof_summary.traffic_if_current(prof_dir, "grids_kernel", wl),
                     "kernel": "grids_kernel", "kernel_ms": r["ms"], "alg_bytes": r["alg_bytes"]},
        "scales": {f"{k}x": {kk: vv for kk, vv in v.items() if kk != "ms_per_step"}
                   for k, v in sorted(per_scale.items())},
    }
    if not args.no_cpu_baseline:
        # the oracle's binning of the first showers' hits for about --cpu-seconds
        gr = presets.calogan_grids(args.scale, half_width=5.0)
        off = out["hit_offsets"].cpu().numpy()
        cnt = out["counts"][:, 1].cpu().numpy().astype(np.int64)
        done, t_cpu, m = 0, 0.0, 64
        while t_cpu < args.cpu_seconds and done < n:
            m = min(2 * m, n - done)
            a, b = int(off[done]), int(off[done + m - 1] + cnt[done + m - 1])
            hx, hy, he, hl = (out[k][a:b].cpu().numpy() for k in ("hit_x", "hit_y", "hit_e", "hit_layer"))
            sid = np.repeat(np.arange(m), cnt[done:done + m])
            c0 = time.perf_counter()
            q = np.rint(he.astype(np.float64) * 2.0 ** 21).astype(np.uint64)
            supa_oracle.grid_images(m, sid, hl, hx, hy, q, gr)
            t_cpu += time.perf_counter() - c0
            done += m
        line["cpu_baseline"] = {"value": round(done / t_cpu, 1), "unit": "showers/s", "cores": 1,
                                "kind": "oracle",
                                "sample": f"grid images of the first {done} showers ({t_cpu:.1f} s, one thread)"}
    print(json.dumps(line), flush=True)


def chunk_slices(n: int, chunk: int):
    """(first shower, showers) of each call when n showers run in calls of at
    most `chunk` showers."""
    return [(s0, min(chunk, n - s0)) for s0 in range(0, n, chunk)]


def bench_batched(args, w):
    """A workload whose outputs do not fit one call (1M showers of 50 layers
    of 256x256 images = 13 TB): one step runs every shower in calls of
    --chunk showers.  By default the step is one supa_simulate_batches call
    over all of them (the propagation of call j+1 runs beside the placement
    of call j); the calls share one set of hit, node and image arrays sized
    for one call (a consumer would copy or reduce them between calls), each
    call having its own ledger, counts and offsets.  Timed: K steps after W
    untimed ones."""
    import torch
    from paper_2202_05012_amd import prof_summary, supa, workloads

    geom = workloads.geometry(w)
    outputs = supa.OUT_HITS | supa.OUT_IMAGES | supa.OUT_TREE
    dev = torch.device("cuda", 0)
    e0, pol, az = workloads.initial_conditions(w)
    te0, tpol, taz = (torch.from_numpy(a).to(dev) for a in (e0, pol, az))
    # 10,000 showers per call: 131 GB of images, half of the device's HBM
    chunk = args.chunk if args.chunk > 0 else 10_000
    calls = chunk_slices(w.n, chunk)
    sim = supa.Simulator(geom, outputs, waves_per_cu=args.waves_per_cu, frontier_cap=args.lds_cap,
                         sub_batches=args.sub_batches, cost_order=args.cost_order)

    def per_call_outputs(shared):
        """Each call: ledger, counts and offsets of its own; the hit, node and
        image arrays of `shared`."""
        outs = []
        for _, m in calls:
            o = {k: v for k, v in shared.items()
                 if k not in ("ledger", "counts", "hit_offsets", "node_offsets", "shower_capacity")}
            o.update(ledger=torch.empty((m, 4), dtype=torch.int64, device=dev),
                     counts=torch.empty((m, 6), dtype=torch.int32, device=dev),
                     hit_offsets=torch.empty(m, dtype=torch.int64, device=dev),
                     node_offsets=torch.empty(m, dtype=torch.int64, device=dev), shower_capacity=m)
            outs.append(o)
        return outs

    # capacities: the largest call's totals (zero-capacity outputs: each call
    # reports its totals; this also grows the library's scratch)
    probe = per_call_outputs(sim.allocate(chunk, 0, 0))
    sim.run_batches(te0, tpol, taz, w.seed, calls, probe)
    need_h = max(o["total_hits"] for o in probe)
    need_n = max(o["total_nodes"] for o in probe)
    del probe
    outs = per_call_outputs(sim.allocate(chunk, int(need_h) + 1, int(need_n) + 1))
    print(f"sized: {len(calls)} calls of {chunk} showers, <= {need_h} hits and {need_n} nodes per call",
          file=sys.stderr, flush=True)
    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        torch.empty_like(a).copy_(a)
        torch.cuda.synchronize()
        del a

    def step():
        """One pass over the workload; returns the kernel times (ms) and the
        calls' totals."""
        tot = np.zeros(4, np.int64)            # nodes, hits, steps, splits
        kt = np.zeros(3)
        if args.serial_calls:
            for (s0, m), o in zip(calls, outs):
                sl = slice(s0, s0 + m)
                assert sim.run(te0[sl], tpol[sl], taz[sl], w.seed, o, shower_id_base=s0) == 0
                tm = sim.timing()
                kt += (tm[0], tm[3], tm[4])
        else:
            assert sim.run_batches(te0, tpol, taz, w.seed, calls, outs) == 0
            tm = sim.timing()
            kt += (tm[0], tm[3], tm[4])
        for (s0, m), o in zip(calls, outs):
            # a split adds two nodes to a shower's primary one
            tot += (o["total_nodes"], o["total_hits"], o["total_steps"], (o["total_nodes"] - m) // 2)
        return kt, tot

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print(f"warm-up: {args.warmup} steps done", file=sys.stderr, flush=True)
    kt = np.zeros(3)
    tot = None
    t0 = time.perf_counter()
    for _ in range(args.steps):
        k, tot = step()
        kt += k
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    print(f"timed: {args.steps} steps in {t1 - t0:.2f} s", file=sys.stderr, flush=True)
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    nodes_total, hits_total, steps_total, splits_total = (int(v) for v in tot)
    prop_ms, place_ms, scatter_ms = kt
    launches = args.steps * len(calls)
    k_prop, k_place, k_scatter = prop_ms / launches, place_ms / launches, scatter_ms / launches
    draws = steps_total - hits_total          # p_stop = 0 here: every hit is a cut
    alg_ops = OPS_PER_ARRIVAL * steps_total + OPS_PER_DRAW * draws + OPS_PER_SPLIT * splits_total
    alu = alg_ops / len(calls) / (k_prop / 1e3) / 1e12
    L = supa.n_layers(geom)
    img_bytes = w.n * L * geom["img_nx"] * geom["img_ny"] * 4
    # per launch (average over the step's calls): what the kernel must write
    place_alg = (BYTES_PER_HIT * hits_total + img_bytes) / len(calls)
    scatter_alg = BYTES_PER_NODE * nodes_total / len(calls)
    prof_dir = os.path.join(ROOT, "profiles")

    def hbm(kernel, alg, ms):
        gbs = alg / (ms / 1e3) / 1e9
        return {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(gbs / PEAK_HBM_GBS, 4),
                "traffic": prof_summary.traffic_if_current(prof_dir, kernel, w.name),
                "kernel": kernel, "kernel_ms": round(ms, 4), "alg_bytes": int(alg), "per": "launch",
                "launches_per_step": len(calls)}

    roof_place = hbm("supa_place", place_alg, k_place)
    roof_scatter = hbm("scatter_nodes", scatter_alg, k_scatter)
    roof_prop = {"bound": "alu", "achieved": round(alu, 3), "peak": round(PEAK_ALU_TOPS, 2),
                 "unit": "T lane-ops/s", "frac": round(alu / PEAK_ALU_TOPS, 4),
                 "traffic": prof_summary.traffic_if_current(prof_dir, "supa_propagate", w.name),
                 "kernel": "supa_propagate", "kernel_ms": round(k_prop, 4),
                 "alg_lane_ops": int(alg_ops / len(calls)), "per": "launch", "launches_per_step": len(calls)}
    if not args.serial_calls:
        # pipelined calls: the propagation of call j + 1 runs on its own stream
        # beside the placement of call j, with the wave slots the placement
        # leaves, and a call of this size fills part of the persistent grid
        waves = len(sim.wave_times())             # the last launch's persistent grid
        roof_prop["note"] = (f"runs beside supa_place (off the critical path); {chunk} showers per call "
                             f"fill {(chunk + 3) // 4} of the launch's {waves} four-shower waves")
    kern = sorted([(k_place, roof_place), (k_prop, roof_prop), (k_scatter, roof_scatter)], key=lambda t: -t[0])
    line = {
        "metric": "showers/s (1 MI355X)", "value": round(w.n / (ms_per_step / 1e3), 1), "unit": "showers/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+u32",
        "data": "synthetic",
        "config": {"workload": w.name, "showers": w.n, "planes": w.n_planes, "outputs": "hits+images+tree",
                   "image": f"{L}x{geom['img_ny']}x{geom['img_nx']}",
                   "showers_per_call": chunk, "calls_per_step": len(calls),
                   "calls": "one at a time" if args.serial_calls else "pipelined (supa_simulate_batches)"},
        "particle_steps_per_s": round(steps_total / (ms_per_step / 1e3), 1),
        "particle_steps": steps_total, "hits": hits_total, "nodes": nodes_total,
        "roofline": kern[0][1], "roofline_other": kern[1][1], "roofline_third": kern[2][1],
        "kernel_ms_per_step": {"supa_propagate": round(prop_ms / args.steps, 2),
                               "supa_place": round(place_ms / args.steps, 2),
                               "scatter_nodes": round(scatter_ms / args.steps, 2)},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_sampled(w, geom, args.cpu_seconds, args.cpu_seconds_1t, True)
        print("oracle baseline done", file=sys.stderr, flush=True)
    print(json.dumps(line), flush=True)


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (showers are "
              "independent and keyed by global id, so GPUs would take disjoint shower_id_base "
              "ranges)", file=sys.stderr)
        sys.exit(2)
    if args.surrogate:
        return bench_surrogate(args)
    if args.shapes:
        return bench_shapes(args)
    if args.grids:
        return bench_grids(args)

    import torch
    from paper_2202_05012_amd import supa, workloads

    w = workloads.WORKLOADS[args.workload]
    if w.tree and w.images:
        return bench_batched(args, w)
    geom = workloads.geometry(w)
    geom["kinematics"] = args.kinematics
    wname = w.name + ("" if args.kinematics == "3d" else "_literal") + \
        (f"_rings{args.rings}" if args.rings >= 2 else "")
    if args.rings >= 2:
        R, N = args.rings, int(geom["n_planes"])
        geom.update(n_regions=R, region_r=[0.05, 0.15, 0.4][:R - 1],
                    p_stop=list(geom.get("p_stop") or [0.0] * N) * R,
                    p_split=list(geom.get("p_split") or [1.0] * N) * R)
    outputs = supa.OUT_HITS | (supa.OUT_IMAGES if w.images else 0) | (supa.OUT_TREE if w.tree else 0)
    if args.outputs:
        names = {"hits": supa.OUT_HITS, "images": supa.OUT_IMAGES, "tree": supa.OUT_TREE}
        outputs = 0
        for t in args.outputs.split(","):
            if t and t != "none":
                outputs |= names[t]
    dev = torch.device("cuda", 0)
    e0, pol, az = workloads.initial_conditions(w)
    te0, tpol, taz = (torch.from_numpy(a).to(dev) for a in (e0, pol, az))
    sim = supa.Simulator(geom, outputs, waves_per_cu=args.waves_per_cu,
                         frontier_cap=args.lds_cap, sub_batches=args.sub_batches,
                         cost_order=args.cost_order, subtree_phases=args.subtrees)

    # size the outputs from one untimed run (also grows the per-wave scratch)
    probe = sim.allocate(w.n, 0, 0)
    sim.run(te0, tpol, taz, w.seed, probe)
    out = sim.allocate(w.n, int(probe["total_hits"] * 1.0) + 1, int(probe["total_nodes"]) + 1)
    del probe

    # launch settings picked by measurement on this batch (untimed), unless
    # given on the command line
    launch = None
    if args.autotune:
        launch = sim.autotune(te0, tpol, taz, w.seed, out)

    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    for _ in range(args.warmup):
        st = sim.run(te0, tpol, taz, w.seed, out)
        assert st == 0
    torch.cuda.synchronize()
    prop_ms, post_ms = [], []
    if args.graph:
        # one captured call replayed: no host work between steps
        g = sim.graph(te0, tpol, taz, w.seed, out)
        sim.run(te0, tpol, taz, w.seed, out)          # kernel times of one eager call
        tm = sim.timing()
        prop_ms.append(tm[0])
        post_ms.append(tm[3] if outputs & (supa.OUT_HITS | supa.OUT_IMAGES) else tm[4])
        for _ in range(args.warmup):
            g.launch()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            g.launch()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        g.check()
        st = 0
    else:
        t0 = time.perf_counter()
        for _ in range(args.steps):
            st = sim.run(te0, tpol, taz, w.seed, out)
            tm = sim.timing()
            prop_ms.append(tm[0])
            post_ms.append(tm[3] if outputs & (supa.OUT_HITS | supa.OUT_IMAGES) else tm[4])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    assert st == 0
    ms_per_step = (t1 - t0) * 1e3 / args.steps

    counts = out["counts"].cpu().numpy().astype(np.int64)
    steps_total = int(counts[:, 2].sum())
    hits_total = int(counts[:, 1].sum())
    splits_total = int(counts[:, 3].sum())
    draws = steps_total - hits_total          # p_stop = 0 in these workloads: every hit is a cut
    showers_per_s = w.n / (ms_per_step / 1e3)

    # propagation kernel: algorithmic lane-operations (ALU roofline)
    k_prop = float(np.mean(prop_ms))
    alg_ops = OPS_PER_ARRIVAL * steps_total + OPS_PER_DRAW * draws + OPS_PER_SPLIT * splits_total
    alu = alg_ops / (k_prop / 1e3) / 1e12
    from paper_2202_05012_amd import prof_summary
    prof_dir = os.path.join(ROOT, "profiles")
    roof_prop = {"bound": "alu", "achieved": round(alu, 3), "peak": round(PEAK_ALU_TOPS, 2),
                 "unit": "T lane-ops/s", "frac": round(alu / PEAK_ALU_TOPS, 4),
                 "traffic": prof_summary.traffic_if_current(prof_dir, "supa_propagate", wname),
                 "kernel": "supa_propagate", "kernel_ms": round(k_prop, 4),
                 "alg_lane_ops": alg_ops,
                 # measured VALU instruction issue (rocprofv3 counters, committed summary)
                 "valu_issue_frac": prof_summary.counter_if_current(prof_dir, "supa_propagate", wname,
                                                                    "valu_issue_fraction")}
    # placement kernel: algorithmic bytes = the outputs it writes (HBM roofline)
    roof = roof_prop
    roof_other = None
    if outputs & (supa.OUT_HITS | supa.OUT_IMAGES | supa.OUT_TREE):
        # the placement kernel alone (hits, images), else the node scatter
        k_post = float(np.mean(post_ms))
        out_bytes = 0
        if outputs & supa.OUT_HITS:
            out_bytes += BYTES_PER_HIT * hits_total
        if outputs & supa.OUT_IMAGES:
            out_bytes += w.n * supa.n_layers(geom) * geom["img_nx"] * geom["img_ny"] * 4
        if not outputs & (supa.OUT_HITS | supa.OUT_IMAGES):
            out_bytes += BYTES_PER_NODE * int(counts[:, 0].sum())
        hbm = out_bytes / (k_post / 1e3) / 1e9
        kname = "supa_place" if outputs & (supa.OUT_HITS | supa.OUT_IMAGES) else "scatter_nodes"
        roof_place = {"bound": "hbm", "achieved": round(hbm, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                      "frac": round(hbm / PEAK_HBM_GBS, 4),
                      "traffic": prof_summary.traffic_if_current(prof_dir, kname, wname),
                      "kernel": kname, "kernel_ms": round(k_post, 4), "alg_bytes": out_bytes}
        # the dominant kernel (longest) is the headline roofline
        roof, roof_other = (roof_place, roof_prop) if k_post >= k_prop else (roof_prop, roof_place)

    line = {
        "metric": "showers/s (1 MI355X)",
        "value": round(showers_per_s, 1),
        "unit": "showers/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+u32",
        "data": "synthetic",
        "config": {"workload": wname,
                   "showers": w.n, "planes": w.n_planes,
                   "outputs": "+".join(n for n, b in (("hits", supa.OUT_HITS),
                                                      ("images", supa.OUT_IMAGES),
                                                      ("tree", supa.OUT_TREE)) if outputs & b)
                              or "counts"},
        "particle_steps_per_s": round(steps_total / (ms_per_step / 1e3), 1),
        "particle_steps": steps_total,
        "hits": hits_total,
        "roofline": roof,
    }
    # how evenly the propagation launch kept its waves busy (one eager call)
    sim.run(te0, tpol, taz, w.seed, out)
    wt = np.array(sim.wave_times())
    if len(wt):
        line["propagation_waves"] = {"waves": int(len(wt)), "median_ms": round(float(np.median(wt)), 4),
                                     "p90_ms": round(float(np.quantile(wt, 0.9)), 4),
                                     "max_ms": round(float(wt.max()), 4),
                                     "max_over_median": round(float(wt.max() / max(np.median(wt), 1e-9)), 3)}
    sub = sim.subtree_counts()
    if sub["shared"]:
        line["subtree_items"] = {"shared_showers": sub["shared"], "items_per_launch": sub["items"]}
    if launch is not None:
        line["launch"] = launch
    if args.graph:
        line["graph"] = True
    if roof_other is not None:
        line["roofline_other"] = roof_other
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_sampled(w, geom, args.cpu_seconds, args.cpu_seconds_1t,
                                                    bool(w.images))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
