"""Subtree work items: showers whose pending particles are handed to other
waves and later launches give the oracle's results.

A particle's further history depends only on its own state, plane and path
id (section "Propagation Model"; Algorithm 1 keys nothing on the rest of the
shower), so a shower finished by several waves must give the same hits,
tree, images, ledger and counts as one finished by a single wave.  Each test
forces the split (an export threshold of zero hands out every oldest group
of 16 or more particles of a shower) and checks that it happened."""
import numpy as np
import pytest
import torch

from oracle import supa_oracle as O
from paper_2202_05012_amd import supa, workloads
from tests import parity

pytestmark = pytest.mark.gpu

ALL = supa.OUT_HITS | supa.OUT_IMAGES | supa.OUT_TREE | supa.OUT_KEYS
HITS_TREE = supa.OUT_HITS | supa.OUT_TREE | supa.OUT_KEYS


def dev_t(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


def run(geom, outputs, e0, pol, az, seed, phases, export_pool=0, base=0, **launch):
    print(f"subtrees: {len(e0)} showers, outputs {outputs}, phases {phases}, export {export_pool}", flush=True)
    sim = supa.Simulator(geom, outputs, subtree_phases=phases, export_pool=export_pool, **launch)
    out = sim.simulate(dev_t(e0), dev_t(pol), dev_t(az), seed, shower_id_base=base)
    torch.cuda.synchronize()
    return parity.to_numpy(out), sim


def assert_split(sim, phases):
    st = sim.subtree_counts()
    assert st["shared"] > 0, st
    for p in range(phases - 1):
        assert st["items"][p] > 0, (p, st)
    assert all(v == 0 for v in st["items"][phases - 1:]), st      # the last launch exports nothing
    return st


def test_split_showers_match_oracle_hits_and_tree():
    w = workloads.WORKLOADS["loge1to1000_20planes_1m"]
    geom = workloads.geometry(w)
    e0, pol, az = workloads.initial_conditions(w, 200)
    gpu, sim = run(geom, HITS_TREE, e0, pol, az, w.seed, phases=3)
    assert_split(sim, 3)
    ref = O.simulate(geom, e0, pol, az, w.seed)
    parity.check_all(gpu, ref, geom, tree=True)


def test_split_showers_match_oracle_with_images():
    w = workloads.WORKLOADS["e1to100_20planes_img32_100k"]
    geom = workloads.geometry(w)
    e0, pol, az = workloads.initial_conditions(w, 300)
    gpu, sim = run(geom, ALL, e0, pol, az, w.seed, phases=4)
    assert_split(sim, 4)
    ref = O.simulate(geom, e0, pol, az, w.seed)
    parity.check_all(gpu, ref, geom, images=True, tree=True)


def test_split_fifty_planes_tree_and_256_images():
    w = workloads.WORKLOADS["loge10to1000_50planes_tree_img256_1m"]
    geom = workloads.geometry(w)
    e0, pol, az = workloads.initial_conditions(w, 24)
    gpu, sim = run(geom, ALL, e0, pol, az, w.seed, phases=3)
    assert_split(sim, 3)
    ref = O.simulate(geom, e0, pol, az, w.seed)
    parity.check_all(gpu, ref, geom, images=True, tree=True)


def test_split_counts_only_and_hits_without_keys():
    """Counts-only calls (no records: tallies and node counts only) and hit
    clouds without path ids (the placement variant the benchmark runs)."""
    w = workloads.WORKLOADS["loge1to1000_20planes_1m"]
    geom = workloads.geometry(w)
    e0, pol, az = workloads.initial_conditions(w, 160)
    ref = O.simulate(geom, e0, pol, az, w.seed)
    gpu, sim = run(geom, 0, e0, pol, az, w.seed, phases=3)
    assert_split(sim, 3)
    parity.check_counts(gpu, ref)
    gpu, sim = run(geom, supa.OUT_HITS, e0, pol, az, w.seed, phases=3)
    assert_split(sim, 3)
    parity.check_counts(gpu, ref)
    parity.check_hits_unkeyed(gpu, ref)


def test_few_large_showers_spread_over_all_waves():
    """Sixteen 1000-unit showers: without items they run on four waves; with
    the default threshold every one of them is shared."""
    w = workloads.WORKLOADS["loge1to1000_20planes_1m"]
    geom = workloads.geometry(w)
    _, pol, az = workloads.initial_conditions(w, 16)
    e0 = np.full(16, 1000.0, np.float32)
    gpu, sim = run(geom, HITS_TREE, e0, pol, az, 3, phases=4, export_pool=64)
    st = assert_split(sim, 4)
    assert st["shared"] == 16, st
    ref = O.simulate(geom, e0, pol, az, 3)
    parity.check_all(gpu, ref, geom, tree=True)


def test_split_with_spill_and_tiny_logs():
    """A small LDS pool (entries spill to the ring in global memory before
    they are exported) and logs that must grow: the rerun after growth splits
    again and still matches."""
    w = workloads.WORKLOADS["loge1to1000_20planes_1m"]
    geom = workloads.geometry(w)
    e0, pol, az = workloads.initial_conditions(w, 120)
    gpu, sim = run(geom, HITS_TREE, e0, pol, az, w.seed, phases=2, export_pool=256,
                   waves_per_cu=1, frontier_cap=128, hit_cap=64, node_cap=64)
    assert_split(sim, 2)
    ref = O.simulate(geom, e0, pol, az, w.seed)
    parity.check_all(gpu, ref, geom, tree=True)


def test_split_noalloc_and_graph_match_oracle():
    w = workloads.WORKLOADS["loge1to1000_20planes_1m"]
    geom = workloads.geometry(w)
    n = 150
    e0, pol, az = workloads.initial_conditions(w, n)
    ref = O.simulate(geom, e0, pol, az, w.seed)
    hc, nc = int(1.1 * len(ref["hit_e"])) + 64, int(1.1 * len(ref["node_e"])) + 64
    sim = supa.Simulator(geom, HITS_TREE, subtree_phases=3, export_pool=0)
    args = (dev_t(e0), dev_t(pol), dev_t(az), w.seed)
    print("subtrees: noalloc call", flush=True)
    out = sim.allocate(n, hc, nc)
    assert sim.run_noalloc(*args, out) == 0
    torch.cuda.synchronize()
    assert_split(sim, 3)
    parity.check_all(parity.to_numpy(out), ref, geom, tree=True)
    print("subtrees: captured call, three replays", flush=True)
    out = sim.allocate(n, hc, nc)
    g = sim.graph(*args, out)
    for rep in range(3):
        for v in out.values():
            if isinstance(v, torch.Tensor):
                v.fill_(-7)
        g.launch()
        g.check()
        torch.cuda.synchronize()
        assert_split(sim, 3)
        parity.check_all(parity.to_numpy(out), ref, geom, tree=True)
    g.close()


def test_subtree_settings_are_validated():
    w = workloads.WORKLOADS["e10_normal_5planes_1k"]
    geom = workloads.geometry(w)
    sim = supa.Simulator(geom, supa.OUT_HITS)
    for bad in ((-1, 0), (5, 0), (2, -1)):
        with pytest.raises(supa.SupaError):
            sim.set_subtrees(*bad)
    lit = supa.Simulator(dict(geom, kinematics="literal"), supa.OUT_HITS)
    with pytest.raises(supa.SupaError):
        lit.set_subtrees(2, 64)
    lit.set_subtrees(1, 64)             # turning them off is always accepted


def test_automatic_mode_splits_only_small_batches():
    """By default a batch small enough to leave most waves idle is split,
    a batch that fills the waves is not, and neither is a literal-kinematics
    batch (no items for that variant)."""
    w = workloads.WORKLOADS["loge1to1000_20planes_1m"]
    geom = workloads.geometry(w)
    _, pol, az = workloads.initial_conditions(w, 32)
    e0 = np.full(32, 800.0, np.float32)
    print("subtrees: automatic, 32 showers", flush=True)
    sim = supa.Simulator(geom, HITS_TREE)
    out = parity.to_numpy(sim.simulate(dev_t(e0), dev_t(pol), dev_t(az), 5))
    assert_split(sim, 2)
    parity.check_all(out, O.simulate(geom, e0, pol, az, 5), geom, tree=True)
    n_big = 4 * 256 * 16 + 4             # more than a quarter of the default launch's waves
    e0b, polb, azb = workloads.initial_conditions(w, n_big)
    print(f"subtrees: automatic, {n_big} showers", flush=True)
    sim.simulate(dev_t(e0b), dev_t(polb), dev_t(azb), 5)
    torch.cuda.synchronize()
    assert sim.subtree_counts()["shared"] == 0
    lit = supa.Simulator(dict(geom, kinematics="literal"), supa.OUT_HITS)
    print("subtrees: automatic, literal kinematics", flush=True)
    lit.simulate(dev_t(e0), dev_t(pol), dev_t(az), 5)
    torch.cuda.synchronize()
    assert lit.subtree_counts()["shared"] == 0
