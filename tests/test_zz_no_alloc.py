"""supa_simulate_noalloc (scratch from the library's fixed per-GPU array, no
allocation) against supa_simulate on the same inputs, through the C ABI.

Both entry points run the same kernels, so every per-shower result is
bit-identical: counts, ledgers, segment offsets and images exactly; hits and
tree nodes exactly once put in path-id order (the order of records within a
plane, and the numbering of nodes, depend on which showers share a wave).
Two calls in a row, the second smaller, check that nothing of the first call
left in the shared array leaks into the second; the smaller one is also
compared with the oracle."""
import numpy as np
import pytest
import torch

from oracle import supa_oracle as O
from paper_2202_05012_amd import supa, workloads
from tests import parity

pytestmark = pytest.mark.gpu

ALL = supa.OUT_HITS | supa.OUT_IMAGES | supa.OUT_TREE | supa.OUT_KEYS


def dev_t(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


def poisoned(sim, n, hc, nc):
    out = sim.allocate(n, hc, nc)
    for v in out.values():
        if isinstance(v, torch.Tensor):
            v.fill_(-7)
    return out


def test_noalloc_matches_simulate_on_two_calls_in_a_row():
    w = workloads.WORKLOADS["e1to100_20planes_img32_100k"]
    geom = workloads.geometry(w)
    e0, pol, az = workloads.initial_conditions(w, 4000)
    ref_sim = supa.Simulator(geom, ALL)
    fix_sim = supa.Simulator(geom, ALL)
    for s0, m in ((0, 1500), (3100, 400)):            # the second call is smaller
        sl = slice(s0, s0 + m)
        print(f"noalloc call: showers {s0}..{s0 + m}", flush=True)
        args = (dev_t(e0[sl]), dev_t(pol[sl]), dev_t(az[sl]), w.seed)
        ref = ref_sim.simulate(*args, shower_id_base=s0)
        hc, nc = int(ref["total_hits"]), int(ref["total_nodes"])
        out = poisoned(fix_sim, m, hc, nc)
        st = fix_sim.run_noalloc(*args, out, shower_id_base=s0)
        assert st == 0, st
        torch.cuda.synchronize()
        parity.check_same_outputs(out, ref)
    # the smaller call also against the oracle
    orc = O.simulate(geom, e0[sl], pol[sl], az[sl], w.seed, shower_id_base=s0)
    parity.check_all(parity.to_numpy(out), orc, geom, images=True, tree=True)


def test_noalloc_hits_only_many_showers_and_capacity_retry():
    """A hits-only call of 2,000 showers of the 20-plane log-uniform
    workload (its largest showers spill out of the LDS pool), first with hit
    arrays too small (CAPACITY, totals set), then again with enough room."""
    w = workloads.WORKLOADS["loge1to1000_20planes_1m"]
    geom = workloads.geometry(w)
    n = 2_000
    e0, pol, az = workloads.initial_conditions(w, n)
    args = (dev_t(e0), dev_t(pol), dev_t(az), w.seed)
    outs = supa.OUT_HITS | supa.OUT_KEYS
    ref = supa.Simulator(geom, outs).simulate(*args)
    sim = supa.Simulator(geom, outs)
    small = poisoned(sim, n, 1000, 0)
    st = sim.run_noalloc(*args, small)
    assert st == 3, st
    assert small["total_hits"] == ref["total_hits"]
    out = poisoned(sim, n, int(ref["total_hits"]), 0)
    st = sim.run_noalloc(*args, out)
    assert st == 0, st
    torch.cuda.synchronize()
    a, b = parity.to_numpy(out), parity.to_numpy(ref)
    for k in ("counts", "ledger", "hit_offsets"):
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)
    for i in range(0, n, 7):
        sl = slice(int(a["hit_offsets"][i]), int(a["hit_offsets"][i]) + int(a["counts"][i, 1]))
        oa, ob = np.argsort(a["hit_key"][sl]), np.argsort(b["hit_key"][sl])
        for f in ("hit_x", "hit_y", "hit_e", "hit_layer", "hit_key"):
            np.testing.assert_array_equal(a[f][sl][oa], b[f][sl][ob], err_msg=f"shower {i}: {f}")


def test_noalloc_refuses_what_does_not_fit_then_runs_again():
    """A batch whose hit records exceed the fixed array fails with NOMEM (the
    kernels' log claims are bounded, nothing is written outside it); a call
    that fits, on the same context, is correct afterwards."""
    w = workloads.WORKLOADS["e1to100_20planes_img32_100k"]
    geom = workloads.geometry(w)
    sim = supa.Simulator(geom, supa.OUT_HITS)
    n = 40_000                                       # ~3.7e7 hit records: more than the array holds
    e0, pol, az = workloads.initial_conditions(w, n)
    out = poisoned(sim, n, 64 * n, 0)
    with pytest.raises(supa.SupaError) as e:
        sim.run_noalloc(dev_t(e0), dev_t(pol), dev_t(az), w.seed, out)
    assert e.value.status == 6 and "fixed" in str(e.value)
    m = 200
    out = poisoned(sim, m, 2500 * m, 0)                # > the most hits a shower of E0 <= 100 makes
    st = sim.run_noalloc(dev_t(e0[:m]), dev_t(pol[:m]), dev_t(az[:m]), w.seed, out)
    assert st == 0, st
    torch.cuda.synchronize()
    th = int(out["total_hits"])
    res = parity.to_numpy({k: (v[:th] if k in ("hit_x", "hit_y", "hit_e", "hit_layer") else v)
                           for k, v in out.items()})
    orc = O.simulate(geom, e0[:m], pol[:m], az[:m], w.seed)
    parity.check_counts(res, orc)
