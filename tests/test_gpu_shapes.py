"""GPU parity of the evaluation kernels (include/supa_shapes.h) against the
shape oracle: shower shape variables of seeded hit clouds and of simulated
showers, and the normalised histogram Wasserstein-1 distance.

Bars:
  - counts, depths and the NaN pattern exact;
  - other fields |gpu - oracle| <= 4e-7 |oracle| + atol, with atol
    2e-6 * rms for means, deviations, centroids and widths (rms = sqrt(mean^2
    + dev^2) of the same variable: the double-precision sums of a layer
    cancel to about 1e-12 of rms^2 at most, which moves a deviation near 0 by
    1e-6 rms; the float result adds 2^-24 relative), plus, for simulated
    showers, the hit coordinate tolerance (the variables move by at most as
    much as the points);
  - W1 per column and group means: relative 1e-9 (integer histograms are
    exact; only the order of double sums differs).
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import shape_oracle as SO
from oracle import supa_oracle as O
from paper_2202_05012_amd import shapes as SH, supa, workloads
from tests import parity

pytestmark = pytest.mark.gpu

LV = {k: i for i, k in enumerate(SO.LAYER_VARS)}
SV = {k: i for i, k in enumerate(SO.SHOWER_VARS)}
DEV = "cuda"


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def cloud(rng, n, L, gaps=True, big=(2000,), centre=100.0):
    """Seeded hit clouds stored segment by segment: per shower a random
    subset of layers in random order, each layer one contiguous run, layer -1
    hits sprinkled anywhere; optional unused gaps between segments."""
    segs, offs, cnts = [], [], []
    pos = 0
    for s in range(n):
        kind = rng.integers(0, 10)
        if s < len(big):
            m = big[s]
        elif kind == 0:
            m = int(rng.integers(0, 4))
        else:
            m = int(rng.integers(4, 300))
        nl = int(rng.integers(1, L + 1))
        lays = rng.permutation(L)[:nl]
        cuts = np.sort(rng.integers(0, m + 1, nl - 1)) if nl > 1 else np.array([], int)
        lens = np.diff(np.concatenate([[0], cuts, [m]]))
        lay = np.repeat(lays, lens).astype(np.int32)
        dead = rng.random(m) < 0.05
        lay[dead] = -1
        c = rng.normal(0, centre, 2)
        x = (c[0] + rng.normal(0, rng.uniform(0.01, 5), m)).astype(np.float32)
        y = (c[1] + rng.normal(0, rng.uniform(0.01, 5), m)).astype(np.float32)
        e = rng.exponential(rng.uniform(0.01, 3), m).astype(np.float32)
        if kind == 1 and m:
            e[:] = np.float32(0.25)            # equal energies: ratio 0, zero deviation
        if kind == 2 and m:
            e[:] = 0                           # zero energy: NaN centroids
        gap = int(rng.integers(0, 7)) if gaps else 0
        pos += gap
        segs.append((gap, x, y, e, lay))
        offs.append(pos)
        cnts.append(m)
        pos += m
    total = pos + 5
    X = np.full(total, 7e7, np.float32)
    Y = np.full(total, -7e7, np.float32)
    E = np.full(total, 1e9, np.float32)
    LAY = np.full(total, 999, np.int32)           # never read
    sid = np.full(total, -1, np.int64)
    for s, (_, x, y, e, lay) in enumerate(segs):
        a = offs[s]
        X[a:a + len(x)], Y[a:a + len(x)], E[a:a + len(x)], LAY[a:a + len(x)] = x, y, e, lay
        sid[a:a + len(x)] = s
    return np.array(offs, np.int64), np.array(cnts, np.int32), X, Y, E, LAY, sid


def oracle_shapes(n, L, sid, lay, x, y, e):
    keep = (sid >= 0) & (lay >= 0)
    return SO.shapes(n, L, sid[keep], lay[keep], x[keep].astype(np.float64),
                     y[keep].astype(np.float64), e[keep].astype(np.float64))


def _close(got, ref, atol, what):
    got = np.asarray(got, np.float64)
    nan_g, nan_r = np.isnan(got), np.isnan(ref)
    assert (nan_g == nan_r).all(), f"{what}: NaN pattern differs at {np.argwhere(nan_g != nan_r)[:5]}"
    ok = nan_r | (np.abs(got - ref) <= 4e-7 * np.abs(ref) + atol)
    if not ok.all():
        i = np.argwhere(~ok)[0]
        raise AssertionError(f"{what} at {tuple(i)}: {got[tuple(i)]} vs {ref[tuple(i)]}")


def check_shapes(glv, gsv, rlv, rsv, coord_atol=0.0):
    glv, gsv = glv.cpu().numpy(), gsv.cpu().numpy()
    np.testing.assert_array_equal(glv[..., LV["count"]], rlv[..., LV["count"]])
    np.testing.assert_array_equal(gsv[:, SV["depth"]], rsv[:, SV["depth"]])
    with np.errstate(invalid="ignore"):
        for v in ("x", "y", "r", "e"):
            m, d = rlv[..., LV["mean_" + v]], rlv[..., LV["std_" + v]]
            rms = np.nan_to_num(np.sqrt(m * m + d * d))
            ca = coord_atol if v != "e" else 0.0
            _close(glv[..., LV["mean_" + v]], m, 2e-6 * rms + ca, "mean_" + v)
            _close(glv[..., LV["std_" + v]], d, 2e-6 * rms + ca, "std_" + v)
        for v in ("x", "y", "r"):
            m, d = rlv[..., LV["centroid_" + v]], rlv[..., LV["width_" + v]]
            rms = np.nan_to_num(np.sqrt(m * m + d * d))
            _close(glv[..., LV["centroid_" + v]], m, 2e-6 * rms + coord_atol, "centroid_" + v)
            _close(glv[..., LV["width_" + v]], d, 2e-6 * rms + coord_atol, "width_" + v)
        for f in ("energy", "fraction", "energy_ratio"):
            _close(glv[..., LV[f]], rlv[..., LV[f]], 0.0, f)
        for f in ("e_tot", "l_d"):
            _close(gsv[:, SV[f]], rsv[:, SV[f]], 0.0, f)
        sd, w = rsv[:, SV["s_d"]], rsv[:, SV["s_d_width"]]
        rms = np.nan_to_num(np.sqrt(sd * sd + w * w))
        _close(gsv[:, SV["s_d"]], sd, 2e-6 * rms, "s_d")
        _close(gsv[:, SV["s_d_width"]], w, 2e-6 * rms, "s_d_width")


@pytest.mark.parametrize("L,seed", [(20, 1), (1, 2), (64, 3), (7, 4)])
def test_shapes_of_seeded_clouds(L, seed):
    rng = np.random.default_rng(seed)
    n = 700
    off, cnt, X, Y, E, LAY, sid = cloud(rng, n, L)
    glv, gsv = SH.shower_shapes(_t(off), _t(cnt), _t(X), _t(Y), _t(E), _t(LAY), L)
    rlv, rsv = oracle_shapes(n, L, sid, LAY, X, Y, E)
    check_shapes(glv, gsv, rlv, rsv)


def test_shapes_counts_stride_and_empty_batch():
    rng = np.random.default_rng(9)
    n, L = 50, 5
    off, cnt, X, Y, E, LAY, sid = cloud(rng, n, L, gaps=False, big=())
    wide = np.zeros((n, 6), np.int32)
    wide[:, 1] = cnt
    glv, gsv = SH.shower_shapes(_t(off), _t(wide).view(-1)[1:], _t(X), _t(Y), _t(E), _t(LAY), L,
                                counts_stride=6)
    rlv, rsv = oracle_shapes(n, L, sid, LAY, X, Y, E)
    check_shapes(glv, gsv, rlv, rsv)
    z = torch.zeros(0, dtype=torch.int64, device=DEV)
    lv, sv = SH.shower_shapes(z, z.int(), _t(X), _t(Y), _t(E), _t(LAY), L)
    assert lv.shape == (0, L, 18) and sv.shape == (0, 5)


def test_shapes_reject_split_layers_and_out_of_range():
    # shower 1 has layer 2 twice with layer 0 between; shower 2 a layer >= L
    lay = np.array([0, 0, 1, 2, 0, 2, 1, 3, 1, 0], np.int32)
    off = np.array([0, 3, 7], np.int64)
    cnt = np.array([3, 4, 3], np.int32)
    x = np.arange(12, dtype=np.float32)
    e = np.ones(12, np.float32)
    lay = np.concatenate([lay, [0, 0]]).astype(np.int32)
    lv, sv = SH.shower_shapes(_t(off), _t(cnt), _t(x), _t(x), _t(e), _t(lay), 3, check=False)
    lv, sv = lv.cpu().numpy(), sv.cpu().numpy()
    assert not np.isnan(lv[0, :, LV["count"]]).any() and np.isnan(lv[1:]).all() and np.isnan(sv[1:]).all()
    with pytest.raises(ValueError, match="2 showers"):
        SH.shower_shapes(_t(off), _t(cnt), _t(x), _t(x), _t(e), _t(lay), 3)


def test_shapes_of_simulated_showers_match_the_oracle_end_to_end():
    """GPU simulation + GPU shapes against oracle simulation + oracle shapes
    (independent on both sides; the hit sets agree to the coordinate bar)."""
    w = workloads.WORKLOADS["e1to100_20planes_img32_100k"]
    geom = workloads.geometry(w)
    n = 96
    e0, pol, az = workloads.initial_conditions(w, n)
    L = supa.n_layers(geom)
    sim = supa.Simulator(geom, supa.OUT_HITS)
    out = sim.simulate(_t(e0), _t(pol), _t(az), seed=w.seed)
    glv, gsv = SH.simulator_shapes(out, L)
    ref = O.simulate(geom, e0, pol, az, seed=w.seed)
    e = (ref["hit_e"].astype(np.float32) * np.float32(2.0 ** -ref["frac_bits"])).astype(np.float64)
    sid = ref["hit_sid"] - ref["shower_id_base"]
    keep = ref["hit_layer"] >= 0
    rlv, rsv = SO.shapes(n, L, sid[keep], ref["hit_layer"][keep], ref["hit_x"][keep],
                         ref["hit_y"][keep], e[keep])
    rmax = float(np.hypot(ref["hit_x"], ref["hit_y"]).max())
    check_shapes(glv, gsv, rlv, rsv, coord_atol=1e-5 * max(rmax, 1.0))


def test_simulated_showers_with_a_non_monotone_layer_map():
    """Layers that are not ranges of planes (plane k read out as layer k mod 4,
    plane 3 not read out): the simulator groups each segment by layer, so the
    shape kernel takes its output as it is, and both match the oracle."""
    w = workloads.WORKLOADS["e1to100_20planes_img32_100k"]
    lmap = [k % 4 for k in range(20)]
    lmap[3] = -1
    geom = dict(workloads.geometry(w), layer_of_plane=lmap)
    n = 96
    e0, pol, az = workloads.initial_conditions(w, n)
    L = supa.n_layers(geom)
    sim = supa.Simulator(geom, supa.OUT_HITS | supa.OUT_KEYS)
    out = sim.simulate(_t(e0), _t(pol), _t(az), seed=w.seed)
    gpu = parity.to_numpy(out)
    ref = O.simulate(geom, e0, pol, az, seed=w.seed)
    parity.check_all(gpu, ref, geom)
    for i in range(n):
        seg = gpu["hit_layer"][gpu["hit_offsets"][i]:gpu["hit_offsets"][i] + gpu["counts"][i, 1]]
        assert (np.diff(seg) >= 0).all(), f"shower {i}: layers not grouped"
    glv, gsv = SH.simulator_shapes(out, L)
    e = (ref["hit_e"].astype(np.float32) * np.float32(2.0 ** -ref["frac_bits"])).astype(np.float64)
    sid = ref["hit_sid"] - ref["shower_id_base"]
    keep = ref["hit_layer"] >= 0
    rlv, rsv = SO.shapes(n, L, sid[keep], ref["hit_layer"][keep], ref["hit_x"][keep],
                         ref["hit_y"][keep], e[keep])
    rmax = float(np.hypot(ref["hit_x"], ref["hit_y"]).max())
    check_shapes(glv, gsv, rlv, rsv, coord_atol=1e-5 * max(rmax, 1.0))


def _w1_case(rng, nr, ns, cols):
    ref = rng.normal(size=(nr, cols)) * rng.uniform(0.1, 10, cols) + rng.normal(0, 50, cols)
    smp = rng.standard_t(5, size=(ns, cols)) * rng.uniform(0.1, 10, cols) + rng.normal(0, 50, cols)
    ref, smp = ref.astype(np.float32), smp.astype(np.float32)
    ref[:, 3] = 1.5                                  # constant reference: skipped
    smp[:, 4] = np.nan                               # empty sample: skipped
    ref[rng.random((nr, cols)) < 0.02] = np.nan      # dropped entries
    smp[rng.random((ns, cols)) < 0.02] = np.inf
    ref[:, 5] = np.round(ref[:, 5])                  # ties on bin edges
    smp[:, 5] = np.round(smp[:, 5])
    return ref, smp


@pytest.mark.parametrize("n_bins", [1, 100, 4096])
def test_w1_columns_match_the_oracle(n_bins):
    rng = np.random.default_rng(n_bins)
    ref, smp = _w1_case(rng, 5003, 3001, 37)
    groups = (np.arange(37) % 4).astype(np.int32)
    groups[7] = -1
    w1, gm = SH.w1_columns(_t(ref), _t(smp), n_bins, groups=_t(groups), n_groups=5)
    want = SO.w1_columns(ref.astype(np.float64), smp.astype(np.float64), n_bins)
    got = w1.cpu().numpy()
    assert (np.isnan(got) == np.isnan(want)).all()
    np.testing.assert_allclose(got, want, rtol=1e-9, atol=0)
    gwant = SO.group_means(want, groups, 5)
    assert np.isnan(gm[4].item()) and np.isnan(gwant[4])
    np.testing.assert_allclose(gm.cpu().numpy()[:4], gwant[:4], rtol=1e-12)


def test_w1_single_column_of_a_million_points():
    rng = np.random.default_rng(21)
    a = rng.gamma(2.0, size=1_000_000).astype(np.float32)
    b = rng.gamma(2.2, size=700_001).astype(np.float32)
    w1, _ = SH.w1_columns(_t(a), _t(b), 512)
    want = SO.w1_columns(a.astype(np.float64)[:, None], b.astype(np.float64)[:, None], 512)
    np.testing.assert_allclose(w1.cpu().numpy(), want, rtol=1e-9)
    x, y = a[:len(b)].astype(np.float64), b.astype(np.float64)
    r = SH.hit_radius(_t(a[:len(b)]), _t(b)).cpu().numpy()
    np.testing.assert_array_equal(r, np.sqrt(x * x + y * y).astype(np.float32))


def test_mean_discrepancy_of_two_simulated_samples():
    """Shape matrices of two oracle samples (different seeds) as inputs."""
    w = workloads.WORKLOADS["e1to100_20planes_img32_100k"]
    geom = workloads.geometry(w)
    L = supa.n_layers(geom)
    mats = []
    for seed in (3, 4):
        n = 300
        e0, pol, az = workloads.initial_conditions(w, n, seed=seed)
        ref = O.simulate(geom, e0, pol, az, seed=seed)
        e = ref["hit_e"].astype(np.float64) * 2.0 ** -ref["frac_bits"]
        sid = ref["hit_sid"] - ref["shower_id_base"]
        k = ref["hit_layer"] >= 0
        pl, ps = SO.shapes(n, L, sid[k], ref["hit_layer"][k], ref["hit_x"][k], ref["hit_y"][k], e[k])
        mats.append(np.concatenate([pl.reshape(n, -1), ps], axis=1).astype(np.float32))
    a, b = mats
    cols = a.shape[1]
    groups = np.concatenate([np.tile(np.arange(18), L), 18 + np.arange(5)]).astype(np.int32)
    w1, gm = SH.w1_columns(_t(a), _t(b), 100, groups=_t(groups), n_groups=23)
    want = SO.w1_columns(a.astype(np.float64), b.astype(np.float64), 100)
    np.testing.assert_allclose(w1.cpu().numpy(), want, rtol=1e-9)
    np.testing.assert_allclose(gm.cpu().numpy(), SO.group_means(want, groups, 23), rtol=1e-12)
    assert cols == L * 18 + 5


def test_full_size_100k_shapes_sampled():
    """Shape variables of the 100,000-shower benchmark sample at full size, in
    one launch over the whole batch as bench.py --shapes times it; the oracle
    simulates and measures sampled blocks of 64 showers (first, last, three
    at random)."""
    w = workloads.WORKLOADS["e1to100_20planes_img32_100k"]
    geom = workloads.geometry(w)
    L = supa.n_layers(geom)
    e0, pol, az = workloads.initial_conditions(w)
    sim = supa.Simulator(geom, supa.OUT_HITS)
    out = sim.simulate(_t(e0), _t(pol), _t(az), seed=w.seed)
    lv, sv = SH.simulator_shapes(out, L)
    assert torch.isfinite(sv[:, SV["e_tot"]]).all()
    rng = np.random.default_rng(2)
    for start in [0, w.n - 64] + list(rng.integers(0, w.n - 64, 3)):
        rows = np.arange(start, start + 64)
        ref = O.simulate(geom, e0[rows], pol[rows], az[rows], w.seed, shower_id_base=int(start))
        e = (ref["hit_e"].astype(np.float32) * np.float32(2.0 ** -ref["frac_bits"])).astype(np.float64)
        sid = ref["hit_sid"] - ref["shower_id_base"]
        rlv, rsv = SO.shapes(64, L, sid, ref["hit_layer"], ref["hit_x"], ref["hit_y"], e)
        rmax = float(np.hypot(ref["hit_x"], ref["hit_y"]).max())
        it = torch.from_numpy(rows).cuda()
        check_shapes(lv[it], sv[it], rlv, rsv, coord_atol=1e-5 * max(rmax, 1.0))


@pytest.mark.parametrize("n", [5_000, 600_000])
def test_every_shower_once_in_either_order(n):
    """Showers are taken longest first: by one order over the whole batch when
    every shower is in flight at once, by windows of consecutive showers when
    there are more showers than lanes (600,000 > 256 CUs x 16 waves x 64).
    Either way every shower is measured once: counts per (shower, layer) and
    layer energies against bincounts over all showers, every variable against
    the oracle on 300 sampled showers."""
    rng = np.random.default_rng(11)
    L = 12
    m = rng.integers(0, 41, n)
    m[rng.random(n) < 0.02] = 400                   # a few long showers
    off = np.concatenate([[0], np.cumsum(m)[:-1]]).astype(np.int64)
    sid = np.repeat(np.arange(n), m)
    j = np.arange(len(sid)) - off[sid]              # hit index within its shower
    nl = rng.integers(1, L + 1, n)
    first = rng.integers(0, L - nl + 1)
    lay = (first[sid] + (j * nl[sid]) // m[sid]).astype(np.int32)
    x = rng.normal(0, 3, len(sid)).astype(np.float32)
    y = rng.normal(0, 3, len(sid)).astype(np.float32)
    e = rng.exponential(1.0, len(sid)).astype(np.float32)
    lv, sv = SH.shower_shapes(_t(off), _t(m.astype(np.int32)), _t(x), _t(y), _t(e), _t(lay), L)
    glv, gsv = lv.cpu().numpy(), sv.cpu().numpy()
    key = sid * L + lay
    cnt = np.bincount(key, minlength=n * L).reshape(n, L)
    np.testing.assert_array_equal(glv[..., LV["count"]], cnt)
    en = np.bincount(key, weights=e.astype(np.float64), minlength=n * L).reshape(n, L)
    np.testing.assert_allclose(glv[..., LV["energy"]], en, rtol=4e-7, atol=0)
    np.testing.assert_allclose(gsv[:, SV["e_tot"]], en.sum(1), rtol=4e-7, atol=0)
    pick = np.sort(rng.choice(n, 300, replace=False))
    sel = np.isin(sid, pick)
    local = np.searchsorted(pick, sid[sel])
    rlv, rsv = SO.shapes(len(pick), L, local, lay[sel], x[sel].astype(np.float64),
                         y[sel].astype(np.float64), e[sel].astype(np.float64))
    it = torch.from_numpy(pick).cuda()
    check_shapes(lv[it], sv[it], rlv, rsv)


def test_usage_example():
    """The usage example of the README, end to end: SUPAv1 showers, their shape
    variables and 2x grids (128 points of 65/128 in layer 0, fraction 1)."""
    from paper_2202_05012_amd import grids, presets
    geom = presets.supa(1)
    e0, pol, az = (torch.tensor(v, device="cuda") for v in presets.incident(1000))
    sim = supa.Simulator(geom, supa.OUT_HITS | supa.OUT_KEYS)
    out = sim.simulate(e0, pol, az, seed=1)
    lv, sv = SH.simulator_shapes(out, n_layers=supa.n_layers(geom))
    img = grids.simulator_grids(out, presets.calogan_grids(2))
    assert lv.shape == (1000, 1, 18) and sv.shape == (1000, 5) and img.shape == (1000, 2016)
    assert (lv[:, 0, LV["count"]] == 128).all() and (lv[:, 0, LV["fraction"]] == 1).all()
    assert torch.allclose(lv[:, 0, LV["mean_e"]], torch.tensor(65.0 / 128, device="cuda"))
    assert torch.allclose(img.sum(1), torch.tensor(65.0, device="cuda"))
