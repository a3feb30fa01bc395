"""Pins of the shower-shape oracle (oracle/shape_oracle.py) against things
other than itself: the SUPAv1 configuration, whose shape is fixed by the
paper (128 equal deposits on sub-layer 7); hand-computed values on tiny
clouds; numpy's own mean, standard deviation and weighted average; and
scipy's Wasserstein distance."""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import shape_oracle as SO
from oracle import supa_oracle as O
from tests.test_oracle_pins import supav1_geom

LV = {k: i for i, k in enumerate(SO.LAYER_VARS)}
SV = {k: i for i, k in enumerate(SO.SHOWER_VARS)}


def test_supav1_shapes_are_fixed_by_the_paper():
    n, e0 = 4, 65.0
    r = O.simulate(supav1_geom(), [e0] * n, [0.2] * n, [1.0] * n, seed=5)
    e = r["hit_e"].astype(np.float64) * 2.0 ** -r["frac_bits"]
    pl, ps = SO.shapes(n, 8, r["hit_sid"], r["hit_layer"], r["hit_x"], r["hit_y"], e)
    assert (pl[:, 7, LV["count"]] == 128).all()
    assert np.allclose(pl[:, 7, LV["energy"]], e0) and (pl[:, :7, LV["energy"]] == 0).all()
    assert np.allclose(pl[:, 7, LV["mean_e"]], e0 / 128) and np.allclose(pl[:, 7, LV["std_e"]], 0)
    assert (pl[:, 7, LV["energy_ratio"]] == 0).all()              # equal top two energies
    assert (pl[:, 7, LV["fraction"]] == 1).all() and (pl[:, :7, LV["fraction"]] == 0).all()
    # equal weights: the energy-weighted centroid is the plain mean
    assert np.allclose(pl[:, 7, LV["centroid_x"]], pl[:, 7, LV["mean_x"]])
    assert np.allclose(pl[:, 7, LV["width_r"]], pl[:, 7, LV["std_r"]])
    assert (ps[:, SV["depth"]] == 7).all() and np.allclose(ps[:, SV["s_d"]], 7)
    assert np.allclose(ps[:, SV["s_d_width"]], 0) and np.allclose(ps[:, SV["l_d"]], 7 * e0)
    assert np.isnan(pl[:, :7, LV["mean_x"]]).all()                # empty layers


def test_hand_computed_layer():
    # points (1, 0, E=1) and (-1, 0, E=3): r = 1 for both
    v = SO.layer_variables([1.0, -1.0], [0.0, 0.0], [1.0, 3.0])
    assert v["count"] == 2 and v["energy"] == 4
    assert v["mean_x"] == 0 and v["std_x"] == 1 and v["mean_r"] == 1 and v["std_r"] == 0
    assert v["mean_e"] == 2 and v["std_e"] == 1
    assert v["centroid_x"] == -0.5 and v["width_x"] == pytest.approx(math.sqrt(0.75))
    assert v["centroid_r"] == 1 and v["width_r"] == 0
    assert v["energy_ratio"] == 0.5
    one = SO.layer_variables([2.0], [0.0], [5.0])
    assert one["energy_ratio"] == 1 and one["std_x"] == 0 and one["centroid_x"] == 2


def test_shower_depth_hand_computed():
    sv = SO.shower_variables([0, 0, 2.0, 0, 2.0, 0])
    assert sv["e_tot"] == 4 and sv["depth"] == 4 and sv["l_d"] == 12
    assert sv["s_d"] == 3 and sv["s_d_width"] == 1
    assert SO.shower_variables([0.0, 0.0])["depth"] == -1


def test_against_numpy_routines_on_random_clouds():
    rng = np.random.default_rng(3)
    n, L = 7, 5
    m = 600
    sid = rng.integers(0, n, m)
    layer = rng.integers(0, L, m)
    x, y = rng.normal(size=m), rng.normal(size=m)
    e = rng.exponential(size=m)
    pl, ps = SO.shapes(n, L, sid, layer, x, y, e)
    for s in range(n):
        assert np.nansum(pl[s, :, LV["fraction"]]) == pytest.approx(1.0)
        assert 0 <= ps[s, SV["s_d"]] <= L - 1
        for l in range(L):
            sel = (sid == s) & (layer == l)
            if not sel.any():
                continue
            r = np.hypot(x[sel], y[sel])
            assert pl[s, l, LV["std_y"]] == pytest.approx(np.std(y[sel]), abs=1e-12)
            assert pl[s, l, LV["std_r"]] == pytest.approx(np.std(r), abs=1e-12)
            assert pl[s, l, LV["centroid_r"]] == pytest.approx(np.average(r, weights=e[sel]))
            wvar = np.average((x[sel] - np.average(x[sel], weights=e[sel])) ** 2, weights=e[sel])
            assert pl[s, l, LV["width_x"]] == pytest.approx(math.sqrt(wvar), abs=1e-12)
            top = np.sort(e[sel])
            want = 1.0 if len(top) == 1 else (top[-1] - top[-2]) / (top[-1] + top[-2])
            assert pl[s, l, LV["energy_ratio"]] == pytest.approx(want)


def test_w1_and_mean_discrepancy():
    rng = np.random.default_rng(4)
    a, b = rng.normal(size=500), rng.normal(0.3, 1.4, size=700)
    assert SO.w1(a, b) == pytest.approx(stats.wasserstein_distance(a, b), rel=1e-12)
    ref = rng.normal(size=(2000, 3)) * [1.0, 2.0, 5.0] + [0.0, 1.0, -3.0]
    assert SO.mean_discrepancy(ref, ref) == 0
    # a sample shifted by one reference standard deviation in every column
    shifted = ref + ref.std(axis=0)
    assert SO.mean_discrepancy(ref, shifted) == pytest.approx(1.0, rel=1e-9)


def test_hist_w1_closed_forms_and_limit():
    # two point masses one apart: the bin centres sit h/2 inside the range
    for n_bins in (1, 2, 7, 100):
        d = SO.hist_w1(np.zeros(10), np.ones(30), n_bins)
        assert d == pytest.approx((n_bins - 1) / n_bins, abs=1e-15)
    rng = np.random.default_rng(5)
    a, b = rng.normal(size=3000), rng.gamma(2.0, size=2000)
    assert SO.hist_w1(a, a.copy(), 50) == 0
    # many bins: within one bin width of the exact distance
    n_bins = 100_000
    h = (max(a.max(), b.max()) - min(a.min(), b.min())) / n_bins
    assert abs(SO.hist_w1(a, b, n_bins) - stats.wasserstein_distance(a, b)) <= h


def test_hist_bins_match_numpy_histogram():
    rng = np.random.default_rng(6)
    v = rng.normal(size=20000).astype(np.float32).astype(np.float64)
    lo, hi = v.min(), v.max()
    for n_bins in (1, 10, 97, 1024):
        mine = np.bincount(SO.hist_bins(v, lo, hi, n_bins), minlength=n_bins)
        ref, _ = np.histogram(v, bins=n_bins, range=(lo, hi))
        assert np.abs(mine - ref).sum() <= 2 and mine.sum() == len(v)
    assert (SO.hist_bins([3.0, 3.0], 3.0, 3.0, 8) == 0).all()


def test_w1_columns_invariances_and_skips():
    rng = np.random.default_rng(7)
    ref = rng.normal(size=(4000, 4)) * [1.0, 3.0, 0.5, 1.0]
    smp = rng.normal(size=(3000, 4)) * [1.2, 3.0, 0.5, 1.0] + [0.1, 0.0, 0.2, 0.0]
    ref[:, 3] = 2.5                                   # constant reference column
    smp[::7, 1] = np.nan                              # dropped entries
    d = SO.w1_columns(ref, smp, 64)
    assert np.isnan(d[3]) and np.isfinite(d[:3]).all()
    # normalisation by the reference: an affine map of both samples keeps it
    d2 = SO.w1_columns(ref * 4.0 - 7.0, smp * 4.0 - 7.0, 64)
    assert np.allclose(d[:3], d2[:3], rtol=1e-9)
    # histogram distance -> exact distance as the bins shrink
    ex = SO.w1_columns(ref, smp, None)
    fine = SO.w1_columns(ref, smp, 50_000)
    assert np.allclose(fine[:3], ex[:3], atol=1e-3)
    assert np.isnan(SO.w1_columns(ref[:1], smp, 8)).all()      # one reference row
    g = SO.group_means([1.0, np.nan, 3.0, 5.0], [0, 0, 0, 2], 3)
    assert g[0] == 2.0 and np.isnan(g[1]) and g[2] == 5.0
