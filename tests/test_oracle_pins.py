"""Pins of the FP64 oracle against what the paper and mathematics fix.

None of these tests re-types the oracle's formulas: they check it against
published known-answer vectors, an independent Philox implementation, the
fully determined SUPAv1 configuration of the paper (Table 2 and the appendix
"Parameters"), closed forms for straight flight and for the mean cascade size,
hand-derived geometry of a one-split shower, library routines (scipy rotations,
numpy histograms) and distribution tests of the sampled quantities.
"""
import math
import os
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import stats
from scipy.spatial.transform import Rotation

from oracle import supa_oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))
S = 21                    # fixed-point fractional bits
TWO32 = 2.0 ** 32


def geom(**kw):
    g = dict(n_planes=5, z_first=1.0, dz=1.0, layer_of_plane=None, p_stop=None,
             p_split=None, e_cut=0.1, angle_mode="rayleigh", angle_a=0.1, angle_b=0.0,
             frac_lo=0.0, frac_hi=1.0, frac_bits=S)
    g.update(kw)
    return g


def u_open(w):
    return (np.asarray(w, np.float64) + 0.5) / TWO32


# --------------------------------------------------------------------------
# Philox4x32-10
# --------------------------------------------------------------------------
def test_philox_known_answer_vectors():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([int(t, 16) for t in line.split()])
    assert len(rows) == 3
    for c0, c1, c2, c3, k0, k1, *out in rows:
        assert O.philox4x32_10(k0 | (k1 << 32), (c0, c1, c2, c3)) == tuple(out)


def test_philox_matches_independent_header():
    """Bit equality with PyTorch's PhiloxRNGEngine.h on random (key, counter)."""
    import torch
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    rng = np.random.default_rng(123)
    n = 20000
    words = rng.integers(0, 2 ** 32, size=(n, 6), dtype=np.uint64)
    words[:50] = 0xFFFFFFFF
    words[50:100] = 0
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "pxc")
        subprocess.run(["g++", "-std=c++17", "-O1", "-I", inc, "-o", exe,
                        os.path.join(HERE, "philox_torch_xcheck.cpp")], check=True)
        text = "\n".join(" ".join(str(int(v)) for v in row) for row in words) + "\n"
        out = subprocess.run([exe], input=text, capture_output=True, text=True, check=True).stdout
    ref = np.array([[int(t) for t in line.split()] for line in out.strip().splitlines()])
    assert ref.shape == (n, 4)
    for row, exp in zip(words[:: 7], ref[:: 7]):
        key = int(row[0]) | (int(row[1]) << 32)
        assert O.philox4x32_10(key, [int(v) for v in row[2:]]) == tuple(int(v) for v in exp)


# --------------------------------------------------------------------------
# Directions reconstructed from the tree: d(node) points from the node's vertex
# to the vertex of its children (or to its hit).
# --------------------------------------------------------------------------
def node_directions(r, sid):
    sel = np.nonzero(r["node_sid"] == sid)[0]
    key_to_local = {int(r["node_key"][j]): i for i, j in enumerate(sel)}
    V = np.stack([r["node_vx"][sel], r["node_vy"][sel], r["node_vz"][sel]], 1)
    target = {}
    for i, j in enumerate(sel):
        p = r["node_parent"][j]
        if p >= 0:
            target.setdefault(int(p), V[i])
    hs = np.nonzero(r["hit_sid"] == sid)[0]
    plane_z = lambda k: 1.0 + k
    for h in hs:
        i = key_to_local[int(r["hit_key"][h])]
        target.setdefault(i, np.array([r["hit_x"][h], r["hit_y"][h], plane_z(r["hit_plane"][h])]))
    D = np.full_like(V, np.nan)
    for i, t in target.items():
        v = t - V[i]
        D[i] = v / np.linalg.norm(v)
    return sel, V, D


def supav1_geom():
    """SUPAv1 (Table 2; appendix "Parameters"): split with certainty on the
    first seven sub-layers, stop with certainty on the eighth, theta = pi/24,
    no deviation (alpha = 0, i.e. every split halves the energy)."""
    return geom(n_planes=8, p_stop=[0.0] * 7 + [1.0], p_split=[1.0] * 7 + [0.0],
                e_cut=0.0, angle_mode="fixed", angle_a=math.pi / 24, frac_lo=0.5, frac_hi=0.5)


@pytest.mark.parametrize("polar,az", [(0.0, 0.0), (0.35, 2.1)])
def test_supav1_exact(polar, az):
    n = 6
    r = O.simulate(supav1_geom(), [65.0] * n, [polar] * n, [az] * n, seed=5)
    # exactly 2^7 = 128 points per event, all on sub-layer 7, all equal energy
    assert (r["counts"][:, 1] == 128).all()
    assert (r["counts"][:, 0] == 255).all() and (r["counts"][:, 3] == 127).all()
    assert (r["hit_plane"] == 7).all()
    assert (r["hit_e"] == 65 * 2 ** 14).all()                 # 65 / 128 = 0.5078125
    assert (r["ledger"][:, 0] == r["ledger"][:, 1]).all()      # everything deposited
    assert (r["ledger"][:, 2:] == 0).all()
    # geometry: every sibling pair opens by pi/24, each daughter deflects by pi/48
    for sid in range(n):
        sel, V, D = node_directions(r, sid)
        parent = r["node_parent"][sel]
        for p in range(len(sel)):
            kids = np.nonzero(parent == p)[0]
            if len(kids) == 0:
                continue
            assert len(kids) == 2
            a, b = D[kids[0]], D[kids[1]]
            assert abs(math.acos(np.clip(a @ b, -1, 1)) - math.pi / 24) < 1e-9
            for c in (a, b):
                assert abs(math.acos(np.clip(c @ D[p], -1, 1)) - math.pi / 48) < 1e-9


def test_hand_traced_single_split():
    """One split at plane 0, stop at plane 1, normal incidence: hits are at
    distance dz*tan(deflection) from the axis along the azimuth omega, on
    opposite sides; energies split by the 32-bit fraction w1 / 2^32."""
    g = geom(n_planes=2, p_split=[1.0, 0.0], p_stop=[0.0, 1.0], e_cut=0.0)
    seed, n = 77, 50
    r = O.simulate(g, [1.0] * n, [0.0] * n, [0.0] * n, seed=seed)
    assert (r["counts"][:, 1] == 2).all()
    for sid in range(n):
        w = O.philox4x32_10(seed, (0, sid, 1, 0))
        E = 2 ** S
        Ea = (E * w[1]) >> 32                       # F = w1 when f ~ U(0, 1)
        f = w[1] / TWO32
        theta = 0.1 * math.sqrt(-2.0 * math.log((w[2] + 0.5) / TWO32))
        omega = 2.0 * math.pi * (w[3] + 0.5) / TWO32
        h = np.nonzero(r["hit_sid"] == sid)[0]
        ka = h[r["hit_key"][h] == 2][0]
        kb = h[r["hit_key"][h] == 3][0]
        assert r["hit_e"][ka] == Ea and r["hit_e"][kb] == E - Ea
        ta, tb = math.tan(theta * (1 - f)), math.tan(theta * f)
        assert abs(r["hit_x"][ka] - ta * math.cos(omega)) < 1e-12
        assert abs(r["hit_y"][ka] - ta * math.sin(omega)) < 1e-12
        assert abs(r["hit_x"][kb] + tb * math.cos(omega)) < 1e-12
        assert abs(r["hit_y"][kb] + tb * math.sin(omega)) < 1e-12


def test_straight_line_and_leakage():
    """p_stop = p_split = 0: the primary flies straight and leaks out entirely;
    stopping it on the last plane puts the hit at x0 + z*tan(a)*(cos b, sin b)."""
    N = 7
    rng = np.random.default_rng(0)
    n = 40
    pol = rng.uniform(0, 1.2, n).astype(np.float32)
    az = rng.uniform(0, 2 * np.pi, n).astype(np.float32)
    x0 = rng.uniform(-2, 2, n).astype(np.float32)
    y0 = rng.uniform(-2, 2, n).astype(np.float32)
    e0 = rng.uniform(1, 50, n).astype(np.float32)
    r = O.simulate(geom(n_planes=N, p_stop=[0.0] * N, p_split=[0.0] * N), e0, pol, az,
                   seed=1, x0=x0, y0=y0)
    assert len(r["hit_e"]) == 0
    assert (r["ledger"][:, 3] == r["ledger"][:, 0]).all()
    assert (r["counts"][:, 2] == N).all() and (r["counts"][:, 4] == 1).all()
    r = O.simulate(geom(n_planes=N, p_stop=[0.0] * (N - 1) + [1.0], p_split=[0.0] * N),
                   e0, pol, az, seed=1, x0=x0, y0=y0)
    zl = 1.0 + (N - 1)
    tp = np.tan(pol.astype(np.float64))
    np.testing.assert_allclose(r["hit_x"], x0 + zl * tp * np.cos(az.astype(np.float64)),
                               rtol=0, atol=1e-12)
    np.testing.assert_allclose(r["hit_y"], y0 + zl * tp * np.sin(az.astype(np.float64)),
                               rtol=0, atol=1e-12)
    # E0 rounded to nearest in fixed point
    np.testing.assert_array_equal(r["hit_e"], np.rint(e0.astype(np.float64) * 2 ** S))


def test_energy_rounding_and_range():
    g = geom(n_planes=1, p_stop=[1.0], p_split=[0.0], e_cut=0.0)
    # ties round to even: 2^-22 is half a unit
    r = O.simulate(g, [2.0 ** -22, 3 * 2.0 ** -22], [0, 0], [0, 0], seed=0)
    assert list(r["hit_e"]) == [0, 2]
    with pytest.raises(ValueError):
        O.simulate(g, [2048.0], [0], [0], seed=0)        # 2048 * 2^21 = 2^32
    with pytest.raises(ValueError):
        O.simulate(g, [-1.0], [0], [0], seed=0)


def test_invalid_parameters_rejected():
    bad = [dict(n_planes=0), dict(n_planes=64), dict(dz=0.0), dict(z_first=0.0),
           dict(p_stop=[0.6] * 5, p_split=[0.5] * 5), dict(frac_lo=0.7, frac_hi=0.6),
           dict(e_cut=-1.0), dict(e_cut=float("nan"))]
    for b in bad:
        with pytest.raises(ValueError):
            O.simulate(geom(**b), [1.0], [0.0], [0.0], seed=0)


# --------------------------------------------------------------------------
# Distributions
# --------------------------------------------------------------------------
def test_free_path_geometric():
    """Constant interaction probability: the primary's first interaction plane
    is geometric with q = C2/2^32 (truncated at N), and a fraction C1/C2 of the
    interactions are stops."""
    N, n = 10, 20000
    ps, pl = 0.1, 0.2
    g = geom(n_planes=N, p_stop=[ps] * N, p_split=[pl] * N, e_cut=0.0)
    r = O.simulate(g, np.full(n, 5.0, np.float32), np.zeros(n, np.float32),
                   np.zeros(n, np.float32), seed=11)
    c1 = math.floor(ps * TWO32)
    c2 = c1 + math.floor(pl * TWO32)
    q = c2 / TWO32
    K = np.full(n, N)                 # N = never interacted
    stopped = np.zeros(n, bool)
    prim_hit = r["hit_key"] == 1
    K[r["hit_sid"][prim_hit]] = r["hit_plane"][prim_hit]
    stopped[r["hit_sid"][prim_hit]] = True
    kids = (r["node_parent"] == 0) & (r["node_key"] == 2)
    K[r["node_sid"][kids]] = np.rint(r["node_vz"][kids] - 1.0).astype(int)
    obs = np.bincount(K, minlength=N + 1)
    p = np.array([(1 - q) ** k * q for k in range(N)] + [(1 - q) ** N])
    assert stats.chisquare(obs, p * n).pvalue > 1e-3
    inter = K < N
    assert stats.binomtest(int(stopped[inter].sum()), int(inter.sum()), c1 / c2).pvalue > 1e-3


def _two_plane_splits(mode, a, b, flo, fhi, n, seed):
    g = geom(n_planes=2, p_split=[1.0, 0.0], p_stop=[0.0, 1.0], e_cut=0.0,
             angle_mode=mode, angle_a=a, angle_b=b, frac_lo=flo, frac_hi=fhi)
    rng = np.random.default_rng(seed)
    pol = rng.uniform(0, 0.6, n).astype(np.float32)
    az = rng.uniform(0, 2 * np.pi, n).astype(np.float32)
    r = O.simulate(g, np.full(n, 7.0, np.float32), pol, az, seed=seed)
    d = np.stack([np.sin(pol.astype(np.float64)) * np.cos(az.astype(np.float64)),
                  np.sin(pol.astype(np.float64)) * np.sin(az.astype(np.float64)),
                  np.cos(pol.astype(np.float64))], 1)
    split_pt = d / d[:, 2:3] * 1.0                     # vertex at z = 1
    out = {}
    for key, name in ((2, "a"), (3, "b")):
        m = r["hit_key"] == key
        sid = r["hit_sid"][m]
        hp = np.stack([r["hit_x"][m], r["hit_y"][m], np.full(m.sum(), 2.0)], 1)
        v = hp - split_pt[sid]
        out[name] = v / np.linalg.norm(v, axis=1, keepdims=True)
        out["e" + name] = r["hit_e"][m].astype(np.float64)
    return d, out


def test_opening_angle_rayleigh_and_fraction_uniform():
    sigma, n = 0.1, 6000
    d, o = _two_plane_splits("rayleigh", sigma, 0.0, 0.0, 1.0, n, 3)
    theta = np.arccos(np.clip(np.sum(o["a"] * o["b"], 1), -1, 1))
    assert stats.kstest(theta, lambda t: 1 - np.exp(-t ** 2 / (2 * sigma ** 2))).pvalue > 1e-3
    f = o["ea"] / (o["ea"] + o["eb"])           # daughter a carries E*f
    assert stats.kstest(f, "uniform").pvalue > 1e-3
    # deflections theta*(1-f) and theta*f, on opposite sides of d: the
    # transverse momenta E_a*theta*(1-f) and E_b*theta*f balance
    aa = np.arccos(np.clip(np.sum(o["a"] * d, 1), -1, 1))
    ab = np.arccos(np.clip(np.sum(o["b"] * d, 1), -1, 1))
    np.testing.assert_allclose(aa + ab, theta, atol=1e-9)
    np.testing.assert_allclose(aa, theta * (1 - f), atol=1e-6)


def test_splitting_azimuth_in_rodrigues_frame():
    """omega is uniform and is measured from R x, R y, with R the rotation
    about z cross d that takes +z to d (computed here with scipy)."""
    n = 4000
    d, o = _two_plane_splits("uniform", 0.05, 0.2, 0.25, 0.75, n, 9)
    axis = np.cross(np.array([0.0, 0.0, 1.0]), d)
    ang = np.arccos(np.clip(d[:, 2], -1, 1))
    nrm = np.linalg.norm(axis, axis=1, keepdims=True)
    rotvec = np.where(nrm > 0, axis / np.where(nrm > 0, nrm, 1) * ang[:, None], 0.0)
    R = Rotation.from_rotvec(rotvec)
    e1 = R.apply(np.array([1.0, 0.0, 0.0]))
    e2 = R.apply(np.array([0.0, 1.0, 0.0]))
    perp = o["a"] - np.sum(o["a"] * d, 1, keepdims=True) * d
    omega = np.mod(np.arctan2(np.sum(perp * e2, 1), np.sum(perp * e1, 1)), 2 * np.pi)
    assert stats.kstest(omega / (2 * np.pi), "uniform").pvalue > 1e-3
    # the b daughter lies on the opposite side (omega + pi)
    perp_b = o["b"] - np.sum(o["b"] * d, 1, keepdims=True) * d
    omega_b = np.arctan2(np.sum(perp_b * e2, 1), np.sum(perp_b * e1, 1))
    diff = np.angle(np.exp(1j * (omega_b - omega - np.pi)))
    assert np.abs(diff).max() < 1e-6
    # UNIFORM opening angle on [0.05, 0.2]; fraction on [1/4, 3/4]
    theta = np.arccos(np.clip(np.sum(o["a"] * o["b"], 1), -1, 1))
    assert stats.kstest(theta, "uniform", args=(0.05, 0.15)).pvalue > 1e-3
    f = o["ea"] / (o["ea"] + o["eb"])
    assert f.min() >= 0.25 - 1e-6 and f.max() < 0.75 + 1e-6


def test_cascade_mean_hits():
    """Split with certainty until below e_cut, planes enough that nothing
    leaks: N(x) = (2/x) int_0^x N(y) dy with N = 1 below e_cut gives
    E[hits] = 2 E0 / e_cut and E[nodes] = 4 E0 / e_cut - 1."""
    N, n, e_cut = 50, 3000, 0.1
    for E0 in (0.5, 3.0):
        r = O.simulate(geom(n_planes=N, e_cut=e_cut), np.full(n, E0, np.float32),
                       np.zeros(n, np.float32), np.zeros(n, np.float32), seed=21)
        hits = r["counts"][:, 1].astype(np.float64)
        assert r["ledger"][:, 3].sum() == 0
        se = hits.std(ddof=1) / math.sqrt(n)
        assert abs(hits.mean() - 2 * E0 / e_cut) < 4 * se
        nodes = r["counts"][:, 0].astype(np.float64)
        assert abs(nodes.mean() - (4 * E0 / e_cut - 1)) < 4 * nodes.std(ddof=1) / math.sqrt(n)


# --------------------------------------------------------------------------
# Invariants on random parameters
# --------------------------------------------------------------------------
def check_invariants(r, n):
    L = r["ledger"]
    assert (L[:, 1] + L[:, 2] + L[:, 3] == L[:, 0]).all()
    c = r["counts"]
    assert (c[:, 0] == 1 + 2 * c[:, 3]).all()
    assert (c[:, 1] + c[:, 4] == c[:, 3] + 1).all()
    assert (np.bincount(r["hit_sid"] - r["shower_id_base"], minlength=n) == c[:, 1]).all()
    assert (np.bincount(r["node_sid"] - r["shower_id_base"], minlength=n) == c[:, 0]).all()
    e_hits = np.zeros(n, np.uint64)
    np.add.at(e_hits, r["hit_sid"] - r["shower_id_base"], r["hit_e"].astype(np.uint64))
    assert (e_hits == L[:, 1] + L[:, 2]).all()
    # tree: daughters' energies sum to the parent's; keys 2p, 2p+1; generation + 1
    start = np.concatenate([[0], np.cumsum(c[:, 0])])
    for s in range(n):
        sl = slice(start[s], start[s + 1])
        par, key, e, gen = (r["node_parent"][sl], r["node_key"][sl], r["node_e"][sl],
                            r["node_gen"][sl])
        assert par[0] == -1 and key[0] == 1 and gen[0] == 0
        kids = np.nonzero(par >= 0)[0]
        assert (key[kids] // 2 == key[par[kids]]).all()
        assert (gen[kids] == gen[par[kids]] + 1).all()
        tot = np.zeros(len(par), np.uint64)
        np.add.at(tot, par[kids], e[kids].astype(np.uint64))
        has = np.unique(par[kids])
        assert (tot[has] == e[has]).all()
        assert len(np.unique(key)) == len(key)
        hk = r["hit_key"][r["hit_sid"] == s + r["shower_id_base"]]
        assert len(np.unique(hk)) == len(hk) and np.isin(hk, key).all()


def test_invariants_random_parameters():
    rng = np.random.default_rng(2024)
    for trial in range(25):
        N = int(rng.integers(1, 24))
        ps = rng.uniform(0, 0.4, N)
        pl = rng.uniform(0, 1, N) * (1 - ps)
        mode = ["fixed", "uniform", "rayleigh"][trial % 3]
        lo = rng.uniform(0, 0.5)
        g = geom(n_planes=N, p_stop=ps, p_split=pl, e_cut=float(rng.choice([0.0, 0.05, 0.3])),
                 angle_mode=mode, angle_a=float(rng.uniform(0.01, 0.4)),
                 angle_b=float(rng.uniform(0.4, 0.8)), frac_lo=lo,
                 frac_hi=float(rng.uniform(lo, 1.0)), z_first=float(rng.uniform(0.2, 2)),
                 dz=float(rng.uniform(0.1, 3)),
                 layer_of_plane=rng.integers(-1, N, N).astype(np.int32))
        n = 30
        e0 = rng.uniform(0, 30, n).astype(np.float32)
        pol = rng.uniform(0, 1.6, n).astype(np.float32)      # some point away from +z
        az = rng.uniform(0, 6.3, n).astype(np.float32)
        base = int(rng.integers(0, 2 ** 31))
        r = O.simulate(g, e0, pol, az, seed=int(rng.integers(0, 2 ** 63)), shower_id_base=base)
        check_invariants(r, n)
        assert (r["counts"][pol > np.pi / 2, 5] == 1).all()   # left at once


def test_chunked_runs_concatenate():
    """Counter-based randomness keyed by the global shower id: a batch run in
    chunks with shifted id bases equals the whole run."""
    g = geom(n_planes=12)
    rng = np.random.default_rng(4)
    n = 60
    e0 = rng.uniform(1, 20, n).astype(np.float32)
    pol = rng.uniform(0, 0.3, n).astype(np.float32)
    az = rng.uniform(0, 6, n).astype(np.float32)
    whole = O.simulate(g, e0, pol, az, seed=99, shower_id_base=1000)
    parts = [O.simulate(g, e0[s:s + 17], pol[s:s + 17], az[s:s + 17], seed=99,
                        shower_id_base=1000 + s) for s in range(0, n, 17)]
    for k in ("hit_x", "hit_y", "hit_e", "hit_key", "hit_sid", "node_e", "node_parent"):
        np.testing.assert_array_equal(whole[k], np.concatenate([p[k] for p in parts]))
    np.testing.assert_array_equal(whole["ledger"], np.concatenate([p["ledger"] for p in parts]))


# --------------------------------------------------------------------------
# Images (appendix "Downsampling") reduce to numpy.histogram2d
# --------------------------------------------------------------------------
def test_images_match_histogram2d():
    g = geom(n_planes=6)
    rng = np.random.default_rng(8)
    n = 25
    e0 = rng.uniform(1, 30, n).astype(np.float32)
    pol = rng.uniform(0, 0.5, n).astype(np.float32)
    az = rng.uniform(0, 6, n).astype(np.float32)
    r = O.simulate(g, e0, pol, az, seed=3)
    nx, ny, x0, x1, y0, y1 = 12, 9, -2.0, 2.0, -1.5, 1.5
    img = O.images(r, 6, nx, ny, x0, x1, y0, y1)
    for s in range(n):
        for layer in range(6):
            m = (r["hit_sid"] == s) & (r["hit_layer"] == layer) & (r["hit_x"] != x1) & (r["hit_y"] != y1)
            H, _, _ = np.histogram2d(r["hit_y"][m], r["hit_x"][m], bins=[ny, nx],
                                     range=[[y0, y1], [x0, x1]],
                                     weights=r["hit_e"][m].astype(np.float64))
            np.testing.assert_array_equal(img[s, layer].astype(np.float64), H)


# --------------------------------------------------------------------------
# Literal kinematics: Algorithm 1 as printed (lateral position only, one
# displacement +-dz (sin(theta/2 + eps), cos(theta/2 + eps)) per split)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("polar,az", [(0.0, 0.0), (0.35, 2.1)])
def test_supav1_literal_points_on_a_line(polar, az):
    """SUPAv1 with eps = 0: after seven splits each point sits at m dz (sin(pi/48),
    cos(pi/48)) with m the sum of seven signs, so m = -7, -5, ..., 7 with
    binomial multiplicities C(7, (m + 7)/2); the impact angles play no part."""
    g = dict(supav1_geom(), kinematics="literal")
    n = 4
    r = O.simulate(g, [65.0] * n, [polar] * n, [az] * n, seed=9, x0=[0.25] * n, y0=[-0.5] * n)
    assert (r["counts"][:, 1] == 128).all() and (r["hit_e"] == 65 * 2 ** 14).all()
    u = np.array([math.sin(math.pi / 48), math.cos(math.pi / 48)])
    for sid in range(n):
        h = r["hit_sid"] == sid
        d = np.stack([r["hit_x"][h] - 0.25, r["hit_y"][h] + 0.5], 1)
        m = d @ u                                        # coordinate along the line
        assert np.abs(d - np.outer(m, u)).max() < 1e-12  # nothing across it
        mi = np.rint(m).astype(int)
        assert np.abs(m - mi).max() < 1e-12
        vals, cnt = np.unique(mi, return_counts=True)
        assert list(vals) == list(range(-7, 8, 2))
        assert list(cnt) == [math.comb(7, (v + 7) // 2) for v in vals]


def test_literal_hand_traced_single_split_and_pass():
    """One split at plane 0, a pass at plane 1, a stop at plane 2: the first
    daughter (energy fraction f = w1/2^32) lands at p + dz (sin(theta/2 + eps),
    cos(theta/2 + eps)), eps = (f - 1/2) theta, the second at p - the same, and
    the pass leaves both where they were."""
    dz = 0.7
    g = geom(n_planes=3, dz=dz, z_first=1.0, p_split=[1.0, 0.0, 0.0], p_stop=[0.0, 0.0, 1.0],
             e_cut=0.0, kinematics="literal")
    seed, n = 31, 40
    x0 = np.linspace(-1, 1, n)
    r = O.simulate(g, [1.0] * n, [0.2] * n, [1.0] * n, seed=seed, x0=x0, y0=[0.5] * n)
    assert (r["counts"][:, 1] == 2).all()
    for sid in range(n):
        w = O.philox4x32_10(seed, (0, sid, 1, 0))
        f = w[1] / TWO32
        theta = 0.1 * math.sqrt(-2.0 * math.log((w[2] + 0.5) / TWO32))
        eps = (f - 0.5) * theta
        ux, uy = dz * math.sin(theta / 2 + eps), dz * math.cos(theta / 2 + eps)
        h = np.nonzero(r["hit_sid"] == sid)[0]
        ka = h[r["hit_key"][h] == 2][0]
        kb = h[r["hit_key"][h] == 3][0]
        assert r["hit_e"][ka] == (2 ** S * w[1]) >> 32
        assert abs(r["hit_x"][ka] - (float(np.float32(x0[sid])) + ux)) < 1e-12
        assert abs(r["hit_y"][ka] - (0.5 + uy)) < 1e-12
        assert abs(r["hit_x"][kb] - (float(np.float32(x0[sid])) - ux)) < 1e-12
        assert abs(r["hit_y"][kb] - (0.5 - uy)) < 1e-12


def test_literal_keeps_topology_and_energies():
    """The choices and energies come from the counters alone, so the two
    kinematics give the same tree, counts, energies and layers whenever no
    particle turns away from +z in the 3-D reading."""
    rng = np.random.default_rng(12)
    N = 12
    g = geom(n_planes=N, p_split=list(rng.uniform(0.3, 0.8, N)), p_stop=list(rng.uniform(0, 0.2, N)),
             e_cut=0.2, angle_mode="uniform", angle_a=math.pi / 32, angle_b=math.pi / 16,
             frac_lo=0.25, frac_hi=0.75, layer_of_plane=[-1] * 3 + [0] * 5 + [1] * 4)
    n = 60
    e0 = rng.uniform(1, 50, n)
    a = O.simulate(g, e0, [0.1] * n, [0.3] * n, seed=4)
    b = O.simulate(dict(g, kinematics="literal"), e0, [0.1] * n, [0.3] * n, seed=4)
    assert (a["counts"][:, 5] == 0).all()
    for k in ("counts", "ledger", "hit_key", "hit_e", "hit_layer", "hit_plane", "node_key", "node_e",
              "node_parent"):
        np.testing.assert_array_equal(a[k], b[k])
    assert not np.allclose(a["hit_x"], b["hit_x"])


def test_invalid_kinematics_rejected():
    with pytest.raises(KeyError):
        O.simulate(geom(n_planes=2, kinematics="other"), [1.0], [0.0], [0.0], seed=1)


def test_grid_images_match_histogram2d_per_layer():
    """Per-layer grids (the appendix "Downsampling": a region and a cell count
    per direction for each layer): every layer's image equals numpy's
    histogram2d of that layer's points, weighted by their energies."""
    rng = np.random.default_rng(17)
    n, m = 5, 4000
    grids = [(96, 3, -4.0, 4.0, -4.0, 4.0), (12, 12, -3.0, 5.0, -4.0, 4.0), (6, 12, -4.0, 4.0, -2.0, 2.5)]
    sid = rng.integers(0, n, m)
    layer = rng.integers(-1, 3, m)
    x = rng.normal(0, 2.5, m)
    y = rng.normal(0, 2.5, m)
    e = rng.integers(1, 2 ** 30, m).astype(np.uint64)
    img = O.grid_images(n, sid, layer, x, y, e, grids)
    off = 0
    for l, (nx, ny, x0, x1, y0, y1) in enumerate(grids):
        for s in range(n):
            k = (sid == s) & (layer == l)
            h, _, _ = np.histogram2d(y[k], x[k], bins=[ny, nx], range=[[y0, y1], [x0, x1]],
                                     weights=e[k].astype(np.float64))
            # histogram2d closes the last bin on the right; no point sits on an edge here
            np.testing.assert_array_equal(img[s, off:off + nx * ny].reshape(ny, nx), h.astype(np.uint64))
        off += nx * ny
    assert img.shape == (n, off)
    inside = np.zeros(m, bool)
    for l, g in enumerate(grids):
        inside |= (layer == l) & (x >= g[2]) & (x < g[3]) & (y >= g[4]) & (y < g[5])
    assert img.sum() == e[inside].sum()              # nothing lost or counted twice


# --------------------------------------------------------------------------
# Regional parameters: rings around the beam axis with their own p_stop, p_split
# --------------------------------------------------------------------------
def test_rings_with_equal_parameters_change_nothing():
    rng = np.random.default_rng(21)
    N = 10
    g = geom(n_planes=N, p_split=list(rng.uniform(0.3, 0.7, N)), p_stop=list(rng.uniform(0, 0.2, N)))
    rg = dict(g, n_regions=3, region_r=[0.05, 0.2], p_split=g["p_split"] * 3, p_stop=g["p_stop"] * 3)
    n = 80
    e0 = rng.uniform(1, 30, n)
    a = O.simulate(g, e0, [0.1] * n, [0.5] * n, seed=6)
    b = O.simulate(rg, e0, [0.1] * n, [0.5] * n, seed=6)
    for k in ("counts", "ledger", "hit_key", "hit_e", "hit_x", "hit_y", "node_key"):
        np.testing.assert_array_equal(a[k], b[k])
    assert np.isinf(a["region_margin"]).all() and np.isfinite(b["region_margin"]).all()


def test_rings_hand_traced():
    """Split at plane 0; at plane 1 a daughter inside radius r1 splits (its
    daughters leave after the last plane) and one outside stops.  The
    daughters' radii are dz tan(theta (1 - f)) and dz tan(theta f) (normal
    incidence), so the counts and the margin follow from the Philox words."""
    r1 = 0.06
    g = geom(n_planes=2, e_cut=0.0, n_regions=2, region_r=[r1],
             p_split=[1.0, 1.0] + [1.0, 0.0], p_stop=[0.0, 0.0] + [0.0, 1.0])
    seed, n = 19, 200
    r = O.simulate(g, [1.0] * n, [0.0] * n, [0.0] * n, seed=seed)
    seen = set()
    for sid in range(n):
        w = O.philox4x32_10(seed, (0, sid, 1, 0))
        f = w[1] / TWO32
        theta = 0.1 * math.sqrt(-2.0 * math.log((w[2] + 0.5) / TWO32))
        radii = [math.tan(theta * (1 - f)), math.tan(theta * f)]
        inner = sum(rr < r1 for rr in radii)
        seen.add(inner)
        c = r["counts"][sid]
        assert c[1] == 2 - inner                       # outer daughters stop: one hit each
        assert c[3] == 1 + inner and c[4] == 2 * inner  # inner ones split and leave
        want = min([r1] + [abs(rr - r1) for rr in radii])
        assert abs(r["region_margin"][sid] - want) < 1e-12
    assert seen == {0, 1, 2}


@pytest.mark.parametrize("bad", [dict(n_regions=5, region_r=[0.1, 0.2, 0.3, 0.4]),
                                 dict(n_regions=3, region_r=[0.2, 0.1]),
                                 dict(n_regions=2, region_r=[-0.1])])
def test_bad_rings_rejected(bad):
    R = bad["n_regions"]
    g = geom(n_planes=2, p_split=[1.0] * 2 * R, p_stop=[0.0] * 2 * R, **bad)
    with pytest.raises(ValueError):
        O.simulate(g, [1.0], [0.0], [0.0], seed=1)
