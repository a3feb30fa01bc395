"""Pins of the surrogate oracle: library routines and finite differences."""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import surrogate_oracle as S


def test_gelu_is_x_times_normal_cdf():
    a = np.linspace(-6, 6, 1001)
    np.testing.assert_allclose(S.gelu(a), a * stats.norm.cdf(a), rtol=1e-13, atol=1e-15)


def test_gelu_grad_finite_difference():
    a = np.linspace(-5, 5, 101)
    h = 1e-6
    fd = (S.gelu(a + h) - S.gelu(a - h)) / (2 * h)
    np.testing.assert_allclose(S.gelu_grad(a), fd, rtol=1e-7, atol=1e-9)


def test_nll_is_gaussian_logpdf_up_to_constant():
    rng = np.random.default_rng(1)
    mu = rng.normal(size=(7, 5))
    s = rng.uniform(-3, 3, size=(7, 5))
    y = rng.normal(size=(7, 5))
    out = np.concatenate([mu, s], axis=1)
    ref = -stats.norm.logpdf(y, loc=mu, scale=np.exp(0.5 * s)) - 0.5 * math.log(2 * math.pi)
    assert abs(S.nll(out, y) - ref.mean()) < 1e-12


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(2)
    dims = [5, 8, 8, 6]          # toy width 8, 3 outputs mu + 3 log-variances
    params = S.init_params(dims, rng)
    for W, b in params:
        b += rng.normal(0, 0.1, size=b.shape)
    x = rng.normal(size=(4, 5))
    y = rng.normal(size=(4, 3))
    out, cache = S.forward(params, x)
    grads = S.backward(params, cache, S.nll_grad(out, y))
    h = 1e-6
    for l, (W, b) in enumerate(params):
        for arr, g in ((W, grads[l][0]), (b, grads[l][1])):
            it = np.nditer(arr, flags=["multi_index"])
            for _ in it:
                idx = it.multi_index
                old = arr[idx]
                arr[idx] = old + h
                up = S.nll(S.forward(params, x)[0], y)
                arr[idx] = old - h
                dn = S.nll(S.forward(params, x)[0], y)
                arr[idx] = old
                fd = (up - dn) / (2 * h)
                assert abs(g[idx] - fd) <= 1e-7 * max(1.0, abs(fd)) + 1e-9, (l, idx, g[idx], fd)


def test_clamped_log_variance_has_no_gradient():
    out = np.array([[0.0, 25.0], [0.0, -30.0]])
    y = np.array([[1.0], [1.0]])
    g = S.nll_grad(out, y)
    assert g[0, 1] == 0.0 and g[1, 1] == 0.0


def test_adam_first_step_moves_by_lr_times_sign():
    p = [[np.array([1.0, -2.0, 3.0]), np.array([0.5])]]
    g = [(np.array([0.3, -4.0, 1e-3]), np.array([-2.0]))]
    m = [[np.zeros(3), np.zeros(1)]]
    v = [[np.zeros(3), np.zeros(1)]]
    S.adam_step(p, g, m, v, t=1, lr=0.01, eps=0.0)
    np.testing.assert_allclose(p[0][0], [1.0 - 0.01, -2.0 + 0.01, 3.0 - 0.01], rtol=1e-12)
    np.testing.assert_allclose(p[0][1], [0.5 + 0.01], rtol=1e-12)


def test_w1_matches_scipy():
    rng = np.random.default_rng(3)
    for na, nb in ((100, 100), (57, 230), (1, 9)):
        a = rng.gamma(2.0, size=na)
        b = rng.normal(1.0, 2.0, size=nb)
        assert abs(S.w1(a, b) - stats.wasserstein_distance(a, b)) < 1e-12


def test_w1_shift_and_identity():
    a = np.random.default_rng(4).normal(size=500)
    assert S.w1(a, a) == 0.0
    assert abs(S.w1(a, a + 0.7) - 0.7) < 1e-12


def test_uncertainty_and_layer_sums():
    mu = np.array([[1.0, 2.0, 3.0, 4.0]])
    s = np.log(np.array([[1.0, 4.0, 0.0 + 1e-300, 4.0]]))
    u = S.uncertainty(mu, s, 2)
    assert abs(u[0] - 3.0 / 10.0) < 1e-12
    np.testing.assert_array_equal(S.layer_sums(mu, 2), [[3.0, 7.0]])


def test_mse_mean_gradient_finite_differences():
    """Means fitted by squared error, log-variances by the NLL: each half of
    the gradient is the central difference of its own objective."""
    rng = np.random.default_rng(11)
    out = rng.normal(size=(5, 8))
    y = rng.normal(size=(5, 4))
    g = S.nll_grad(out, y, s_clamp=20.0, mse_mean=True)
    h = 1e-6
    for (r, c) in [(0, 0), (2, 3), (4, 1)]:          # mean half
        up, dn = out.copy(), out.copy()
        up[r, c] += h
        dn[r, c] -= h
        fd = (S.mse(up, y) - S.mse(dn, y)) / (2 * h)
        assert abs(fd - g[r, c]) < 1e-7 * max(1.0, abs(fd))
    for (r, c) in [(1, 4), (3, 7)]:                  # log-variance half
        up, dn = out.copy(), out.copy()
        up[r, c] += h
        dn[r, c] -= h
        fd = (S.nll(up, y, 20.0) - S.nll(dn, y, 20.0)) / (2 * h)
        assert abs(fd - g[r, c]) < 1e-7 * max(1.0, abs(fd))
    # and the plain mode differs from it only in the mean half
    g0 = S.nll_grad(out, y, s_clamp=20.0)
    np.testing.assert_array_equal(g0[:, 4:], g[:, 4:])
    assert not np.allclose(g0[:, :4], g[:, :4])


# ---------------------------------------------------------------------------
# the random parts: Philox words, Box-Muller normals, noise features and the
# sampled per-layer energies, pinned to published vectors, an independent
# generator and distributions derived separately
# ---------------------------------------------------------------------------
def test_numpy_philox_matches_published_vectors_and_the_c_oracle():
    import os
    from oracle import supa_oracle
    path = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    assert rows
    for r in rows:
        v = [int(t, 16) for t in r if t != "->"]
        ctr, key, want = v[0:4], v[4] | (v[5] << 32), v[6:10]
        got = S.philox4x32_10(key, *ctr)
        assert [int(g) for g in got] == want
    rng = np.random.default_rng(9)
    c = rng.integers(0, 2 ** 32, size=(4, 3000), dtype=np.uint64)
    key = int(rng.integers(0, 2 ** 63))
    w = S.philox4x32_10(key, *c)
    for i in range(0, 3000, 131):
        assert tuple(int(x[i]) for x in w) == supa_oracle.philox4x32_10(key, [int(t[i]) for t in c])


def test_noise_features_are_independent_standard_normals():
    from scipy import stats
    B = 40000
    x = S.features(np.linspace(1, 100, B), np.zeros(B), np.zeros(B), 0.01, 1.0, 1.0, 16, seed=77,
                    row_base=5, stream_id=2)
    np.testing.assert_allclose(x[:, 0], np.linspace(1, 100, B) * 0.01)
    z = x[:, 3:]
    assert stats.kstest(z.ravel(), "norm").pvalue > 1e-3
    assert abs(z.mean()) < 0.005 and abs(z.std() - 1) < 0.005
    # columns uncorrelated (the two normals of a pair, and across blocks)
    cc = np.corrcoef(z.T)
    assert np.abs(cc - np.eye(16)).max() < 0.03
    # another stream or seed gives other numbers; the same ones repeat
    y = S.features(np.ones(B), np.zeros(B), np.zeros(B), 1, 1, 1, 16, seed=77, row_base=5, stream_id=3)
    assert np.abs(np.corrcoef(z[:, 0], y[:, 3])[0, 1]) < 0.03
    x2 = S.features(np.linspace(1, 100, B), np.zeros(B), np.zeros(B), 0.01, 1.0, 1.0, 16, seed=77,
                     row_base=5, stream_id=2)
    np.testing.assert_array_equal(x, x2)
    # a row's noise depends on its global row id only
    x3 = S.features(np.ones(10), np.zeros(10), np.zeros(10), 1, 1, 1, 16, seed=77, row_base=105,
                     stream_id=2)
    np.testing.assert_array_equal(x3[:, 3:], z[100:110])


@pytest.mark.parametrize("rho", [0.0, 0.4, 1.0])
def test_sampled_layer_energy_is_the_sum_of_correlated_bins(rho):
    """The sampled energy of a layer against a Monte Carlo of what it stands
    for: bins drawn as normals N(mu_b, sigma_b^2) with correlation rho
    between any two (a common normal with weight sqrt(rho), an own one with
    weight sqrt(1 - rho)), summed.  Two-sample KS test on many rows of the
    same prediction."""
    from scipy import stats
    rng = np.random.default_rng(int(rho * 10) + 1)
    L, bins, B = 3, 16, 30000
    D = L * bins
    mu = rng.uniform(0, 2, D)
    s = rng.uniform(-3, 1, D)
    out = np.tile(np.concatenate([mu, s]), (B, 1))
    e0 = np.full(B, 50.0)
    le, unc = S.gate(out, e0, L, y_scale=100.0, rho=rho, seed=3, row_base=11)
    sig = np.exp(0.5 * s)
    common = rng.normal(size=(B, 1))
    own = rng.normal(size=(B, D))
    bins_mc = mu + sig * (np.sqrt(rho) * common + np.sqrt(1 - rho) * own)
    mc = bins_mc.reshape(B, L, bins).sum(axis=2) * 0.5
    for l in range(L):
        assert stats.ks_2samp(le[:, l], mc[:, l]).pvalue > 1e-3, l
    # rho < 0: the means, and the score of the oracle's uncertainty()
    lm, um = S.gate(out[:5], e0[:5], L, y_scale=100.0)
    np.testing.assert_allclose(lm, S.layer_sums(out[:5, :D], L) * 0.5)
    np.testing.assert_allclose(um, S.uncertainty(out[:5, :D], out[:5, D:], L))
    # layers of a row draw independent normals
    z = (le - mu.reshape(L, bins).sum(axis=1) * 0.5)
    assert np.abs(np.corrcoef(z.T) - np.eye(L)).max() < 0.03


def test_occupied_cells_by_hand():
    img = np.array([[0.0, 0.2, 0.01, 0.5, 0.011, 0.0],
                    [1.0, 1.0, 1.0, 0.0, 0.0, 0.009]])
    np.testing.assert_array_equal(S.occupied(img, 2, 0.01), [[1, 2], [3, 0]])
    np.testing.assert_array_equal(S.occupied(img, 1, 0.0), [[4], [4]])
