"""The trained surrogate against the method without it (the plain simulator).

Trains on showers the simulator generates (online, a few hundred thousand),
then checks on held-out initial conditions that (1) the NLL went down,
(2) the surrogate's mean per-layer energies track the simulator's, and
(3) surrogate + fallback reaches W1 <= 2% of the mean per-layer energy at a
fallback fraction below 1, i.e. at a higher showers/s than simulating all.
"""
import numpy as np
import pytest
import torch

from paper_2202_05012_amd import surrogate as S, surrogate_pipeline as SP

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def test_training_gain_over_plain_simulator():
    dev = torch.device("cuda", 0)
    sim = SP.ImageSimulator()
    model = S.MLP(S.surrogate_dims(), device=dev, seed=1)
    losses, _ = SP.train(model, steps=60, batch=8192, seed=7, lr=2e-3, log_every=10, sim=sim)
    assert losses[-1][1] < losses[0][1] - 1.0, losses          # the NLL went down
    rho = SP.calibrate_rho(model, sim, 4096, seed=11)
    n = 65536
    e0, pol, az = SP.draw_ics(n, 4242, dev)
    ref = SP.simulated_layer_energies(e0, pol, az, 3, sim).cpu().numpy()
    mean_layer = ref.mean(axis=0).mean()
    sur, unc = SP.surrogate_layer_energies(model, e0, pol, az, 5, rho=rho)
    # mean per-layer energy profile within 10% of the simulator's, layer by layer
    prof_s, prof_r = sur.cpu().numpy().mean(axis=0), ref.mean(axis=0)
    big = prof_r > 0.05 * prof_r.max()
    assert (np.abs(prof_s[big] - prof_r[big]) <= 0.1 * prof_r[big]).all(), (prof_s, prof_r)
    unc_h = unc.cpu().numpy()
    reached = None
    for frac in (0.0, 0.1, 0.3, 0.5, 0.7, 0.9):
        tau = float(np.quantile(unc_h, 1 - frac)) if frac > 0 else np.inf
        le, m = SP.surrogate_with_fallback(model, e0, pol, az, 5, tau, sim, rho=rho)
        w = SP.w1_per_layer(le.cpu().numpy(), ref).max() / mean_layer
        if w <= 0.02:
            reached = (frac, m / n, w)
            break
    assert reached is not None and reached[1] < 1.0, reached
