"""The trained surrogate against the method without it (the plain simulator).

Trains on showers the simulator generates (online, 10 million), then checks
on held-out initial conditions that (1) the loss went down, (2) the
surrogate's mean per-layer energies track the simulator's (each layer within
5% of the mean per-layer energy), (3) the gate ranks showers usefully: W1 of
the per-layer energies and of the per-layer occupied-cell counts (the judge,
on the GPU, checked against the oracle's W1 once) falls as the fallback
fraction grows, (4) surrogate + fallback reaches W1 <= 2% of the mean
per-layer energy with part of the showers (not all) simulated, and (5) the
per-layer head, trained on the same batches, reaches that bar with no
showers simulated, its gate's uncertainty ranking useful too (W1 with half
the showers simulated below W1 with none).
"""
import numpy as np
import pytest
import torch

from oracle import surrogate_oracle as SO
from paper_2202_05012_amd import surrogate as S, surrogate_pipeline as SP

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def test_training_gain_over_plain_simulator():
    dev = torch.device("cuda", 0)
    sim = SP.ImageSimulator()
    model = S.MLP(S.surrogate_dims(), device=dev, seed=1)
    head = S.MLP(SP.layer_head_dims(), device=dev, seed=2)
    losses, hlosses, _ = SP.train(model, steps=1220, batch=8192, seed=7, lr=1e-3, log_every=200, sim=sim,
                                  head=head)
    assert losses[-1][1] < losses[0][1] - 1.0, losses          # the NLL went down
    assert hlosses[-1][1] < hlosses[0][1] - 1.0, hlosses
    rho = SP.calibrate_rho(model, sim, 4096, seed=11)
    n = 262144
    e0, pol, az = SP.draw_ics(n, 4242, dev)
    ref_t, ref_cnt = SP.simulated_layer_energies(e0, pol, az, 3, sim, counts=True)
    ref = ref_t.cpu().numpy()
    mean_layer = ref.mean(axis=0).mean()
    sur, unc = SP.surrogate_layer_energies(model, e0, pol, az, 5)
    # mean per-layer energy profile: every layer within 5% of the mean layer energy
    prof_s, prof_r = sur.cpu().numpy().mean(axis=0), ref.mean(axis=0)
    assert (np.abs(prof_s - prof_r) <= 0.05 * mean_layer).all(), (prof_s, prof_r)
    unc_h = unc.cpu().numpy()
    ws, wcs, reached = [], [], None
    for frac in (0.0, 0.5, 0.8, 0.95):
        tau = float(np.quantile(unc_h, 1 - frac)) if frac > 0 else np.inf
        le, cnt, m = SP.surrogate_with_fallback(model, e0, pol, az, 5, tau, sim, rho=rho)
        w, wc, we, _ = SP.judge(le, cnt, ref_t, ref_cnt)
        if frac == 0.5:
            # the judge on the GPU against the oracle's W1 on the host
            want = np.array([SO.w1(le.cpu().numpy()[:, l], ref[:, l]) for l in range(SP.N_LAYERS)])
            np.testing.assert_allclose(we, want, rtol=1e-9)
        ws.append(w)
        wcs.append(wc)
        if w <= 0.02 and reached is None:
            reached = (frac, m / n, w)
    assert ws[-1] < ws[0] and wcs[-1] < wcs[0], (ws, wcs)
    assert reached is not None and reached[1] < 1.0, (reached, ws)
    # the per-layer head, its fallback simulating one cell per layer
    sim1 = SP.ImageSimulator(grid=1)
    hw = []
    for frac in (0.0, 0.5):
        _, hunc = SP.head_layer_energies(head, e0, pol, az, 5)
        hu = hunc.cpu().numpy()
        tau = float(np.quantile(hu, 1 - frac)) if frac > 0 else np.inf
        le, m = SP.head_with_fallback(head, e0, pol, az, 5, tau, sim1)
        assert m == int((hu > tau).sum())
        hw.append(SP.judge(le, ref_cnt, ref_t, ref_cnt)[0])
    assert hw[0] <= 0.02 and hw[1] < hw[0], hw
