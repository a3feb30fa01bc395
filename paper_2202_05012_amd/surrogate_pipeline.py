"""Training of the surrogate on simulated showers, and surrogate-plus-fallback
inference (argument marshalling; every step runs in the library's kernels).

Workload: initial conditions of the 100,000-shower, 20-plane workload
(E0 ~ U[1, 100], polar ~ U[0, 15 deg], azimuth ~ U[0, 2 pi)), images of
20 layers x 16 x 16 cells over [-5, 5)^2, drawn online (never stored).
"""
from __future__ import annotations

import math
import time

import numpy as np
import torch

from . import supa, surrogate as S, workloads

N_LAYERS = 20
GRID = 16
BINS = GRID * GRID
D = N_LAYERS * BINS
# a cell counts as occupied above a tenth of the energy threshold (the
# images have no hit counts, so the judge counts occupied cells instead)
OCC_THR = 0.01
# the per-layer head's targets: y_scale * (layer energy) / E0, of order one
# (a layer holds about 1/20 of E0)
Y_SCALE_HEAD = 20.0


def layer_head_dims():
    """The per-layer head: the image model's inputs and hidden layers, with the
    mean and log-variance of each of the 20 per-layer energies as outputs."""
    return [S.IN_PAD, 256, 256, 256, 256, 2 * N_LAYERS]


def geometry(grid=GRID):
    w = workloads.WORKLOADS["e1to100_20planes_img32_100k"]
    return workloads.geometry(w, img_nx=grid, img_ny=grid, img_x0=-5.0, img_x1=5.0,
                              img_y0=-5.0, img_y1=5.0)


def draw_ics(n, seed, device):
    """Initial conditions of the 100,000-shower workload's distribution."""
    w = workloads.WORKLOADS["e1to100_20planes_img32_100k"]
    e0, pol, az = workloads.initial_conditions(w, n, seed=seed)
    t = lambda a: torch.from_numpy(a).to(device)
    return t(e0), t(pol), t(az)


class ImageSimulator:
    """supa_simulate producing only per-layer images (no hit arrays): 16x16
    cells by default; with grid=1 one cell per layer over the same window,
    i.e. the per-layer energies alone."""

    def __init__(self, device=0, grid=GRID):
        self.sim = supa.Simulator(geometry(grid), supa.OUT_IMAGES, device=device)
        self.d = N_LAYERS * grid * grid

    def images(self, e0, pol, az, seed, shower_id_base=0):
        n = int(e0.shape[0])
        out = self.sim.allocate(n)
        st = self.sim.run(e0, pol, az, seed, out, shower_id_base=shower_id_base)
        assert st == 0
        return out["images"].view(n, self.d), out


def train(model: S.MLP | None, steps: int, batch: int, seed: int = 100, lr: float = 1e-3,
          log_every: int = 0, sim: ImageSimulator | None = None, device="cuda",
          mean_first: float = 0.0, head: S.MLP | None = None):
    """Online training: every step simulates a fresh batch (shower ids never
    repeat) and takes one Adam step for the image model: its log-variances on
    the Gaussian NLL, its means by squared error (fitted by the NLL, the many
    near-empty cells with tiny variances dominate the shared layers and the
    per-layer sums drift); the first `mean_first` fraction of the steps fit
    the means only (log-variance held at 0).  With `head`, the per-layer head
    takes a step on the same batch, its targets the images' per-layer sums,
    means and log-variances both on the Gaussian NLL.  Returns the image
    model's loss curve (and the head's) and the seconds taken."""
    sim = sim or ImageSimulator()
    losses, head_losses = [], []
    t0 = time.perf_counter()
    for step in range(steps):
        e0, pol, az = draw_ics(batch, seed + 1000003 * (step + 1), device)
        img, _ = sim.images(e0, pol, az, seed, shower_id_base=step * batch)
        x = S.features(e0, pol, az, seed, row_base=step * batch, stream_id=1)
        cur_lr = lr * (0.5 * (1 + math.cos(math.pi * step / max(steps, 1))) * 0.9 + 0.1)
        loss = model.train_step(x, img, e0, lr=cur_lr,
                                s_clamp=0.0 if step < mean_first * steps else None) \
            if model is not None else None
        # the head fits means and log-variances by the Gaussian NLL (it has no
        # near-empty outputs to dominate the fit; see the image model's step)
        hloss = head.train_step(x, S.group_sums(img, N_LAYERS), e0, lr=cur_lr, y_scale=Y_SCALE_HEAD,
                                mse_mean=False) if head is not None else None
        if log_every and (step % log_every == 0 or step == steps - 1):
            if model is not None:
                losses.append((step, float(loss.item())))
            if head is not None:
                head_losses.append((step, float(hloss.item())))
    torch.cuda.synchronize()
    if head is not None:
        return losses, head_losses, time.perf_counter() - t0
    return losses, time.perf_counter() - t0


def surrogate_layer_energies(model: S.MLP, e0, pol, az, seed, chunk=65536, row_base=0, rho=-1.0,
                             counts=False):
    """Predicted per-layer energies (sampled when rho >= 0) and uncertainty
    scores, in chunks; with counts, also the predicted occupied cells per
    layer (bins whose predicted energy exceeds OCC_THR)."""
    n = int(e0.shape[0])
    layer_e = torch.empty((n, N_LAYERS), dtype=torch.float32, device=e0.device)
    unc = torch.empty(n, dtype=torch.float32, device=e0.device)
    cnt = torch.empty((n, N_LAYERS), dtype=torch.float32, device=e0.device) if counts else None
    for s in range(0, n, chunk):
        sl = slice(s, min(n, s + chunk))
        x = S.features(e0[sl], pol[sl], az[sl], seed, row_base=row_base + s, stream_id=2)
        r = model.layer_energies(x, e0[sl], N_LAYERS, rho=rho, seed=seed, row_base=row_base + s,
                                 cnt_thr=OCC_THR if counts else None)
        layer_e[sl] = r[0]
        unc[sl] = r[1]
        if counts:
            cnt[sl] = r[2]
    return (layer_e, unc, cnt) if counts else (layer_e, unc)


def head_layer_energies(head: S.MLP, e0, pol, az, seed, chunk=1 << 20, row_base=0):
    """Per-layer energies sampled from the per-layer head (mean + sigma z per
    layer) and its uncertainty score sqrt(sum of layer variances) / (sum of
    layer means), in chunks."""
    n = int(e0.shape[0])
    layer_e = torch.empty((n, N_LAYERS), dtype=torch.float32, device=e0.device)
    unc = torch.empty(n, dtype=torch.float32, device=e0.device)
    for s in range(0, n, chunk):
        sl = slice(s, min(n, s + chunk))
        x = S.features(e0[sl], pol[sl], az[sl], seed, row_base=row_base + s, stream_id=2)
        le, u, _ = S.gate(head.forward_fused(x), e0[sl], N_LAYERS, rho=0.0, seed=seed, row_base=row_base + s,
                          y_scale=Y_SCALE_HEAD)
        layer_e[sl] = le
        unc[sl] = u
    return layer_e, unc


def head_with_fallback(head: S.MLP, e0, pol, az, seed, tau, sim: ImageSimulator):
    """Per-layer energies from the per-layer head, replaced by the
    simulator's (sim: a one-cell-per-layer ImageSimulator) for every shower
    whose uncertainty exceeds tau.  Returns (layer_e, n_fallback)."""
    layer_e, unc = head_layer_energies(head, e0, pol, az, seed)
    idx = S.select_above(unc, tau)
    m = int(idx.shape[0])
    if m:
        fe, fp, fa = S.gather3(idx, e0, pol, az)
        img, _ = sim.images(fe, fp, fa, seed, shower_id_base=0x40000000)
        S.scatter_rows(idx, S.group_sums(img, N_LAYERS), layer_e)
    return layer_e, m


def surrogate_with_fallback(model: S.MLP, e0, pol, az, seed, tau, sim: ImageSimulator,
                            chunk=65536, rho=-1.0):
    """Per-layer energies and occupied-cell counts: the surrogate's, replaced
    by the simulator's for every shower whose uncertainty exceeds tau.
    Returns (layer_e, layer_counts, n_fallback)."""
    layer_e, unc, cnt = surrogate_layer_energies(model, e0, pol, az, seed, chunk, rho=rho, counts=True)
    idx = S.select_above(unc, tau)
    m = int(idx.shape[0])
    if m:
        fe, fp, fa = S.gather3(idx, e0, pol, az)
        img, _ = sim.images(fe, fp, fa, seed, shower_id_base=0x40000000)
        S.scatter_rows(idx, S.group_sums(img, N_LAYERS), layer_e)
        S.scatter_rows(idx, S.occupied_counts(img, N_LAYERS, OCC_THR), cnt)
    return layer_e, cnt, m


def simulated_layer_energies(e0, pol, az, seed, sim: ImageSimulator, shower_id_base=0, counts=False):
    """The simulator's per-layer energies (and, with counts, occupied cells)."""
    img, _ = sim.images(e0, pol, az, seed, shower_id_base=shower_id_base)
    le = S.group_sums(img, N_LAYERS)
    return (le, S.occupied_counts(img, N_LAYERS, OCC_THR)) if counts else le


def judge(le, cnt, ref_le, ref_cnt):
    """The W1 judge on the GPU (supa_w1_equal): per layer, the exact W1 of
    the energies and of the occupied-cell counts against the simulator's on
    the same initial conditions, each relative to the simulator's mean per
    layer (averaged over layers).  Returns (max over layers of the relative
    energy W1, the same for counts, per-layer energy W1, per-layer count W1)."""
    we = S.w1_equal(le, ref_le).cpu().numpy()
    wc = S.w1_equal(cnt, ref_cnt).cpu().numpy()
    mean_e = float(ref_le.double().mean(dim=0).mean())
    mean_c = float(ref_cnt.double().mean(dim=0).mean())
    return float(we.max() / mean_e), float(wc.max() / mean_c), we, wc


def calibrate_rho(model: S.MLP, sim: ImageSimulator, n: int, seed: int, device="cuda"):
    """The bin correlation rho that matches the spread of the simulated
    per-layer energies around the predicted ones on a validation batch:
    E[(E_sim - E_pred)^2] = rho * A + (1 - rho) * B with A = (sum sigma)^2,
    B = sum sigma^2 (scaled by E0), least squares over showers and layers,
    clipped to [0, 1].  A one-off fit, done on the host in float64."""
    e0, pol, az = draw_ics(n, seed, device)
    sim_e = simulated_layer_energies(e0, pol, az, seed, sim, shower_id_base=0x60000000)
    x = S.features(e0, pol, az, seed, row_base=0x60000000, stream_id=3)
    out = model.forward(x)
    mean_e, _, _ = S.gate(out, e0, N_LAYERS)
    o = out.cpu().numpy().astype(np.float64)
    e0h = e0.cpu().numpy().astype(np.float64)[:, None] / S.Y_SCALE
    sig = np.exp(0.5 * np.clip(o[:, D:], -S.S_CLAMP, S.S_CLAMP)).reshape(n, N_LAYERS, BINS)
    A = (sig.sum(-1) * e0h) ** 2
    Bv = (sig ** 2).sum(-1) * e0h ** 2
    resid = (sim_e.cpu().numpy().astype(np.float64) - mean_e.cpu().numpy()) ** 2
    a = (A - Bv).ravel()
    r = (resid - Bv).ravel()
    return float(np.clip((a @ r) / max(a @ a, 1e-300), 0.0, 1.0))
