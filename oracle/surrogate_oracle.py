"""FP64 numpy oracle of the learned surrogate (test infrastructure only).

Only the test-suite and the benchmark's CPU-baseline leg import this module.

The surrogate is the build's extension of the paper's method: a conditional
MLP that maps a shower's initial condition (energy, polar angle, azimuth:
the conditioning variables of section "Extensions") plus Gaussian noise to
the mean and log-variance of its coarse per-layer deposit images (the image
representation of appendix "Downsampling").  Everything here is the plain
definition, written out:

  h_0 = x,  h_l = GELU(h_{l-1} W_l + b_l)  (hidden layers),
  out = h_L W_o + b_o = [mu | s],  s = log sigma^2 clamped to [-S, S],
  GELU(a) = a * Phi(a) = a/2 * (1 + erf(a / sqrt 2)),
  NLL = mean over bins and rows of 1/2 * (s + (y - mu)^2 exp(-s))
        (the Gaussian negative log-likelihood without its constant),
  Adam (Kingma & Ba, 2015) with bias correction,
  W1(a, b) = integral |F_a - F_b| = mean |a_(i) - b_(i)| for equal sizes.

Its random parts (noise inputs, sampled per-layer energies) take their
uniform words from Philox4x32-10 (Salmon et al., SC'11) and turn them into
normals by the Box-Muller transform; a layer's sampled energy treats its
bins as equicorrelated normals, whose sum has variance
(1 - rho) sum sigma^2 + rho (sum sigma)^2.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

SQRT2 = math.sqrt(2.0)
SQRT2PI = math.sqrt(2.0 * math.pi)
S_CLAMP = 20.0


def gelu(a):
    return 0.5 * a * (1.0 + erf(a / SQRT2))


def gelu_grad(a):
    """d/da of a * Phi(a) = Phi(a) + a * phi(a)."""
    return 0.5 * (1.0 + erf(a / SQRT2)) + a * np.exp(-0.5 * a * a) / SQRT2PI


def init_params(dims, rng):
    """He-style normal initialisation; dims = [in, h1, ..., out]."""
    params = []
    for din, dout in zip(dims[:-1], dims[1:]):
        params.append([rng.normal(0.0, math.sqrt(2.0 / din), size=(din, dout)),
                       np.zeros(dout)])
    return params


def forward(params, x):
    """Returns (out, cache); cache keeps pre-activations for the backward."""
    h = np.asarray(x, np.float64)
    cache = [h]
    for l, (W, b) in enumerate(params):
        a = h @ W + b
        if l < len(params) - 1:
            cache.append(a)
            h = gelu(a)
            cache.append(h)
        else:
            h = a
    return h, cache


def split_out(out, s_clamp=S_CLAMP):
    d = out.shape[1] // 2
    mu = out[:, :d]
    s_raw = out[:, d:]
    s = np.clip(s_raw, -s_clamp, s_clamp)
    return mu, s, s_raw


def nll(out, y, s_clamp=S_CLAMP):
    """Mean Gaussian NLL (without 1/2 log 2 pi) over all bins and rows."""
    mu, s, _ = split_out(out, s_clamp)
    return float(np.mean(0.5 * (s + (y - mu) ** 2 * np.exp(-s))))


def mse(out, y):
    """Half the mean squared error of the means."""
    mu = out[:, :out.shape[1] // 2]
    return float(np.mean(0.5 * (y - mu) ** 2))


def nll_grad(out, y, s_clamp=S_CLAMP, mse_mean=False):
    """d NLL / d out (the clamp passes no gradient outside [-S, S]).  With
    mse_mean the mean half is instead d mse / d mu (means fitted by squared
    error), and the log-variance half stays d NLL / d s at the given means."""
    mu, s, s_raw = split_out(out, s_clamp)
    n = y.size
    r = (y - mu) * np.exp(-s)
    d_mu = -(y - mu) / n if mse_mean else -r / n
    d_s = 0.5 * (1.0 - (y - mu) * r) / n
    d_s = np.where(np.abs(s_raw) <= s_clamp, d_s, 0.0)
    return np.concatenate([d_mu, d_s], axis=1)


def backward(params, cache, d_out):
    """Gradients [(dW, db), ...] of a scalar loss with d loss/d out = d_out."""
    grads = [None] * len(params)
    g = d_out
    L = len(params)
    for l in range(L - 1, -1, -1):
        W, _ = params[l]
        h_in = cache[2 * l] if l > 0 else cache[0]
        grads[l] = (h_in.T @ g, g.sum(axis=0))
        if l > 0:
            a_prev = cache[2 * l - 1]
            g = (g @ W.T) * gelu_grad(a_prev)
    return grads


def adam_step(params, grads, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update in place; t counts from 1."""
    for (p, g, mm, vv) in zip(params, grads, m, v):
        for q in range(2):
            mm[q] = b1 * mm[q] + (1 - b1) * g[q]
            vv[q] = b2 * vv[q] + (1 - b2) * g[q] ** 2
            mhat = mm[q] / (1 - b1 ** t)
            vhat = vv[q] / (1 - b2 ** t)
            p[q] -= lr * mhat / (np.sqrt(vhat) + eps)


def uncertainty(mu, s, n_layers):
    """Per shower: sqrt(sum of predicted variances) / max(sum of means, eps)."""
    var = np.exp(s)
    tot = np.maximum(mu.sum(axis=1), 1e-6)
    return np.sqrt(var.sum(axis=1)) / tot


def layer_sums(img, n_layers):
    """Per-layer totals of flattened images (rows = showers)."""
    return img.reshape(img.shape[0], n_layers, -1).sum(axis=2)


def w1(a, b):
    """1-D Wasserstein-1 distance between two samples (any sizes): integral of
    |F_a - F_b| over the real line, from the two empirical CDFs."""
    a = np.sort(np.asarray(a, np.float64))
    b = np.sort(np.asarray(b, np.float64))
    xs = np.concatenate([a, b])
    xs.sort()
    Fa = np.searchsorted(a, xs[:-1], side="right") / len(a)
    Fb = np.searchsorted(b, xs[:-1], side="right") / len(b)
    return float(np.sum(np.abs(Fa - Fb) * np.diff(xs)))


# ---------------------------------------------------------------------------
# The surrogate's random parts: Philox4x32-10 words, Box-Muller normals, the
# noise features of the network's inputs and the sampled per-layer energies
# of the gate.  The random numbers are not inputs here: both sides draw them
# from the same counter-based generator, each from its own implementation of
# the published definition.
# ---------------------------------------------------------------------------
_M32 = np.uint64(0xFFFFFFFF)


def philox4x32_10(key: int, c0, c1, c2, c3):
    """Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) over arrays of
    counters: ten rounds, each multiplying counter words 0 and 2 by the two
    round multipliers (full 64-bit products), the high halves mixed with
    words 1 and 3 and the round key, the key advanced by the two Weyl
    constants between rounds.  Returns the four output words (uint64 arrays
    holding 32-bit values)."""
    c = [np.asarray(v, np.uint64) & _M32 for v in np.broadcast_arrays(c0, c1, c2, c3)]
    k0, k1 = np.uint64(key & 0xFFFFFFFF), np.uint64((key >> 32) & 0xFFFFFFFF)
    m0, m1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
    for _ in range(10):
        p0 = m0 * c[0]
        p1 = m1 * c[2]
        c = [(p1 >> np.uint64(32)) ^ c[1] ^ k0, p1 & _M32, (p0 >> np.uint64(32)) ^ c[3] ^ k1, p0 & _M32]
        k0 = (k0 + np.uint64(0x9E3779B9)) & _M32
        k1 = (k1 + np.uint64(0xBB67AE85)) & _M32
    return c


def unit(w):
    """u(w) = (w + 1/2) / 2^32, in (0, 1)."""
    return (np.asarray(w, np.float64) + 0.5) * 2.0 ** -32


def box_muller(w_a, w_b):
    """Two independent standard normals from two uniform words (Box and
    Muller, 1958): r = sqrt(-2 ln u_a), angle 2 pi u_b; (r cos, r sin)."""
    r = np.sqrt(-2.0 * np.log(unit(w_a)))
    t = 2.0 * np.pi * unit(w_b)
    return r * np.cos(t), r * np.sin(t)


NOISE_TAG = 0x5EED
GATE_TAG = 0x9A7E


def features(e0, polar, az, e_scale, polar_scale, az_scale, n_noise, seed, row_base=0, stream_id=0):
    """Input rows of the network: the scaled initial condition, then n_noise
    standard normals.  Row b draws Philox blocks counted by (row_base + b,
    stream_id, NOISE_TAG, q), q = 0, 4, 8, ...; the words (w0, w1) and
    (w2, w3) of a block give normals q, q+1 and q+2, q+3."""
    e0 = np.asarray(e0, np.float64)
    B = len(e0)
    x = np.zeros((B, 3 + n_noise))
    x[:, 0] = e0 * e_scale
    x[:, 1] = np.asarray(polar, np.float64) * polar_scale
    x[:, 2] = np.asarray(az, np.float64) * az_scale
    rows = (np.arange(B, dtype=np.uint64) + np.uint64(row_base)) & _M32
    for q in range(0, n_noise, 4):
        w = philox4x32_10(seed, rows, stream_id, NOISE_TAG, q)
        z = list(box_muller(w[0], w[1])) + list(box_muller(w[2], w[3]))
        for e in range(4):
            if q + e < n_noise:
                x[:, 3 + q + e] = z[e]
    return x


def gate(out, e0, n_layers, y_scale, s_clamp=S_CLAMP, rho=-1.0, seed=0, row_base=0):
    """Per-layer energies and uncertainty score of each row of out = [mu | s].

    Layer l of row b: the bins' means and variances exp(s) (s clamped) are
    summed; with rho < 0 the energy is e0/y_scale * sum mu; with 0 <= rho <= 1
    it is a sample, e0/y_scale * (sum mu + sd z), where the bins of a layer
    are normal with correlation rho between any two of them, so the variance
    of their sum is sd^2 = (1 - rho) sum sigma^2 + rho (sum sigma)^2, and z is
    the first Box-Muller normal of the Philox block counted by
    (row_base + b, l, GATE_TAG, 0).  The score is sqrt(sum of all variances)
    / max(sum of all means, 1e-6)."""
    out = np.asarray(out, np.float64)
    B, D2 = out.shape
    D = D2 // 2
    mu, s, _ = split_out(out, s_clamp)
    m = layer_sums(mu, n_layers)
    var = layer_sums(np.exp(s), n_layers)
    sig = layer_sums(np.exp(0.5 * s), n_layers)
    v = m.copy()
    if rho >= 0:
        rows = ((np.arange(B, dtype=np.uint64) + np.uint64(row_base)) & _M32)[:, None]
        layers = np.arange(n_layers, dtype=np.uint64)[None, :]
        w = philox4x32_10(seed, rows, layers, GATE_TAG, 0)
        z, _ = box_muller(w[0], w[1])
        v = m + np.sqrt((1.0 - rho) * var + rho * sig * sig) * z
    scale = np.asarray(e0, np.float64)[:, None] / y_scale
    unc = np.sqrt(var.sum(axis=1)) / np.maximum(m.sum(axis=1), 1e-6)
    return v * scale, unc


def occupied(values, n_layers, thr):
    """Per row and layer, the number of cells whose value exceeds thr
    (values [rows, L * cells]): the occupied cells of an image, or of a
    predicted image."""
    v = np.asarray(values, np.float64)
    return (v.reshape(v.shape[0], n_layers, -1) > thr).sum(axis=2)
