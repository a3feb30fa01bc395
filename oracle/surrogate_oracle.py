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
