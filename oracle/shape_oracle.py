"""Shower shape variables of hit clouds, and the mean discrepancy between two
samples of them -- the plain FP64 definitions (numpy), shower by shower.

Test infrastructure only (tests and the benchmark's host baseline); the
device kernel (supa_shapes.hip) shares nothing with this file.

Definitions (paper, section "Shower Shape Variables" and the appendix
"More shower shape variables"), for the points j of layer i of one shower,
with lateral coordinates eta = x, phi = y, r = sqrt(x^2 + y^2) and energy E:
  feature means      <x>, <y>, <r>, <E>           unweighted means over the points
  feature std devs   sqrt(<v^2> - <v>^2)           unweighted, for v in x, y, r, E
  layer energy       E_i = sum_j E_j
  layer centroids    <v>_E = sum_j E_j v_j / E_i   for v in x, y, r
  lateral widths     sqrt(sum_j E_j v_j^2 / E_i - <v>_E^2)
  energy fraction    f_i = E_i / E_tot
  energy ratio       (E[1] - E[2]) / (E[1] + E[2]), the two largest point
                     energies of the layer (E[2] = 0 with one point)
and per shower
  total energy       E_tot = sum_i E_i
  depth              d = the deepest layer with a non-zero deposit (-1: none)
  weighted energy    l_d = sum_i i E_i
  shower depth       s_d = l_d / E_tot
  depth width        sqrt(sum_i i^2 E_i / E_tot - s_d^2)
Readings where the paper is silent: layers are numbered from 0; a layer
without points has count 0, energy 0, fraction E_i / E_tot, and NaN for
every mean, deviation, centroid, width and ratio (as does a layer whose
energy is 0 for the weighted ones); a shower without energy has NaN s_d,
depth width and fractions; a variance that rounds below 0 is taken as 0; the
depth width sums over every layer (the printed formula's upper bound 2 is the
three layers of the calorimeter it was written for).

Mean discrepancy (paper, section "Performance Analysis of Generative
Models"): for each variable, both samples are normalised by the mean and
standard deviation of the reference (ground-truth) sample, the 1-D
Wasserstein-1 distance between the histograms of the normalised samples is
taken, and the distances are averaged over a group of variables.  Readings
where the paper is silent: the histograms share n_bins equal bins over the
range of the two samples together, each bin's mass sitting at its centre
(n_bins = None takes the exact distance of the empirical distributions, the
limit of many bins); the deviation is the population one; non-finite
entries are dropped; a column whose finite reference values are fewer than
two or all equal, or whose sample has none, is skipped.
"""
from __future__ import annotations

import numpy as np

LAYER_VARS = ("count", "mean_x", "mean_y", "mean_r", "mean_e", "std_x", "std_y", "std_r", "std_e",
              "energy", "centroid_x", "centroid_y", "centroid_r", "width_x", "width_y", "width_r",
              "fraction", "energy_ratio")
SHOWER_VARS = ("e_tot", "depth", "l_d", "s_d", "s_d_width")


def _std(m1, m2):
    return np.sqrt(max(m2 - m1 * m1, 0.0))


def layer_variables(x, y, e):
    """The per-layer variables (except the fraction) of one layer's points."""
    x, y, e = (np.asarray(v, np.float64) for v in (x, y, e))
    n = len(e)
    out = dict.fromkeys(LAYER_VARS, np.nan)
    out["count"] = float(n)
    out["energy"] = float(e.sum()) if n else 0.0
    if n == 0:
        return out
    r = np.sqrt(x * x + y * y)
    for name, v in (("x", x), ("y", y), ("r", r), ("e", e)):
        out["mean_" + name] = v.mean()
        out["std_" + name] = _std(v.mean(), (v * v).mean())
    E = out["energy"]
    if E > 0:
        for name, v in (("x", x), ("y", y), ("r", r)):
            c = (e * v).sum() / E
            out["centroid_" + name] = c
            out["width_" + name] = _std(c, (e * v * v).sum() / E)
    top = np.sort(e)[::-1]
    e1 = top[0]
    e2 = top[1] if n > 1 else 0.0
    out["energy_ratio"] = (e1 - e2) / (e1 + e2) if e1 + e2 > 0 else np.nan
    return out


def shower_variables(layer_energy):
    """E_tot, depth, l_d, s_d and the depth width from per-layer energies."""
    le = np.asarray(layer_energy, np.float64)
    i = np.arange(len(le), dtype=np.float64)
    tot = le.sum()
    nz = np.nonzero(le > 0)[0]
    depth = float(nz.max()) if len(nz) else -1.0
    ld = (i * le).sum()
    if tot > 0:
        sd = ld / tot
        width = _std(sd, (i * i * le).sum() / tot)
    else:
        sd = width = np.nan
    return {"e_tot": tot, "depth": depth, "l_d": ld, "s_d": sd, "s_d_width": width}


def shapes(n_showers, n_layers, sid, layer, x, y, e):
    """Shape variables of every shower of a hit cloud given as flat arrays
    (shower index sid in [0, n_showers), layer, x, y, e per hit): returns
    (per_layer [n][L][18], per_shower [n][5]) float64, columns in the order
    of LAYER_VARS and SHOWER_VARS."""
    sid = np.asarray(sid)
    layer = np.asarray(layer)
    per_layer = np.full((n_showers, n_layers, len(LAYER_VARS)), np.nan)
    per_shower = np.full((n_showers, len(SHOWER_VARS)), np.nan)
    order = np.lexsort((layer, sid))
    sid_s, layer_s = sid[order], layer[order]
    x_s, y_s, e_s = (np.asarray(v)[order] for v in (x, y, e))
    bounds = np.searchsorted(sid_s, np.arange(n_showers + 1))
    for s in range(n_showers):
        a, b = bounds[s], bounds[s + 1]
        le = np.zeros(n_layers)
        for l in range(n_layers):
            m = slice(a, b)
            sel = layer_s[m] == l
            v = layer_variables(x_s[m][sel], y_s[m][sel], e_s[m][sel])
            per_layer[s, l] = [v[k] for k in LAYER_VARS]
            le[l] = v["energy"]
        sv = shower_variables(le)
        per_shower[s] = [sv[k] for k in SHOWER_VARS]
        tot = sv["e_tot"]
        per_layer[s, :, LAYER_VARS.index("fraction")] = le / tot if tot > 0 else np.nan
    return per_layer, per_shower


def w1(a, b):
    """1-D Wasserstein-1 distance of two samples (any sizes): the integral of
    |F_a - F_b| over the merged support."""
    a = np.sort(np.asarray(a, np.float64))
    b = np.sort(np.asarray(b, np.float64))
    allv = np.concatenate([a, b])
    allv.sort()
    d = np.diff(allv)
    fa = np.searchsorted(a, allv[:-1], side="right") / len(a)
    fb = np.searchsorted(b, allv[:-1], side="right") / len(b)
    return float(np.sum(np.abs(fa - fb) * d))


def hist_bins(v, lo, hi, n_bins):
    """Bin index of each value for n_bins equal bins over [lo, hi]: floor of
    (v - lo) * (n_bins / (hi - lo)) in double precision, the top edge put in
    the last bin; every value in bin 0 when hi == lo."""
    v = np.asarray(v, np.float64)
    w = np.float64(hi) - np.float64(lo)
    if w == 0:
        return np.zeros(len(v), np.int64)
    scale = np.float64(n_bins) / w
    k = np.floor((v - np.float64(lo)) * scale).astype(np.int64)
    return np.clip(k, 0, n_bins - 1)


def hist_w1(a, b, n_bins):
    """Wasserstein-1 distance between the histograms of a and b over n_bins
    shared equal bins spanning both samples, each bin's mass at its centre:
    bin width times the sum over bins of |F_a - F_b| (cumulative fractions)."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    lo = min(a.min(), b.min())
    hi = max(a.max(), b.max())
    ca = np.bincount(hist_bins(a, lo, hi, n_bins), minlength=n_bins)
    cb = np.bincount(hist_bins(b, lo, hi, n_bins), minlength=n_bins)
    fa = np.cumsum(ca) / len(a)
    fb = np.cumsum(cb) / len(b)
    return float((hi - lo) / n_bins * np.sum(np.abs(fa - fb)))


def w1_columns(reference, sample, n_bins=None):
    """Per column: W1 between the reference and the sample after normalising
    both by the reference column's mean and standard deviation (histograms of
    n_bins bins, or the exact empirical distance when n_bins is None); NaN
    for a skipped column (see the module's readings)."""
    ref = np.asarray(reference, np.float64)
    smp = np.asarray(sample, np.float64)
    out = np.full(ref.shape[1], np.nan)
    for c in range(ref.shape[1]):
        r = ref[:, c][np.isfinite(ref[:, c])]
        s = smp[:, c][np.isfinite(smp[:, c])]
        if len(r) < 2 or len(s) < 1 or r.min() == r.max():
            continue
        mu, sd = r.mean(), r.std()
        if n_bins is None:
            out[c] = w1((r - mu) / sd, (s - mu) / sd)
        else:
            out[c] = hist_w1(r, s, n_bins) / sd
    return out


def group_means(values, group_of_col, n_groups):
    """Mean of the non-NaN values of each group (NaN for an empty group)."""
    values = np.asarray(values, np.float64)
    g = np.asarray(group_of_col)
    out = np.full(n_groups, np.nan)
    for k in range(n_groups):
        v = values[(g == k) & ~np.isnan(values)]
        if len(v):
            out[k] = v.mean()
    return out


def mean_discrepancy(reference, sample, n_bins=None):
    """Mean over the columns of the normalised W1 (w1_columns), skipped
    columns left out."""
    d = w1_columns(reference, sample, n_bins)
    d = d[~np.isnan(d)]
    return float(d.mean()) if len(d) else float("nan")
