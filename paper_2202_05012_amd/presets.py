"""The paper's standard configurations SUPAv1-v5 (section "SUPA Datasets",
Table 2; appendix "Parameters"), as parameter dicts for supa.Simulator.

Table 2 fixes, per configuration, the splitting angle theta, the deviation
eps (Table 2's alpha), the layer configuration and the incident particle
(65 energy units, perpendicular, at the origin).  The energy fraction of the
first daughter is f = 1/2 + eps/theta, so eps ~ U(-theta/4, theta/4) is
f ~ U(1/4, 3/4) and eps = 0 is f = 1/2.  Sub-layers outside every layer are
dead material (layer -1: their hits are kept in the clouds with layer -1 and
left out of images).

Only SUPAv1's stopping and splitting probabilities are stated in the text
(split with certainty on sub-layers 0-6, stop with certainty on sub-layer 7).
Those of SUPAv2-v5 are given only as curves in a figure, so they must be
passed in (one value per sub-layer); the presets fill in everything else.
"""
from __future__ import annotations

import math

E0 = 65.0
N_PLANES = {1: 11, 2: 21, 3: 21, 4: 13, 5: 29}
LAYERS = {1: [(5, 10)], 2: [(7, 20)], 3: [(7, 20)], 4: [(7, 12)], 5: [(7, 12), (13, 28)]}


def layer_of_plane(version: int):
    """Sub-layer -> layer index (-1 outside every layer) from Table 2."""
    lop = [-1] * N_PLANES[version]
    for i, (a, b) in enumerate(LAYERS[version]):
        for k in range(a, b + 1):
            lop[k] = i
    return lop


def supa(version: int, p_split=None, p_stop=None, kinematics: str = "3d", e_cut: float = 0.0,
         dz: float = 1.0, image=None) -> dict:
    """Parameters of SUPAv<version>.  p_split / p_stop: per sub-layer
    probabilities (required for v2-v5, fixed for v1).  image: optional
    (nx, ny, x0, x1, y0, y1) grid for image outputs."""
    if version not in N_PLANES:
        raise ValueError("SUPA versions are 1..5")
    N = N_PLANES[version]
    if version == 1:
        if p_split is not None or p_stop is not None:
            raise ValueError("SUPAv1's probabilities are fixed by the paper")
        p_split = [1.0] * 7 + [0.0] * (N - 7)
        p_stop = [0.0] * 7 + [1.0] + [0.0] * (N - 8)
    elif p_split is None or p_stop is None:
        raise ValueError(f"SUPAv{version}'s p_split and p_stop per sub-layer are only plotted in the "
                         f"paper: pass {N} values of each")
    if len(p_split) != N or len(p_stop) != N:
        raise ValueError(f"SUPAv{version} has {N} sub-layers")
    if version <= 2:
        angle = dict(angle_mode="fixed", angle_a=math.pi / 24, angle_b=0.0, frac_lo=0.5, frac_hi=0.5)
    else:
        angle = dict(angle_mode="uniform", angle_a=math.pi / 32, angle_b=math.pi / 16, frac_lo=0.25,
                     frac_hi=0.75)
    g = dict(n_planes=N, z_first=dz, dz=dz, layer_of_plane=layer_of_plane(version),
             p_split=[float(v) for v in p_split], p_stop=[float(v) for v in p_stop], e_cut=e_cut,
             frac_bits=21, kinematics=kinematics, **angle)
    if image is not None:
        nx, ny, x0, x1, y0, y1 = image
        g.update(img_nx=nx, img_ny=ny, img_x0=x0, img_x1=x1, img_y0=y0, img_y1=y1)
    return g


def incident(n: int):
    """Initial conditions of every configuration: E0 = 65, perpendicular
    incidence (polar angle 0), impact point (0, 0)."""
    return [E0] * n, [0.0] * n, [0.0] * n


# CaloGAN's read-out (section "Downsampling"/appendix: 3 x 96, 12 x 12 and
# 12 x 6 cells for layers 0, 1, 2 at the "1x" resolution, multiples at 2x
# and 3x).  Rows x columns = phi (y) x eta (x) cells; the three layers cover
# the same square region of interest, as CaloGAN's layers do.
CALOGAN_CELLS = [(96, 3), (12, 12), (6, 12)]     # (nx, ny) per layer at 1x


def calogan_grids(scale: int = 1, half_width: float = 5.0):
    """Per-layer grids (nx, ny, x0, x1, y0, y1) of the three CaloGAN-like
    layers at resolution `scale`x over [-half_width, half_width)^2."""
    if scale < 1:
        raise ValueError("scale >= 1")
    w = float(half_width)
    return [(nx * scale, ny * scale, -w, w, -w, w) for nx, ny in CALOGAN_CELLS]
