"""Seeded synthetic workloads: initial conditions and process parameters.

This module only draws inputs.  It holds none of the simulation's arithmetic,
so the HIP path and the CPU oracle can both be fed from it.

Initial conditions are the paper's conditioning variables (section "Using
SUPA", "Extensions": initial energy, impact angle, impact position) drawn
from a numpy generator seeded by the workload seed and cast to float32, so
every consumer receives bit-identical arrays.  Angles are in radians; the
polar angle is measured from the +z axis (0 = normal incidence).

Process parameters: p_split = 1 and p_stop = 0 on every plane, so particles
split at every plane until they fall below the energy threshold e_cut = 0.1,
energy fraction f ~ U(0, 1), opening angle theta ~ Rayleigh(sigma = 0.1 rad),
planes at z = 1, 2, ..., N (slice gap 1).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    n: int                      # showers
    n_planes: int
    e0: tuple                   # ("fixed", v) | ("uniform", a, b) | ("loguniform", a, b)
    polar_deg: tuple            # ("fixed", v) | ("uniform", a, b)
    azimuth: tuple              # ("fixed", v) | ("uniform", 0, 2pi)
    seed: int
    images: tuple | None        # (nx, ny, x0, x1, y0, y1) or None
    tree: bool = False
    description: str = ""


TWO_PI = 2.0 * math.pi

WORKLOADS = {
    w.name: w for w in [
        Workload("e10_normal_5planes_1k", 1000, 5, ("fixed", 10.0), ("fixed", 0.0),
                 ("fixed", 0.0), 0, None,
                 description="1,000 showers, E0 = 10, normal incidence at the origin, "
                             "5 planes, hit clouds only, seed 0"),
        Workload("e1to100_20planes_img32_100k", 100_000, 20, ("uniform", 1.0, 100.0),
                 ("uniform", 0.0, 15.0), ("uniform", 0.0, TWO_PI), 1,
                 (32, 32, -5.0, 5.0, -5.0, 5.0),
                 description="100,000 showers, E0 ~ U[1,100], polar ~ U[0,15 deg], "
                             "azimuth ~ U[0,2pi), 20 planes, hit clouds + 20 x 32x32 "
                             "images over [-5,5)^2, seed 1"),
        Workload("loge1to1000_20planes_1m", 1_000_000, 20, ("loguniform", 1.0, 1000.0),
                 ("uniform", 0.0, 15.0), ("uniform", 0.0, TWO_PI), 1, None,
                 description="1,000,000 showers, E0 log-uniform on [1,1000], same angles, "
                             "20 planes, hit clouds + counts, persistent work queue"),
        Workload("loge10to1000_50planes_tree_img256_1m", 1_000_000, 50,
                 ("loguniform", 10.0, 1000.0), ("uniform", 0.0, 15.0),
                 ("uniform", 0.0, TWO_PI), 1, (256, 256, -5.0, 5.0, -5.0, 5.0), tree=True,
                 description="1,000,000 showers, E0 log-uniform on [10,1000], 50 planes, "
                             "propagation tree + 50 x 256x256 images"),
        Workload("e1000_20planes_tree_256", 256, 20, ("fixed", 1000.0), ("uniform", 0.0, 15.0),
                 ("uniform", 0.0, TWO_PI), 2, None, tree=True,
                 description="256 showers of E0 = 1000 (the top of the log-uniform range), same "
                             "angles, 20 planes, hit clouds + propagation tree: a small call "
                             "whose showers occupy 64 of the GPU's waves unless they are split"),
    ]
}


def geometry(w: Workload, **overrides) -> dict:
    """Process parameters of a workload as a plain dict (both sides read it)."""
    g = {
        "n_planes": w.n_planes,
        "z_first": 1.0,
        "dz": 1.0,
        "layer_of_plane": None,
        "p_stop": None,
        "p_split": None,
        "e_cut": 0.1,
        "angle_mode": "rayleigh",
        "angle_a": 0.1,
        "angle_b": 0.0,
        "frac_lo": 0.0,
        "frac_hi": 1.0,
        "frac_bits": 21,
    }
    if w.images is not None:
        nx, ny, x0, x1, y0, y1 = w.images
        g.update(img_nx=nx, img_ny=ny, img_x0=x0, img_x1=x1, img_y0=y0, img_y1=y1)
    g.update(overrides)
    return g


def _draw(rng: np.random.Generator, spec: tuple, n: int) -> np.ndarray:
    kind = spec[0]
    if kind == "fixed":
        return np.full(n, spec[1], dtype=np.float64)
    if kind == "uniform":
        return rng.uniform(spec[1], spec[2], size=n)
    if kind == "loguniform":
        return np.exp(rng.uniform(math.log(spec[1]), math.log(spec[2]), size=n))
    raise ValueError(f"unknown distribution {spec}")


def initial_conditions(w: Workload, n: int | None = None, seed: int | None = None):
    """(e0, polar, azimuth) float32 arrays of the first n showers of a workload.

    The arrays of a smaller n are prefixes of those of a larger n, so a shower
    id always maps to the same initial condition.
    """
    n = w.n if n is None else n
    rng = np.random.Generator(np.random.PCG64(w.seed if seed is None else seed))
    # one stream per variable so prefixes are stable across n
    r_e, r_p, r_a = rng.spawn(3)
    e0 = _draw(r_e, w.e0, n).astype(np.float32)
    polar = np.deg2rad(_draw(r_p, w.polar_deg, n)).astype(np.float32)
    az = _draw(r_a, w.azimuth, n).astype(np.float32)
    return e0, polar, az
