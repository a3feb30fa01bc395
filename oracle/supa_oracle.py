"""ctypes wrapper of the FP64 C oracle, plus the oracle's image binning.

Test infrastructure only (tests, smoke check, CPU-baseline timing).

`simulate(geom, e0, polar, azimuth, seed, ...)` runs the propagation model of
the paper (section "Propagation Model", Algorithm 1) shower by shower in plain
C and returns every hit, every tree node, the per-shower energy ledger and
counts as numpy arrays.  `images(...)` bins hits into per-layer images the
plain way of the paper's appendix "Downsampling": a region of interest, a grid
of cells, and per cell the sum of the energies of the points inside it.
"""
from __future__ import annotations

import ctypes as C
import os
import threading
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from . import build_oracle

ANGLE_MODES = {"fixed": 0, "uniform": 1, "rayleigh": 2}
KINEMATICS = {"3d": 0, "literal": 1}
ERRORS = {1: "invalid argument", 2: "energy out of range", 6: "out of memory"}

_lib = None
_lock = threading.Lock()


class _Geometry(C.Structure):
    _fields_ = [
        ("n_planes", C.c_int32),
        ("z_first", C.c_double), ("dz", C.c_double),
        ("layer_of_plane", C.POINTER(C.c_int32)),
        ("p_stop", C.POINTER(C.c_double)),
        ("p_split", C.POINTER(C.c_double)),
        ("e_cut", C.c_double),
        ("angle_mode", C.c_int32),
        ("angle_a", C.c_double), ("angle_b", C.c_double),
        ("frac_lo", C.c_double), ("frac_hi", C.c_double),
        ("frac_bits", C.c_int32),
        ("kinematics", C.c_int32),
        ("n_regions", C.c_int32),
        ("region_r", C.POINTER(C.c_double)),
    ]


class _Result(C.Structure):
    _fields_ = [
        ("n_hits", C.c_int64), ("cap_hits", C.c_int64),
        ("hit_sid", C.POINTER(C.c_int32)), ("hit_plane", C.POINTER(C.c_int32)),
        ("hit_layer", C.POINTER(C.c_int32)), ("hit_kind", C.POINTER(C.c_int32)),
        ("hit_x", C.POINTER(C.c_double)), ("hit_y", C.POINTER(C.c_double)),
        ("hit_e", C.POINTER(C.c_uint32)), ("hit_key", C.POINTER(C.c_uint64)),
        ("n_nodes", C.c_int64), ("cap_nodes", C.c_int64),
        ("node_sid", C.POINTER(C.c_int32)), ("node_parent", C.POINTER(C.c_int32)),
        ("node_gen", C.POINTER(C.c_int32)),
        ("node_vx", C.POINTER(C.c_double)), ("node_vy", C.POINTER(C.c_double)),
        ("node_vz", C.POINTER(C.c_double)),
        ("node_e", C.POINTER(C.c_uint32)), ("node_key", C.POINTER(C.c_uint64)),
        ("n_showers", C.c_int64),
        ("ledger", C.POINTER(C.c_uint64)), ("counts", C.POINTER(C.c_int32)),
        ("peak_frontier", C.POINTER(C.c_int32)),
        ("region_margin", C.POINTER(C.c_double)),
    ]


def lib():
    """Load liboracle.so, building it from source if it is not there."""
    global _lib
    with _lock:
        if _lib is None:
            path = build_oracle.LIB
            if not os.path.exists(path):
                build_oracle.build()
            L = C.CDLL(path)
            L.oracle_simulate.restype = C.c_int
            L.oracle_simulate.argtypes = [
                C.POINTER(_Geometry), C.c_int64,
                C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                C.c_uint32, C.c_uint64, C.POINTER(_Result)]
            L.oracle_free.restype = None
            L.oracle_free.argtypes = [C.POINTER(_Result)]
            L.oracle_philox4x32_10.restype = None
            L.oracle_philox4x32_10.argtypes = [C.c_uint32] * 6 + [C.POINTER(C.c_uint32)]
            _lib = L
    return _lib


def philox4x32_10(key: int, ctr) -> tuple:
    """One Philox4x32-10 block for a 64-bit key and four 32-bit counter words."""
    out = (C.c_uint32 * 4)()
    lib().oracle_philox4x32_10(key & 0xFFFFFFFF, (key >> 32) & 0xFFFFFFFF,
                               *(int(c) & 0xFFFFFFFF for c in ctr), out)
    return tuple(int(v) for v in out)


def _f32(a, n):
    if a is None:
        return None
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    if a.shape != (n,):
        raise ValueError(f"expected shape ({n},), got {a.shape}")
    return a


def _copy(ptr, n, dtype):
    if n == 0:
        return np.zeros(0, dtype=dtype)
    return np.ctypeslib.as_array(ptr, shape=(n,)).astype(dtype, copy=True)


def simulate(geom: dict, e0, polar, azimuth, seed: int, x0=None, y0=None,
             shower_id_base: int = 0) -> dict:
    """Run the oracle on n showers; returns a dict of numpy arrays.

    geom keys: n_planes, z_first, dz, layer_of_plane (opt), p_stop (opt),
    p_split (opt), e_cut, angle_mode ('fixed'|'uniform'|'rayleigh'), angle_a,
    angle_b, frac_lo, frac_hi, frac_bits, kinematics ('3d' (default) |
    'literal'), n_regions (0/1: none; 2..4 lateral rings) with region_r
    (n_regions - 1 ascending radii), in which case p_stop / p_split have
    n_regions * n_planes entries, ring-major.
    """
    e0 = np.ascontiguousarray(np.asarray(e0, dtype=np.float32))
    n = e0.shape[0]
    polar, azimuth = _f32(polar, n), _f32(azimuth, n)
    x0, y0 = _f32(x0, n), _f32(y0, n)
    N = int(geom["n_planes"])
    keep = []

    R = int(geom.get("n_regions", 0) or 0)
    rings = R if R >= 2 else 1

    def arr(key, ctype, dtype, size=N):
        v = geom.get(key)
        if v is None:
            return None
        a = np.ascontiguousarray(np.asarray(v, dtype=dtype)).reshape(-1)
        if a.shape != (size,):
            raise ValueError(f"{key} must have {size} entries")
        keep.append(a)
        return a.ctypes.data_as(C.POINTER(ctype))

    g = _Geometry()
    g.n_planes = N
    g.z_first = float(geom.get("z_first", geom["dz"]))
    g.dz = float(geom["dz"])
    g.layer_of_plane = arr("layer_of_plane", C.c_int32, np.int32)
    g.p_stop = arr("p_stop", C.c_double, np.float64, rings * N)
    g.p_split = arr("p_split", C.c_double, np.float64, rings * N)
    g.n_regions = R
    g.region_r = arr("region_r", C.c_double, np.float64, max(R - 1, 0)) if R >= 2 else None
    g.e_cut = float(geom["e_cut"])
    g.angle_mode = ANGLE_MODES[geom["angle_mode"]]
    g.angle_a = float(geom.get("angle_a", 0.0))
    g.angle_b = float(geom.get("angle_b", 0.0))
    g.frac_lo = float(geom.get("frac_lo", 0.0))
    g.frac_hi = float(geom.get("frac_hi", 1.0))
    g.frac_bits = int(geom.get("frac_bits", 21))
    g.kinematics = KINEMATICS[geom.get("kinematics", "3d")]

    res = _Result()
    ptr = lambda a: None if a is None else a.ctypes.data
    status = lib().oracle_simulate(C.byref(g), n, ptr(e0), ptr(polar), ptr(azimuth),
                                   ptr(x0), ptr(y0), shower_id_base & 0xFFFFFFFF,
                                   seed & 0xFFFFFFFFFFFFFFFF, C.byref(res))
    try:
        if status != 0:
            raise ValueError(f"oracle error {status}: {ERRORS.get(status, '?')}")
        nh, nn = res.n_hits, res.n_nodes
        out = {
            "hit_sid": _copy(res.hit_sid, nh, np.int32).view(np.uint32).astype(np.int64),
            "hit_plane": _copy(res.hit_plane, nh, np.int32),
            "hit_layer": _copy(res.hit_layer, nh, np.int32),
            "hit_kind": _copy(res.hit_kind, nh, np.int32),
            "hit_x": _copy(res.hit_x, nh, np.float64),
            "hit_y": _copy(res.hit_y, nh, np.float64),
            "hit_e": _copy(res.hit_e, nh, np.uint32),
            "hit_key": _copy(res.hit_key, nh, np.uint64),
            "node_sid": _copy(res.node_sid, nn, np.int32).view(np.uint32).astype(np.int64),
            "node_parent": _copy(res.node_parent, nn, np.int32),
            "node_gen": _copy(res.node_gen, nn, np.int32),
            "node_vx": _copy(res.node_vx, nn, np.float64),
            "node_vy": _copy(res.node_vy, nn, np.float64),
            "node_vz": _copy(res.node_vz, nn, np.float64),
            "node_e": _copy(res.node_e, nn, np.uint32),
            "node_key": _copy(res.node_key, nn, np.uint64),
            "ledger": _copy(res.ledger, 4 * n, np.uint64).reshape(n, 4),
            "counts": _copy(res.counts, 6 * n, np.int32).reshape(n, 6),
            "peak_frontier": _copy(res.peak_frontier, n, np.int32),
            "region_margin": _copy(res.region_margin, n, np.float64),
        }
        out["frac_bits"] = g.frac_bits
        out["n"] = n
        out["shower_id_base"] = shower_id_base
        return out
    finally:
        lib().oracle_free(C.byref(res))


def simulate_parallel(geom: dict, e0, polar, azimuth, seed: int, threads: int,
                      chunk: int = 256, shower_id_base: int = 0) -> dict:
    """Same as `simulate`, split into chunks run on `threads` host threads.

    ctypes releases the interpreter lock for the duration of each C call, so
    the chunks run concurrently.  Used only to time the oracle; only the
    per-shower ledger and counts of the chunks are kept.
    """
    e0 = np.asarray(e0, dtype=np.float32)
    polar = np.asarray(polar, dtype=np.float32)
    azimuth = np.asarray(azimuth, dtype=np.float32)
    n = e0.shape[0]
    starts = list(range(0, n, chunk))

    def run(s):
        r = simulate(geom, e0[s:s + chunk], polar[s:s + chunk], azimuth[s:s + chunk],
                     seed, shower_id_base=shower_id_base + s)
        return s, r["ledger"], r["counts"], len(r["hit_e"])

    ledger = np.zeros((n, 4), np.uint64)
    counts = np.zeros((n, 6), np.int32)
    with ThreadPoolExecutor(max_workers=threads) as ex:
        for s, led, cnt, _ in ex.map(run, starts):
            ledger[s:s + len(led)] = led
            counts[s:s + len(cnt)] = cnt
    return {"ledger": ledger, "counts": counts}


def bin_index(v, lo: float, hi: float, nbins: int):
    """Cell index floor((v - lo) * nbins / (hi - lo)) in double; -1 when outside."""
    idx = np.floor((np.asarray(v, np.float64) - lo) * nbins / (hi - lo))
    ok = (idx >= 0) & (idx < nbins)
    return np.where(ok, idx, -1).astype(np.int64)


def images(res: dict, n_layers: int, nx: int, ny: int, x0: float, x1: float,
           y0: float, y1: float) -> np.ndarray:
    """Per shower, per layer image of summed fixed-point hit energies (uint64).

    Shape (n, n_layers, ny, nx).  A hit lands in cell (iy, ix) when both
    indices are inside the grid; cells are half-open [lo, hi).  Hits of planes
    that are not read out (layer -1) and hits outside the window are dropped.
    """
    n = res["n"]
    out = np.zeros((n, n_layers, ny, nx), dtype=np.uint64)
    ix = bin_index(res["hit_x"], x0, x1, nx)
    iy = bin_index(res["hit_y"], y0, y1, ny)
    layer = res["hit_layer"]
    ok = (ix >= 0) & (iy >= 0) & (layer >= 0) & (layer < n_layers)
    local = res["hit_sid"][ok].astype(np.int64) - res["shower_id_base"]
    np.add.at(out, (local, layer[ok], iy[ok], ix[ok]), res["hit_e"][ok].astype(np.uint64))
    return out


def grid_images(n: int, sid, layer, x, y, e_int, grids) -> np.ndarray:
    """Per shower, the concatenation over layers of [ny_l][nx_l] images of
    summed integer energies (uint64), each layer on its own grid
    grids[l] = (nx, ny, x0, x1, y0, y1) -- the appendix "Downsampling": a
    region of interest per layer and a number of cells in each direction.
    sid in [0, n); hits of layer -1 (or >= len(grids)) and hits outside their
    layer's region are dropped.  Shape (n, sum_l nx_l * ny_l)."""
    sid = np.asarray(sid, np.int64)
    layer = np.asarray(layer)
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    e_int = np.asarray(e_int, np.uint64)
    cells = [int(g[0]) * int(g[1]) for g in grids]
    off = np.concatenate([[0], np.cumsum(cells)]).astype(np.int64)
    out = np.zeros((n, int(off[-1])), dtype=np.uint64)
    for l, (nx, ny, x0, x1, y0, y1) in enumerate(grids):
        sel = layer == l
        ix = bin_index(x[sel], x0, x1, int(nx))
        iy = bin_index(y[sel], y0, y1, int(ny))
        ok = (ix >= 0) & (iy >= 0)
        np.add.at(out, (sid[sel][ok], off[l] + iy[ok] * int(nx) + ix[ok]), e_int[sel][ok])
    return out
