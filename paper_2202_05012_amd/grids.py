"""Per-layer grid images on the GPU (include/supa_grids.h): argument
marshalling only; the binning runs in the library's HIP kernel.  Definition:
paper, appendix "Downsampling"."""
from __future__ import annotations

import ctypes as C

import torch

from . import supa


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("x0", C.c_double), ("x1", C.c_double),
                ("y0", C.c_double), ("y1", C.c_double)]


def _lib():
    L = supa.load()
    if not hasattr(L, "_grids_bound"):
        vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        L.supa_grid_cells.restype = C.c_int64
        L.supa_grid_cells.argtypes = [vp, i32]
        L.supa_bin_grids.restype = C.c_int
        L.supa_bin_grids.argtypes = [vp, i64, i32, vp, i32, vp, vp, i32, i64, vp, vp, vp, vp, vp]
        L.supa_grids_last_error.restype = C.c_char_p
        L._grids_bound = True
    return L


def _grids(grids):
    arr = (Grid * len(grids))(*[Grid(int(g[0]), int(g[1]), *map(float, g[2:6])) for g in grids])
    return arr


def cells(grids) -> int:
    return int(_lib().supa_grid_cells(C.cast(_grids(grids), C.c_void_p), len(grids)))


def bin_grids(hit_offsets, hit_counts, hit_x, hit_y, hit_e, hit_layer, grids, frac_bits: int = 21,
              counts_stride: int = 1):
    """float [n][cells] images, layer l's [ny][nx] image after the earlier
    layers' cells; grids[l] = (nx, ny, x0, x1, y0, y1)."""
    L = _lib()
    g = _grids(grids)
    nc = int(L.supa_grid_cells(C.cast(g, C.c_void_p), len(grids)))
    n = int(hit_offsets.numel())
    out = torch.empty((n, max(nc, 0)), dtype=torch.float32, device=hit_x.device)
    hit_len = min(int(t.numel()) for t in (hit_x, hit_y, hit_e, hit_layer))
    p = lambda t: t.data_ptr()
    st = L.supa_bin_grids(torch.cuda.current_stream().cuda_stream, n, len(grids), C.cast(g, C.c_void_p),
                          frac_bits, p(hit_offsets), p(hit_counts), counts_stride, hit_len, p(hit_x),
                          p(hit_y), p(hit_e), p(hit_layer), p(out))
    if st != 0:
        raise supa.SupaError(st, L.supa_grids_last_error().decode())
    return out


def simulator_grids(out: dict, grids, frac_bits: int = 21):
    """Per-layer grid images of a supa.Simulator output dict (hits requested)."""
    return bin_grids(out["hit_offsets"], out["counts"].view(-1)[1:], out["hit_x"], out["hit_y"],
                     out["hit_e"], out["hit_layer"], grids, frac_bits, counts_stride=6)
