"""Shower shape variables and normalised Wasserstein-1 distances on the GPU.

Argument marshalling over the C ABI of include/supa_shapes.h: the variables,
statistics, histograms and distances are computed by the library's HIP
kernels; PyTorch only holds device memory.  Definitions: paper, section
"Shower Shape Variables" and appendix "More shower shape variables";
distance: section "Performance Analysis of Generative Models".
"""
from __future__ import annotations

import ctypes as C

import torch

from . import supa

LAYER_VARS = ("count", "mean_x", "mean_y", "mean_r", "mean_e", "std_x", "std_y", "std_r", "std_e",
              "energy", "centroid_x", "centroid_y", "centroid_r", "width_x", "width_y", "width_r",
              "fraction", "energy_ratio")
SHOWER_VARS = ("e_tot", "depth", "l_d", "s_d", "s_d_width")
DEFAULT_BINS = 100


def _lib():
    L = supa.load()
    if not hasattr(L, "_shapes_bound"):
        vp, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
        sig = {
            "supa_shower_shapes": (C.c_int, [vp, i64, i32, vp, vp, i32, i64, vp, vp, vp, vp, vp, vp, vp,
                                             i64]),
            "supa_shapes_work_ints": (i64, [i64]),
            "supa_hit_radius": (C.c_int, [vp, i64, vp, vp, vp]),
            "supa_w1_workspace_bytes": (sz, [i32, i32, i64, i64]),
            "supa_w1_normalized": (C.c_int, [vp, i32, vp, i64, i64, vp, i64, i64, i32, vp, i32, vp, vp,
                                             vp, sz]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        L.supa_shapes_last_error.restype = C.c_char_p
        L._shapes_bound = True
    return L


def _check(st):
    if st != 0:
        raise supa.SupaError(st, _lib().supa_shapes_last_error().decode())


def _p(t):
    return None if t is None else t.data_ptr()


def _stream():
    return torch.cuda.current_stream().cuda_stream


def shower_shapes(hit_offsets, hit_counts, hit_x, hit_y, hit_e, hit_layer, n_layers: int,
                  counts_stride: int = 1, check: bool = True):
    """Per-layer (float [n][n_layers][18]) and per-shower (float [n][5])
    shape variables of hits stored segment by segment.  hit_counts may be the
    simulator's counts array ([n][6], hits in column 1: pass counts[:, 1:] is
    not contiguous, so pass the flat array offset by one with counts_stride=6).
    check=True synchronises and raises if a shower broke the layer contiguity
    rule or carried a layer >= n_layers."""
    L = _lib()
    n = int(hit_offsets.numel())
    dev = hit_x.device
    lv = torch.empty((n, n_layers, len(LAYER_VARS)), dtype=torch.float32, device=dev)
    sv = torch.empty((n, len(SHOWER_VARS)), dtype=torch.float32, device=dev)
    work = torch.empty(int(L.supa_shapes_work_ints(n)), dtype=torch.int32, device=dev)
    if not all(t.is_contiguous() for t in (hit_x, hit_y, hit_e, hit_layer)):
        raise ValueError("hit arrays must be contiguous")
    hit_len = min(int(t.numel()) for t in (hit_x, hit_y, hit_e, hit_layer))
    _check(L.supa_shower_shapes(_stream(), n, n_layers, _p(hit_offsets), _p(hit_counts), counts_stride,
                                hit_len, _p(hit_x), _p(hit_y), _p(hit_e), _p(hit_layer), _p(lv),
                                _p(sv), _p(work), work.numel()))
    if check:
        bad = int(work[0].item())
        if bad:
            raise ValueError(f"{bad} showers have a layer split into several runs or a layer >= "
                             f"{n_layers}")
    return lv, sv


def simulator_shapes(out: dict, n_layers: int, check: bool = True):
    """Shape variables of a supa.Simulator output dict (hits requested)."""
    counts = out["counts"]
    return shower_shapes(out["hit_offsets"], counts.view(-1)[1:], out["hit_x"], out["hit_y"],
                         out["hit_e"], out["hit_layer"], n_layers, counts_stride=6, check=check)


def hit_radius(x, y):
    """r = sqrt(x^2 + y^2) of every point (float)."""
    r = torch.empty_like(x)
    _check(_lib().supa_hit_radius(_stream(), int(x.numel()), _p(x), _p(y), _p(r)))
    return r


class W1Workspace:
    """Device workspace of supa_w1_normalized, grown on demand."""

    def __init__(self, device="cuda"):
        self.device = torch.device(device)
        self.buf = torch.empty(0, dtype=torch.uint8, device=self.device)

    def get(self, n_cols, n_bins, n_ref, n_smp):
        need = int(_lib().supa_w1_workspace_bytes(n_cols, n_bins, n_ref, n_smp))
        if self.buf.numel() < need:
            self.buf = torch.empty(need, dtype=torch.uint8, device=self.device)
        return self.buf


def w1_columns(ref: torch.Tensor, smp: torch.Tensor, n_bins: int = DEFAULT_BINS, groups=None,
               n_groups: int = 0, workspace: W1Workspace | None = None):
    """Normalised W1 between the histograms of each column of ref and smp
    (float [rows][cols] with unit column stride; a 1-D tensor is one column).
    Returns (w1 double [cols], group means double [n_groups] or None)."""
    if ref.dim() == 1:
        ref, smp = ref.view(-1, 1), smp.view(-1, 1)
    if ref.stride(1) != 1 or smp.stride(1) != 1:
        raise ValueError("columns must have unit stride")
    n_cols = ref.shape[1]
    dev = ref.device
    ws = (workspace or W1Workspace(dev)).get(n_cols, n_bins, ref.shape[0], smp.shape[0])
    w1 = torch.empty(n_cols, dtype=torch.float64, device=dev)
    gm = None
    if groups is not None:
        gm = torch.empty(n_groups, dtype=torch.float64, device=dev)
    _check(_lib().supa_w1_normalized(_stream(), n_cols, _p(ref), ref.shape[0], ref.stride(0), _p(smp),
                                     smp.shape[0], smp.stride(0), n_bins, _p(groups), n_groups, _p(w1),
                                     _p(gm), _p(ws), ws.numel()))
    return w1, gm
