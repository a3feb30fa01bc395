"""Learned surrogate: conditional MLP trained on simulated showers, with an
uncertainty gate that sends doubtful showers back to the simulator.

Argument marshalling over the C ABI of include/supa_surrogate.h: every
product, activation, loss, gradient, optimiser step, noise draw, gate and
compaction runs in the library's HIP kernels; PyTorch only holds device memory.

Model (the reading of the extension, not part of the paper): inputs
(E0 / 100, polar / 15 deg, azimuth / 2 pi) and 16 standard normals, four
hidden layers of 256 with GELU, output 2 * D with D = 20 layers x 16 x 16:
mean and log-variance of the per-bin deposit fraction y = image / E0.
Trained with the Gaussian negative log-likelihood and Adam.
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np
import torch

from . import supa

IN_FEATURES = 3
N_NOISE = 16
IN_PAD = 32                 # input row length (multiple of 32 for the matrix cores)
S_CLAMP = 20.0
Y_SCALE = 1000.0            # targets are 1000 * image / E0: per-bin values of order 1


def _lib():
    L = supa.load()
    if not hasattr(L, "_surrogate_bound"):
        vp, i, i64, f, u32, u64 = C.c_void_p, C.c_int, C.c_int64, C.c_float, C.c_uint32, C.c_uint64
        sig = {
            "supa_gemm_bf16": [vp, i, i, i, i, i, i, vp, i, vp, i, vp, vp, i, vp],
            "supa_nll_grad": [vp, i, i, vp, vp, vp, f, f, i, vp, vp],
            "supa_colsum_bf16": [vp, i, i, vp, i, vp, vp],
            "supa_adam": [vp, i64, vp, vp, vp, vp, vp, f, f, f, f, i],
            "supa_to_bf16": [vp, i64, vp, vp],
            "supa_surrogate_features": [vp, i, i, i, vp, vp, vp, f, f, f, u32, u32, u64, vp],
            "supa_surrogate_gate": [vp, i, i, i, vp, vp, f, f, vp, vp, vp, f, u32, u64],
            "supa_select_above": [vp, i, vp, f, vp, vp, vp],
            "supa_gather3": [vp, i, vp, vp, vp, vp, vp, vp, vp],
            "supa_scatter_rows": [vp, i, i, vp, vp, vp],
            "supa_group_sums": [vp, i, i, i, vp, vp],
            "supa_surrogate_gate_fused": [vp, i, i, i, i, vp, i, vp, i, vp, vp, f, f, vp, vp, vp, f, u32,
                                          u64, f, vp],
            "supa_transpose_to_bf16": [vp, i, i, vp, vp],
            "supa_gemm_bf16_splitk": [vp, i, i, i, i, i, vp, i, vp, i, vp, i, vp],
            "supa_gemm_splitk_parts": [i, i, i],
            "supa_w1_equal": [vp, i64, C.c_int32, vp, i64, vp, i64, vp, vp, i64],
            "supa_sort_columns": [vp, i64, C.c_int32, vp, i64, vp, vp, i64],
            "supa_occupied_counts": [vp, i64, C.c_int32, C.c_int32, vp, f, vp],
            "supa_surrogate_timing": [i],
            "supa_mlp_forward_fused": [vp, i, i, i, vp, i, vp, vp, i, vp, i, vp, i],
            "supa_mlp_fused_weights": [vp, i, i, vp, i, vp],
            "supa_surrogate_last_times": [vp, C.c_int32],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.restype = C.c_int
            fn.argtypes = args
        for name in ("supa_w1_equal_workspace_bytes", "supa_sort_columns_workspace_bytes"):
            fn = getattr(L, name)
            fn.restype = C.c_int64
            fn.argtypes = [i64, C.c_int32]
        L.supa_surrogate_last_error.restype = C.c_char_p
        L._surrogate_bound = True
    return L


def _check(st):
    if st != 0:
        raise supa.SupaError(st, _lib().supa_surrogate_last_error().decode())


def _p(t):
    return None if t is None else t.data_ptr()


def _stream():
    return torch.cuda.current_stream().cuda_stream


# ---------------------------------------------------------------------------
# thin wrappers, one per entry point
# ---------------------------------------------------------------------------
def gemm(A, B, C_out, trans_a=0, trans_b=0, epilogue=0, bias=None, pre=None, M=None, N=None,
         K=None):
    """C = op(A) op(B) on bf16 (int16-typed) tensors; see supa_surrogate.h."""
    M = M if M is not None else (A.shape[1] if trans_a else A.shape[0])
    K = K if K is not None else (A.shape[0] if trans_a else A.shape[1])
    N = N if N is not None else (B.shape[0] if trans_b else B.shape[1])
    _check(_lib().supa_gemm_bf16(_stream(), trans_a, trans_b, epilogue, M, N, K, _p(A), A.stride(0),
                                 _p(B), B.stride(0), _p(bias), _p(C_out), C_out.stride(0), _p(pre)))


def gemm_splitk(A, B, C_out, trans_a=0, trans_b=0):
    """C = op(A) op(B) (float32 C, contiguous) with K split over workgroups."""
    M = A.shape[1] if trans_a else A.shape[0]
    K = A.shape[0] if trans_a else A.shape[1]
    N = B.shape[0] if trans_b else B.shape[1]
    L = _lib()
    L.supa_gemm_splitk_parts.restype = C.c_int32
    parts = int(L.supa_gemm_splitk_parts(M, N, K))
    scratch = torch.empty(parts * M * N if parts > 1 else 1, dtype=torch.float32, device=C_out.device)
    _check(L.supa_gemm_bf16_splitk(_stream(), trans_a, trans_b, M, N, K, _p(A), A.stride(0), _p(B),
                                   B.stride(0), _p(C_out), parts, _p(scratch)))


def to_bf16(x: torch.Tensor) -> torch.Tensor:
    """float32 tensor -> bf16 bit patterns (int16 tensor) via the library."""
    x = x.contiguous()
    y = torch.empty(x.shape, dtype=torch.int16, device=x.device)
    _check(_lib().supa_to_bf16(_stream(), x.numel(), _p(x), _p(y)))
    return y


def bf16_to_float(y: torch.Tensor) -> torch.Tensor:
    """bf16 bit patterns -> float32 values (exact; a reinterpretation)."""
    return (y.to(torch.int32) << 16).view(torch.float32)


def features(e0, polar, az, seed, row_base=0, stream_id=0):
    B = int(e0.shape[0])
    x = torch.empty((B, IN_PAD), dtype=torch.int16, device=e0.device)
    _check(_lib().supa_surrogate_features(_stream(), B, IN_PAD, N_NOISE, _p(e0), _p(polar), _p(az),
                                          1.0 / 100.0, 1.0 / math.radians(15.0), 1.0 / (2 * math.pi),
                                          row_base & 0xFFFFFFFF, stream_id & 0xFFFFFFFF,
                                          seed & 0xFFFFFFFFFFFFFFFF, _p(x)))
    return x


def gate(out, e0, n_layers, want_image=False, rho=-1.0, seed=0, row_base=0, y_scale=None):
    """Per-layer energies (means, or samples when rho >= 0), uncertainty
    scores and optionally the predicted images; see supa_surrogate.h."""
    B, D2 = out.shape
    D = D2 // 2
    layer_e = torch.empty((B, n_layers), dtype=torch.float32, device=out.device)
    unc = torch.empty(B, dtype=torch.float32, device=out.device)
    img = torch.empty((B, D), dtype=torch.float32, device=out.device) if want_image else None
    ys = Y_SCALE if y_scale is None else y_scale
    _check(_lib().supa_surrogate_gate(_stream(), B, D, n_layers, _p(out), _p(e0), ys, S_CLAMP,
                                      _p(layer_e), _p(unc), _p(img), float(rho),
                                      row_base & 0xFFFFFFFF, seed & 0xFFFFFFFFFFFFFFFF))
    return layer_e, unc, img


def transpose_to_bf16(x: torch.Tensor) -> torch.Tensor:
    """float32 [r, c] -> bf16 bit patterns of its transpose [c, r] (library kernel)."""
    x = x.contiguous()
    r, c = x.shape
    y = torch.empty((c, r), dtype=torch.int16, device=x.device)
    _check(_lib().supa_transpose_to_bf16(_stream(), r, c, _p(x), _p(y)))
    return y


def gate_fused(h, w_t, bias, e0, n_layers, rho=-1.0, seed=0, row_base=0, cnt_thr=None):
    """Final layer + gate in one pass (supa_surrogate_gate_fused): h bf16 [B, K]
    last hidden activations, w_t bf16 [2D, K] the final weights transposed.
    With cnt_thr, also the per-layer counts of bins predicted above it."""
    B, K = h.shape
    D = w_t.shape[0] // 2
    layer_e = torch.empty((B, n_layers), dtype=torch.float32, device=h.device)
    unc = torch.empty(B, dtype=torch.float32, device=h.device)
    cnt = torch.empty((B, n_layers), dtype=torch.float32, device=h.device) if cnt_thr is not None else None
    partial = torch.empty((max(B, 1), (2 * D) // 128, 2), dtype=torch.float32, device=h.device)
    _check(_lib().supa_surrogate_gate_fused(_stream(), B, K, D, n_layers, _p(h), h.stride(0), _p(w_t),
                                            w_t.stride(0), _p(bias), _p(e0), Y_SCALE, S_CLAMP, _p(partial),
                                            _p(layer_e), _p(unc), float(rho), row_base & 0xFFFFFFFF,
                                            seed & 0xFFFFFFFFFFFFFFFF, float(cnt_thr or 0.0), _p(cnt)))
    return (layer_e, unc) if cnt is None else (layer_e, unc, cnt)


def timing(on: bool):
    """Switch the event timing of gate_fused on or off (supa_surrogate_timing)."""
    _check(_lib().supa_surrogate_timing(1 if on else 0))


def last_times():
    """Milliseconds of the last timed gate_fused call: (mean-tile product,
    log-variance product, per-row gate)."""
    ms = (C.c_float * 3)()
    _check(_lib().supa_surrogate_last_times(C.cast(ms, C.c_void_p), 3))
    return tuple(float(v) for v in ms)


def w1_equal(a, b):
    """Exact W1 between the columns of two equal-size float samples [n, cols]
    (supa_w1_equal); returns a float64 tensor [cols] on the device."""
    a, b = a.contiguous(), b.contiguous()
    n, cols = a.shape
    if b.shape != a.shape:
        raise ValueError("samples of equal shape")
    L = _lib()
    wb = int(L.supa_w1_equal_workspace_bytes(n, cols))
    work = torch.empty(max(wb, 1), dtype=torch.uint8, device=a.device)
    w1 = torch.empty(cols, dtype=torch.float64, device=a.device)
    _check(L.supa_w1_equal(_stream(), n, cols, _p(a), a.stride(0), _p(b), b.stride(0), _p(w1), _p(work), wb))
    return w1


def sort_columns(x):
    """Columns of a float [n, cols] tensor sorted (supa_sort_columns): [cols, n]."""
    x = x.contiguous()
    n, cols = x.shape
    L = _lib()
    wb = int(L.supa_sort_columns_workspace_bytes(n, cols))
    work = torch.empty(max(wb, 1), dtype=torch.uint8, device=x.device)
    out = torch.empty((cols, n), dtype=torch.float32, device=x.device)
    _check(L.supa_sort_columns(_stream(), n, cols, _p(x), x.stride(0), _p(out), _p(work), wb))
    return out


def occupied_counts(img, n_layers, thr):
    """Per row and layer, the cells of a flattened [rows, L * g] image above thr."""
    rows, width = img.shape
    cnt = torch.empty((rows, n_layers), dtype=torch.float32, device=img.device)
    _check(_lib().supa_occupied_counts(_stream(), rows, n_layers, width // n_layers, _p(img.contiguous()),
                                       float(thr), _p(cnt)))
    return cnt


def select_above(v, tau):
    n = int(v.shape[0])
    idx = torch.empty(max(n, 1), dtype=torch.int32, device=v.device)
    count = torch.zeros(1, dtype=torch.int32, device=v.device)
    scratch = torch.empty(max(1, (n + 1023) // 1024), dtype=torch.int32, device=v.device)
    _check(_lib().supa_select_above(_stream(), n, _p(v), float(tau), _p(idx), _p(count),
                                    _p(scratch)))
    m = int(count.item())
    return idx[:m]


def gather3(idx, a, b, c):
    m = int(idx.shape[0])
    oa, ob, oc = (torch.empty(m, dtype=torch.float32, device=a.device) for _ in range(3))
    _check(_lib().supa_gather3(_stream(), m, _p(idx), _p(a), _p(b), _p(c), _p(oa), _p(ob), _p(oc)))
    return oa, ob, oc


def scatter_rows(idx, src, dst):
    m, w = src.shape
    _check(_lib().supa_scatter_rows(_stream(), m, w, _p(idx), _p(src), _p(dst)))


def group_sums(x, n_groups):
    rows, width = x.shape
    out = torch.empty((rows, n_groups), dtype=torch.float32, device=x.device)
    _check(_lib().supa_group_sums(_stream(), rows, n_groups, width // n_groups, _p(x), _p(out)))
    return out


# ---------------------------------------------------------------------------
# the MLP
# ---------------------------------------------------------------------------
def _colsum_scratch(M, N, device):
    L = _lib()
    L.supa_colsum_scratch_floats.restype = C.c_int64
    L.supa_colsum_scratch_floats.argtypes = [C.c_int, C.c_int]
    return torch.empty(max(1, L.supa_colsum_scratch_floats(M, N)), dtype=torch.float32, device=device)


class MLP:
    """bf16 weights with float32 master copies and Adam moments, on device."""

    def __init__(self, dims, device="cuda", seed=0):
        self.dims = list(dims)            # [IN_PAD, h, ..., out]
        self.device = torch.device(device)
        rng = np.random.default_rng(seed)
        self.W, self.b = [], []
        for l, (din, dout) in enumerate(zip(self.dims[:-1], self.dims[1:])):
            fan_in = din if l > 0 else IN_FEATURES + N_NOISE
            w = rng.normal(0.0, math.sqrt(2.0 / fan_in), size=(din, dout)).astype(np.float32)
            if l == 0:
                w[IN_FEATURES + N_NOISE:] = 0.0       # padding inputs
            if l == len(self.dims) - 2:
                w *= 0.1                              # start near mu = 0, log var = 0
            self.W.append(torch.from_numpy(w).to(self.device))
            self.b.append(torch.zeros(dout, dtype=torch.float32, device=self.device))
        self.Wb = [to_bf16(w) for w in self.W]
        self.mW = [torch.zeros_like(w) for w in self.W]
        self.vW = [torch.zeros_like(w) for w in self.W]
        self.mb = [torch.zeros_like(b) for b in self.b]
        self.vb = [torch.zeros_like(b) for b in self.b]
        self.step = 0

    def load_float_weights(self, Ws, bs):
        for l, (w, b) in enumerate(zip(Ws, bs)):
            self.W[l].copy_(torch.as_tensor(w, dtype=torch.float32))
            self.b[l].copy_(torch.as_tensor(b, dtype=torch.float32))
            self.Wb[l] = to_bf16(self.W[l])
        self._wt_step = None

    def forward(self, x, keep=False):
        """x: bf16 [B, IN_PAD] -> float32 [B, out]; keep=True also returns
        the activations and pre-activations the backward needs (without it
        the pre-activations are not stored)."""
        B = x.shape[0]
        h = x
        acts, pres = [x], []
        nl = len(self.Wb)
        for l in range(nl):
            dout = self.dims[l + 1]
            if l < nl - 1:
                y = torch.empty((B, dout), dtype=torch.int16, device=self.device)
                pre = torch.empty((B, dout), dtype=torch.int16, device=self.device) if keep else None
                gemm(h, self.Wb[l], y, epilogue=2, bias=self.b[l], pre=pre)
                pres.append(pre)
                acts.append(y)
                h = y
            else:
                out = torch.empty((B, dout), dtype=torch.float32, device=self.device)
                gemm(h, self.Wb[l], out, epilogue=1, bias=self.b[l])
        return (out, acts, pres) if keep else out

    def hidden(self, x):
        """x: bf16 [B, IN_PAD] -> the last hidden activations, bf16 [B, hidden]."""
        h = x
        for l in range(len(self.Wb) - 1):
            y = torch.empty((x.shape[0], self.dims[l + 1]), dtype=torch.int16, device=self.device)
            gemm(h, self.Wb[l], y, epilogue=2, bias=self.b[l])
            h = y
        return h

    def fused_ok(self):
        """True when the fused forward pass takes this network: hidden layers
        of 256 (1..8), inputs a multiple of 16 up to 256."""
        hid = self.dims[1:-1]
        return (1 <= len(hid) <= 8 and all(d == 256 for d in hid) and self.dims[0] % 16 == 0
                and self.dims[0] <= 256)

    def fused_weights(self):
        """The layers' weights for the fused forward pass (transposed, inputs of
        layers after the first permuted), cached per optimiser step."""
        if getattr(self, "_fw_step", None) != self.step:
            ws = []
            for l, W in enumerate(self.W):
                din, dout = W.shape
                wt = torch.empty((dout, din), dtype=torch.int16, device=self.device)
                _check(_lib().supa_mlp_fused_weights(_stream(), din, dout, _p(W), 1 if l > 0 else 0, _p(wt)))
                ws.append(wt)
            self._fw, self._fw_step = ws, self.step
        return self._fw

    def _fused(self, x, n_hidden, n_out, out, h):
        ws = self.fused_weights()
        layers = n_hidden + (1 if n_out else 0)
        wt = (C.c_void_p * layers)(*[w.data_ptr() for w in ws[:layers]])
        bs = (C.c_void_p * layers)(*[b.data_ptr() for b in self.b[:layers]])
        _check(_lib().supa_mlp_forward_fused(_stream(), x.shape[0], self.dims[0], n_hidden, _p(x), x.stride(0),
                                             C.cast(wt, C.c_void_p), C.cast(bs, C.c_void_p), n_out, _p(out),
                                             out.stride(0) if out is not None else 0, _p(h),
                                             h.stride(0) if h is not None else 0))

    def forward_fused(self, x):
        """The whole forward pass in one kernel (supa_mlp_forward_fused; the
        output layer at most 64 wide): x bf16 [B, in] -> float32 [B, out]."""
        n_out = self.dims[-1]
        out = torch.empty((x.shape[0], n_out), dtype=torch.float32, device=self.device)
        self._fused(x, len(self.dims) - 2, n_out, out, None)
        return out

    def hidden_fused(self, x):
        """The hidden layers in one kernel: x bf16 [B, in] -> the last hidden
        activations, bf16 [B, 256]."""
        h = torch.empty((x.shape[0], 256), dtype=torch.int16, device=self.device)
        self._fused(x, len(self.dims) - 2, 0, None, h)
        return h

    def final_weights_t(self):
        """bf16 transpose of the final layer's weights (cached per optimiser step)."""
        if getattr(self, "_wt_step", None) != self.step:
            self._wt = transpose_to_bf16(self.W[-1])
            self._wt_step = self.step
        return self._wt

    def layer_energies(self, x, e0, n_layers, rho=-1.0, seed=0, row_base=0, cnt_thr=None):
        """Per-layer energies and uncertainty scores of the inputs x (and, with
        cnt_thr, per-layer counts of bins predicted above it), with the final
        layer fused into the gate (no [B, 2D] output)."""
        h = self.hidden_fused(x) if self.fused_ok() else self.hidden(x)
        return gate_fused(h, self.final_weights_t(), self.b[-1], e0, n_layers, rho=rho,
                          seed=seed, row_base=row_base, cnt_thr=cnt_thr)

    def backward(self, acts, pres, dout):
        """dout: bf16 [B, out] = d loss / d out; returns float32 (dW, db) lists."""
        B = dout.shape[0]
        nl = len(self.Wb)
        dWs, dbs = [None] * nl, [None] * nl
        g = dout
        for l in range(nl - 1, -1, -1):
            din, dout_l = self.dims[l], self.dims[l + 1]
            dW = torch.empty((din, dout_l), dtype=torch.float32, device=self.device)
            gemm_splitk(acts[l], g, dW, trans_a=1, trans_b=0)              # h^T g
            db = torch.empty(dout_l, dtype=torch.float32, device=self.device)
            _check(_lib().supa_colsum_bf16(_stream(), B, dout_l, _p(g), g.stride(0), _p(db),
                                           _p(_colsum_scratch(B, dout_l, self.device))))
            dWs[l], dbs[l] = dW, db
            if l > 0:
                gn = torch.empty((B, din), dtype=torch.int16, device=self.device)
                gemm(g, self.Wb[l], gn, trans_a=0, trans_b=1, epilogue=3, pre=pres[l - 1])
                g = gn
        return dWs, dbs

    def adam(self, dWs, dbs, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.step += 1
        L = _lib()
        for l in range(len(self.W)):
            _check(L.supa_adam(_stream(), self.W[l].numel(), _p(self.W[l]), _p(dWs[l]),
                               _p(self.mW[l]), _p(self.vW[l]), _p(self.Wb[l]), lr, b1, b2, eps,
                               self.step))
            _check(L.supa_adam(_stream(), self.b[l].numel(), _p(self.b[l]), _p(dbs[l]),
                               _p(self.mb[l]), _p(self.vb[l]), None, lr, b1, b2, eps, self.step))

    def train_step(self, x, img, e0, lr=1e-3, s_clamp=None, mse_mean=True, y_scale=None):
        """One step on targets y_scale * img / e0 (img float [B, D]; default
        scale Y_SCALE); returns the mean NLL.  Means are fitted by squared
        error (mse_mean) or by the NLL, log-variances by the NLL; s_clamp = 0
        holds the log-variances at 0."""
        out, acts, pres = self.forward(x, keep=True)
        B, D2 = out.shape
        dout = torch.empty((B, D2), dtype=torch.int16, device=self.device)
        loss = torch.zeros(1, dtype=torch.float32, device=self.device)
        sc = S_CLAMP if s_clamp is None else s_clamp
        ys = Y_SCALE if y_scale is None else y_scale
        _check(_lib().supa_nll_grad(_stream(), B, D2 // 2, _p(out), _p(img), _p(e0), ys,
                                    sc, 1 if mse_mean else 0, _p(dout), _p(loss)))
        dWs, dbs = self.backward(acts, pres, dout)
        self.adam(dWs, dbs, lr=lr)
        return loss / (B * (D2 // 2))


def surrogate_dims(n_layers=20, bins=256, hidden=256, depth=4):
    return [IN_PAD] + [hidden] * depth + [2 * n_layers * bins]
