"""Python binding of libsupa.so (C ABI in include/supa.h).

Argument marshalling only: PyTorch supplies device memory and the stream,
every step of the simulation runs in the library's HIP kernels.  There is no
CPU fallback: if the library is missing or no GPU is present, calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsupa.so")

ANGLE_MODES = {"fixed": 0, "uniform": 1, "rayleigh": 2}
KINEMATICS = {"3d": 0, "literal": 1}
OUT_HITS, OUT_IMAGES, OUT_TREE, OUT_KEYS = 1, 2, 4, 8
STATUS = {0: "OK", 1: "INVALID_ARG", 2: "RANGE", 3: "CAPACITY", 4: "DEVICE", 5: "STATE",
          6: "NOMEM"}


class SupaError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Geometry(C.Structure):
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
        ("energy_frac_bits", C.c_int32),
        ("img_nx", C.c_int32), ("img_ny", C.c_int32),
        ("img_x0", C.c_double), ("img_x1", C.c_double),
        ("img_y0", C.c_double), ("img_y1", C.c_double),
        ("outputs", C.c_uint32),
        ("kinematics", C.c_int32),
        ("n_regions", C.c_int32),
        ("region_r", C.POINTER(C.c_double)),
    ]


class Batch(C.Structure):
    _fields_ = [
        ("e0", C.c_void_p), ("polar", C.c_void_p), ("azimuth", C.c_void_p),
        ("x0", C.c_void_p), ("y0", C.c_void_p),
        ("n", C.c_int64), ("shower_id_base", C.c_uint32),
    ]


class Output(C.Structure):
    _fields_ = [
        ("hit_offsets", C.c_void_p),
        ("hit_x", C.c_void_p), ("hit_y", C.c_void_p), ("hit_e", C.c_void_p),
        ("hit_layer", C.c_void_p), ("hit_key", C.c_void_p), ("hit_capacity", C.c_int64),
        ("images", C.c_void_p),
        ("node_offsets", C.c_void_p),
        ("node_parent", C.c_void_p), ("node_gen", C.c_void_p),
        ("node_vx", C.c_void_p), ("node_vy", C.c_void_p), ("node_vz", C.c_void_p),
        ("node_e", C.c_void_p), ("node_key", C.c_void_p), ("node_capacity", C.c_int64),
        ("ledger", C.c_void_p), ("counts", C.c_void_p), ("shower_capacity", C.c_int64),
        ("total_hits", C.c_int64), ("total_nodes", C.c_int64), ("total_steps", C.c_int64),
    ]


EXPORTS = ["supa_abi_version", "supa_validate_geometry", "supa_validate_call", "supa_init_geometry", "supa_destroy",
           "supa_simulate", "supa_simulate_batches", "supa_simulate_noalloc", "supa_set_launch", "supa_set_schedule", "supa_set_subtrees", "supa_last_subtrees", "supa_autotune", "supa_autotune_forget",
           "supa_graph_create", "supa_graph_launch", "supa_graph_check", "supa_graph_destroy", "supa_last_timing", "supa_last_kernel_times", "supa_last_wave_times", "supa_philox", "supa_azimuth",
           "supa_last_error"]

_lib = None


def load():
    """Load libsupa.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it first (python -m "
                               "paper_2202_05012_amd.build)")
        L = C.CDLL(LIB_PATH)
        L.supa_abi_version.restype = C.c_int32
        L.supa_validate_geometry.restype = C.c_int
        L.supa_validate_geometry.argtypes = [C.POINTER(Geometry)]
        L.supa_validate_call.restype = C.c_int
        L.supa_validate_call.argtypes = [C.POINTER(Geometry), C.POINTER(Batch), C.POINTER(Output)]
        L.supa_init_geometry.restype = C.c_int
        L.supa_init_geometry.argtypes = [C.POINTER(Geometry), C.c_int, C.c_void_p,
                                         C.POINTER(C.c_void_p)]
        L.supa_destroy.restype = C.c_int
        L.supa_destroy.argtypes = [C.c_void_p]
        L.supa_simulate.restype = C.c_int
        L.supa_simulate.argtypes = [C.c_void_p, C.POINTER(Batch), C.c_uint64, C.POINTER(Output)]
        L.supa_simulate_batches.restype = C.c_int
        L.supa_simulate_batches.argtypes = [C.c_void_p, C.c_int32, C.POINTER(Batch), C.c_uint64,
                                            C.POINTER(Output)]
        L.supa_simulate_noalloc.restype = C.c_int
        L.supa_simulate_noalloc.argtypes = [C.c_void_p, C.POINTER(Batch), C.c_uint64, C.POINTER(Output)]
        L.supa_set_launch.restype = C.c_int
        L.supa_set_launch.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32]
        L.supa_autotune.restype = C.c_int
        L.supa_autotune.argtypes = [C.c_void_p, C.POINTER(Batch), C.c_uint64, C.POINTER(Output),
                                    C.POINTER(C.c_int32), C.POINTER(C.c_float)]
        L.supa_autotune_forget.restype = C.c_int
        L.supa_autotune_forget.argtypes = [C.c_void_p]
        L.supa_graph_create.restype = C.c_int
        L.supa_graph_create.argtypes = [C.c_void_p, C.POINTER(Batch), C.c_uint64, C.POINTER(Output),
                                        C.POINTER(C.c_void_p)]
        L.supa_graph_launch.restype = C.c_int
        L.supa_graph_launch.argtypes = [C.c_void_p, C.c_void_p]
        L.supa_graph_check.restype = C.c_int
        L.supa_graph_check.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(C.c_int64)]
        L.supa_graph_destroy.restype = C.c_int
        L.supa_graph_destroy.argtypes = [C.c_void_p]
        L.supa_set_schedule.restype = C.c_int
        L.supa_set_schedule.argtypes = [C.c_void_p, C.c_int32, C.c_int32]
        L.supa_set_subtrees.restype = C.c_int
        L.supa_set_subtrees.argtypes = [C.c_void_p, C.c_int32, C.c_int32]
        L.supa_last_subtrees.restype = C.c_int
        L.supa_last_subtrees.argtypes = [C.c_void_p, C.POINTER(C.c_int64)]
        L.supa_last_timing.restype = C.c_int
        L.supa_last_timing.argtypes = [C.c_void_p, C.POINTER(C.c_float)]
        L.supa_last_wave_times.restype = C.c_int
        L.supa_last_wave_times.argtypes = [C.c_void_p, C.POINTER(C.c_float), C.c_int32, C.POINTER(C.c_int32)]
        L.supa_last_kernel_times.restype = C.c_int
        L.supa_last_kernel_times.argtypes = [C.c_void_p, C.POINTER(C.c_float), C.c_int32]
        L.supa_philox.restype = C.c_int
        L.supa_philox.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_uint64, C.c_void_p]
        L.supa_azimuth.restype = C.c_int
        L.supa_azimuth.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]
        L.supa_last_error.restype = C.c_char_p
        L.supa_last_error.argtypes = [C.c_void_p]
        _lib = L
    return _lib


def make_geometry(geom: dict, outputs: int):
    """Fill the C struct from a parameter dict; returns (struct, keep-alive list)."""
    N = int(geom["n_planes"])
    keep = []

    R = int(geom.get("n_regions", 0) or 0)
    rings = R if R >= 2 else 1

    def arr(key, ctype, size=N):
        v = geom.get(key)
        if v is None:
            return None
        v = [float(x) if ctype is C.c_double else int(x) for x in v]
        if len(v) != size:
            raise ValueError(f"{key} must have {size} entries")
        a = (ctype * size)(*[ctype(x).value for x in v])
        keep.append(a)
        return C.cast(a, C.POINTER(ctype))

    g = Geometry()
    g.n_planes = N
    g.z_first = float(geom.get("z_first", geom["dz"]))
    g.dz = float(geom["dz"])
    g.layer_of_plane = arr("layer_of_plane", C.c_int32)
    g.p_stop = arr("p_stop", C.c_double, rings * N)
    g.p_split = arr("p_split", C.c_double, rings * N)
    g.n_regions = R
    g.region_r = arr("region_r", C.c_double, R - 1) if R >= 2 else None
    g.e_cut = float(geom["e_cut"])
    g.angle_mode = ANGLE_MODES[geom["angle_mode"]]
    g.angle_a = float(geom.get("angle_a", 0.0))
    g.angle_b = float(geom.get("angle_b", 0.0))
    g.frac_lo = float(geom.get("frac_lo", 0.0))
    g.frac_hi = float(geom.get("frac_hi", 1.0))
    g.energy_frac_bits = int(geom.get("frac_bits", 21))
    g.img_nx = int(geom.get("img_nx", 0))
    g.img_ny = int(geom.get("img_ny", 0))
    g.img_x0 = float(geom.get("img_x0", 0.0))
    g.img_x1 = float(geom.get("img_x1", 0.0))
    g.img_y0 = float(geom.get("img_y0", 0.0))
    g.img_y1 = float(geom.get("img_y1", 0.0))
    g.outputs = outputs
    g.kinematics = KINEMATICS[geom.get("kinematics", "3d")]
    return g, keep


def n_layers(geom: dict) -> int:
    lop = geom.get("layer_of_plane")
    if lop is None:
        return int(geom["n_planes"])
    return int(max(lop)) + 1


def _ptr(t):
    return None if t is None else t.data_ptr()


class Simulator:
    """A library context bound to one device and the current torch stream."""

    def __init__(self, geom: dict, outputs: int = OUT_HITS, device: int = 0,
                 waves_per_cu: int = 0, frontier_cap: int = 0, hit_cap: int = 0,
                 node_cap: int = 0, sub_batches: int = 0, cost_order: int = -1,
                 subtree_phases: int | None = None, export_pool: int = 0):
        self.lib = load()
        if not torch.cuda.is_available():
            raise RuntimeError("libsupa needs a GPU; none is visible")
        self.geom = dict(geom)
        self.outputs = outputs
        self.device = torch.device("cuda", device)
        self.L = n_layers(geom)
        g, keep = make_geometry(geom, outputs)
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
        ctx = C.c_void_p()
        st = self.lib.supa_init_geometry(C.byref(g), device, C.c_void_p(self.stream.cuda_stream),
                                         C.byref(ctx))
        if st != 0:
            raise SupaError(st, self.lib.supa_last_error(None).decode())
        self.ctx = ctx
        if waves_per_cu or frontier_cap or hit_cap or node_cap:
            self.set_launch(waves_per_cu, frontier_cap, hit_cap, node_cap)
        if sub_batches or cost_order != -1:
            self.set_schedule(sub_batches, cost_order)
        if subtree_phases is not None:
            self.set_subtrees(subtree_phases, export_pool)

    def set_launch(self, waves_per_cu=0, frontier_cap=0, hit_cap=0, node_cap=0):
        st = self.lib.supa_set_launch(self.ctx, waves_per_cu, frontier_cap, hit_cap, node_cap)
        self._check(st)

    def set_schedule(self, sub_batches=0, cost_order=-1):
        self._check(self.lib.supa_set_schedule(self.ctx, sub_batches, cost_order))

    def set_subtrees(self, phases=0, export_pool=0):
        """supa_set_subtrees: propagation launches per call (0 = automatic,
        1 = no subtree work items) and the pool size beyond one step from
        which a wave exports."""
        self._check(self.lib.supa_set_subtrees(self.ctx, phases, export_pool))

    def subtree_counts(self):
        """Shared showers and items exported per launch of the last call."""
        v = (C.c_int64 * 5)()
        self._check(self.lib.supa_last_subtrees(self.ctx, v))
        return {"shared": v[0], "items": list(v[1:])}

    def _check(self, st):
        if st != 0:
            raise SupaError(st, self.lib.supa_last_error(self.ctx).decode())

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.supa_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def timing(self):
        """Device ms of the last call: propagation, placement + node scatter,
        whole call, placement alone, node scatter alone."""
        ms = (C.c_float * 5)()
        self._check(self.lib.supa_last_kernel_times(self.ctx, ms, 5))
        return list(ms)

    def wave_times(self):
        """Per-wave busy time (ms) of the last propagation launch, as a list."""
        cap = 32 * 1024
        ms = (C.c_float * cap)()
        count = C.c_int32()
        self._check(self.lib.supa_last_wave_times(self.ctx, ms, cap, C.byref(count)))
        return list(ms[:min(count.value, cap)])

    def allocate(self, n: int, hit_capacity: int = 0, node_capacity: int = 0) -> dict:
        """Output tensors for n showers with the given capacities."""
        dev = self.device
        o = {"ledger": torch.empty((n, 4), dtype=torch.int64, device=dev),
             "counts": torch.empty((n, 6), dtype=torch.int32, device=dev)}
        if self.outputs & OUT_HITS:
            o["hit_offsets"] = torch.empty(n, dtype=torch.int64, device=dev)
            for k in ("hit_x", "hit_y", "hit_e"):
                o[k] = torch.empty(hit_capacity, dtype=torch.float32, device=dev)
            o["hit_layer"] = torch.empty(hit_capacity, dtype=torch.int32, device=dev)
            if self.outputs & OUT_KEYS:
                o["hit_key"] = torch.empty(hit_capacity, dtype=torch.int64, device=dev)
        if self.outputs & OUT_IMAGES:
            o["images"] = torch.empty((n, self.L, int(self.geom["img_ny"]),
                                       int(self.geom["img_nx"])), dtype=torch.float32, device=dev)
        if self.outputs & OUT_TREE:
            o["node_offsets"] = torch.empty(n, dtype=torch.int64, device=dev)
            o["node_parent"] = torch.empty(node_capacity, dtype=torch.int32, device=dev)
            o["node_gen"] = torch.empty(node_capacity, dtype=torch.int32, device=dev)
            for k in ("node_vx", "node_vy", "node_vz", "node_e"):
                o[k] = torch.empty(node_capacity, dtype=torch.float32, device=dev)
            if self.outputs & OUT_KEYS:
                o["node_key"] = torch.empty(node_capacity, dtype=torch.int64, device=dev)
        o["hit_capacity"] = hit_capacity
        o["node_capacity"] = node_capacity
        o["shower_capacity"] = n
        return o

    def _marshal(self, e0, polar, azimuth, out, x0, y0, shower_id_base):
        n = int(e0.shape[0])
        for t in (e0, polar, azimuth, x0, y0):
            if t is not None:
                if t.device != self.device or t.dtype != torch.float32 or not t.is_contiguous() \
                        or t.shape != (n,):
                    raise ValueError("initial conditions must be contiguous float32 device "
                                     "tensors of equal length on the simulator's device")
        b = Batch(_ptr(e0), _ptr(polar), _ptr(azimuth), _ptr(x0), _ptr(y0), n,
                  shower_id_base & 0xFFFFFFFF)
        self._check_output_sizes(out, n)
        o = Output()
        for name, _ in Output._fields_:
            if name in out and isinstance(out[name], torch.Tensor):
                setattr(o, name, out[name].data_ptr())
        o.hit_capacity = int(out.get("hit_capacity", 0))
        o.node_capacity = int(out.get("node_capacity", 0))
        o.shower_capacity = self._shower_capacity(out)
        return b, o

    # elements per shower of the per-shower outputs (images: L * ny * nx)
    _PER_SHOWER = {"ledger": 4, "counts": 6, "hit_offsets": 1, "node_offsets": 1, "images": None}
    _PER_HIT = ("hit_x", "hit_y", "hit_e", "hit_layer", "hit_key")
    _PER_NODE = ("node_parent", "node_gen", "node_vx", "node_vy", "node_vz", "node_e", "node_key")
    # element types the library writes through each pointer
    _DTYPES = {"ledger": (torch.int64, torch.uint64), "counts": (torch.int32,),
               "hit_offsets": (torch.int64,), "node_offsets": (torch.int64,),
               "hit_x": (torch.float32,), "hit_y": (torch.float32,), "hit_e": (torch.float32,),
               "hit_layer": (torch.int32,), "hit_key": (torch.int64, torch.uint64),
               "images": (torch.float32,), "node_parent": (torch.int32,), "node_gen": (torch.int32,),
               "node_vx": (torch.float32,), "node_vy": (torch.float32,), "node_vz": (torch.float32,),
               "node_e": (torch.float32,), "node_key": (torch.int64, torch.uint64)}

    def _per_image(self):
        return self.L * int(self.geom.get("img_ny", 0) or 0) * int(self.geom.get("img_nx", 0) or 0)

    def _shower_capacity(self, out):
        """Showers every per-shower output tensor holds (the library's bound on
        the rows it writes)."""
        per_img = self._per_image()
        cap = None
        for name, k in self._PER_SHOWER.items():
            t = out.get(name)
            if isinstance(t, torch.Tensor):
                per = per_img if k is None else k
                if per > 0:
                    c = t.numel() // per
                    cap = c if cap is None else min(cap, c)
        return 0 if cap is None else cap

    def _check_output_sizes(self, out, n):
        """The library writes per-shower outputs for all n showers of a call
        and per-record outputs up to the stated capacities through plain
        pointers: refuse tensors of the wrong element type or too small for
        that before anything runs."""
        per_img = self._per_image()
        need = {}
        for name, k in self._PER_SHOWER.items():
            need[name] = n * (per_img if k is None else k)
        for name in self._PER_HIT:
            need[name] = int(out.get("hit_capacity", 0))
        for name in self._PER_NODE:
            need[name] = int(out.get("node_capacity", 0))
        for name, m in need.items():
            t = out.get(name)
            if not isinstance(t, torch.Tensor):
                continue
            if t.dtype not in self._DTYPES[name]:
                raise ValueError(f"output '{name}' must have dtype "
                                 f"{' or '.join(str(d) for d in self._DTYPES[name])}, not {t.dtype}")
            if t.device != self.device or not t.is_contiguous() or t.numel() < m:
                raise ValueError(f"output '{name}' must be a contiguous tensor on the simulator's device "
                                 f"holding at least {m} elements for this call ({n} showers); it has "
                                 f"{t.numel()}")

    @staticmethod
    def _totals(out, o):
        out["total_hits"], out["total_nodes"], out["total_steps"] = (o.total_hits, o.total_nodes,
                                                                     o.total_steps)

    def run(self, e0, polar, azimuth, seed: int, out: dict, x0=None, y0=None,
            shower_id_base: int = 0) -> int:
        """One supa_simulate call into preallocated outputs; returns the status
        (OK or CAPACITY) and fills out['total_*']."""
        b, o = self._marshal(e0, polar, azimuth, out, x0, y0, shower_id_base)
        st = self.lib.supa_simulate(self.ctx, C.byref(b), seed & 0xFFFFFFFFFFFFFFFF, C.byref(o))
        self._totals(out, o)
        if st not in (0, 3):
            self._check(st)
        return st

    def run_batches(self, e0, polar, azimuth, seed: int, calls, outs) -> int:
        """supa_simulate_batches: call j simulates showers calls[j] = (s0, m)
        of the initial-condition arrays (global ids s0 .. s0+m-1) into outs[j]
        (dicts as from allocate; record and image tensors may be shared
        between calls, ledger and counts of consecutive calls may not).
        Returns the status (OK or CAPACITY); fills outs[j]['total_*']."""
        k = len(calls)
        if len(outs) != k:
            raise ValueError("one output dict per call")
        bs, os_ = (Batch * max(k, 1))(), (Output * max(k, 1))()
        for j, ((s0, m), out) in enumerate(zip(calls, outs)):
            sl = slice(s0, s0 + m)
            b, o = self._marshal(e0[sl], polar[sl], azimuth[sl], out, None, None, s0)
            bs[j], os_[j] = b, o
        st = self.lib.supa_simulate_batches(self.ctx, k, bs, seed & 0xFFFFFFFFFFFFFFFF, os_)
        for j, out in enumerate(outs):
            self._totals(out, os_[j])
        if st not in (0, 3):
            self._check(st)
        return st

    def run_noalloc(self, e0, polar, azimuth, seed: int, out: dict, x0=None, y0=None,
                    shower_id_base: int = 0) -> int:
        """supa_simulate_noalloc into preallocated outputs (the library's
        scratch from its fixed per-GPU array); returns the status (OK or
        CAPACITY) and fills out['total_*'], raises on other errors."""
        b, o = self._marshal(e0, polar, azimuth, out, x0, y0, shower_id_base)
        st = self.lib.supa_simulate_noalloc(self.ctx, C.byref(b), seed & 0xFFFFFFFFFFFFFFFF, C.byref(o))
        self._totals(out, o)
        if st not in (0, 3):
            self._check(st)
        return st

    def autotune(self, e0, polar, azimuth, seed: int, out: dict, x0=None, y0=None,
                 shower_id_base: int = 0) -> dict:
        """supa_autotune on this batch (outputs preallocated and large
        enough); returns the chosen settings and the fastest call time."""
        b, o = self._marshal(e0, polar, azimuth, out, x0, y0, shower_id_base)
        best = (C.c_int32 * 4)()
        ms = C.c_float()
        st = self.lib.supa_autotune(self.ctx, C.byref(b), seed & 0xFFFFFFFFFFFFFFFF, C.byref(o),
                                    best, C.byref(ms))
        self._totals(out, o)
        self._check(st)
        return {"waves_per_cu": best[0], "frontier_cap": best[1], "sub_batches": best[2],
                "cost_order": best[3], "ms": round(ms.value, 4)}

    def autotune_forget(self):
        """Clears the launch settings supa_autotune keeps per batch size."""
        self._check(self.lib.supa_autotune_forget(self.ctx))

    def graph(self, e0, polar, azimuth, seed: int, out: dict, x0=None, y0=None,
              shower_id_base: int = 0) -> "Graph":
        """Captures this call as a HIP graph (see supa_graph_create)."""
        b, o = self._marshal(e0, polar, azimuth, out, x0, y0, shower_id_base)
        g = C.c_void_p()
        st = self.lib.supa_graph_create(self.ctx, C.byref(b), seed & 0xFFFFFFFFFFFFFFFF, C.byref(o),
                                        C.byref(g))
        self._totals(out, o)
        self._check(st)
        return Graph(self, g, (e0, polar, azimuth, x0, y0), out)

    def simulate(self, e0, polar, azimuth, seed: int, x0=None, y0=None,
                 shower_id_base: int = 0, hit_capacity: int | None = None,
                 node_capacity: int | None = None) -> dict:
        """Simulate a batch; grows the output arrays once if they were too small."""
        n = int(e0.shape[0])
        hc = hit_capacity if hit_capacity is not None else max(1024, 64 * n)
        nc = node_capacity if node_capacity is not None else max(1024, 128 * n)
        hc = hc if self.outputs & OUT_HITS else 0
        nc = nc if self.outputs & OUT_TREE else 0
        out = self.allocate(n, hc, nc)
        st = self.run(e0, polar, azimuth, seed, out, x0, y0, shower_id_base)
        if st == 3:
            # only the record arrays grow: the per-shower outputs (images
            # included) are kept, so the device never holds two sets of them
            hc, nc = max(hc, out["total_hits"]), max(nc, out["total_nodes"])
            for k in self._PER_HIT + self._PER_NODE:
                out.pop(k, None)
            grown = self.allocate(0, hc, nc)
            for k in self._PER_HIT + self._PER_NODE + ("hit_capacity", "node_capacity"):
                if k in grown:
                    out[k] = grown[k]
            st = self.run(e0, polar, azimuth, seed, out, x0, y0, shower_id_base)
            self._check(st)
        th, tn = out["total_hits"], out["total_nodes"]
        for k in ("hit_x", "hit_y", "hit_e", "hit_layer", "hit_key"):
            if k in out:
                out[k] = out[k][:th]
        for k in ("node_parent", "node_gen", "node_vx", "node_vy", "node_vz", "node_e", "node_key"):
            if k in out:
                out[k] = out[k][:tn]
        return out

    def azimuth(self, w: torch.Tensor):
        """The kernel's sine and cosine of the azimuth 2 pi u(w) for uint32
        words w (int32 tensor, n) -> (sin, cos), float32 (n)."""
        w = w.contiguous()
        sn = torch.empty(w.shape[0], dtype=torch.float32, device=w.device)
        cs = torch.empty_like(sn)
        self._check(self.lib.supa_azimuth(self.ctx, w.data_ptr(), w.shape[0], sn.data_ptr(), cs.data_ptr()))
        return sn, cs

    def philox(self, ctr: torch.Tensor, key: int) -> torch.Tensor:
        """Philox4x32-10 blocks on the device: ctr int32/uint32 (n, 4) -> (n, 4)."""
        ctr = ctr.contiguous()
        out = torch.empty_like(ctr)
        self._check(self.lib.supa_philox(self.ctx, ctr.data_ptr(), ctr.shape[0],
                                         key & 0xFFFFFFFFFFFFFFFF, out.data_ptr()))
        return out


def validate_geometry(geom: dict, outputs: int = OUT_HITS):
    """Host-only check of the parameters (no GPU needed); raises SupaError."""
    lib = load()
    g, keep = make_geometry(geom, outputs)
    st = lib.supa_validate_geometry(C.byref(g))
    if st != 0:
        raise SupaError(st, lib.supa_last_error(None).decode())


def validate_call(geom: dict, outputs: int, n: int, out: dict):
    """Host-only check of a simulate call's arguments through the C ABI
    (supa_validate_call: no GPU needed).  `out` maps output names to
    integers standing for device addresses (never dereferenced) plus
    hit_capacity, node_capacity and shower_capacity; raises SupaError."""
    lib = load()
    g, keep = make_geometry(geom, outputs)
    fake = 4096
    b = Batch(fake, fake, fake, None, None, n, 0)
    o = Output()
    for name, _ in Output._fields_:
        if name in out:
            setattr(o, name, out[name])
    st = lib.supa_validate_call(C.byref(g), C.byref(b), C.byref(o))
    if st != 0:
        raise SupaError(st, lib.supa_last_error(None).decode())


class Graph:
    """A captured supa_simulate call; keeps its tensors alive."""

    def __init__(self, sim: Simulator, handle, inputs, out):
        self.sim, self.handle, self.inputs, self.out = sim, handle, inputs, out

    def launch(self, stream=None):
        s = (stream or torch.cuda.current_stream(self.sim.device)).cuda_stream
        self.sim._check(self.sim.lib.supa_graph_launch(self.handle, C.c_void_p(s)))

    def check(self, stream=None):
        s = (stream or torch.cuda.current_stream(self.sim.device)).cuda_stream
        t = (C.c_int64 * 3)()
        st = self.sim.lib.supa_graph_check(self.handle, C.c_void_p(s), t)
        self.out["total_hits"], self.out["total_nodes"], self.out["total_steps"] = t[0], t[1], t[2]
        self.sim._check(st)

    def close(self):
        if self.handle:
            self.sim.lib.supa_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
