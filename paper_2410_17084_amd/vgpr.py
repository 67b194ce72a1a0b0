"""Thin ctypes binding of libvgpr.so (the C ABI in include/vgpr.h).

Argument marshalling only: every step of the hot path runs in the HIP library.
PyTorch provides device memory (tensors' data_ptr) and the stream. Loading
fails loudly when the library has not been built; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import weakref
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvgpr.so")

OK, E_INVALID, E_NOMEM, E_CAPACITY, E_RANGE, E_BUDGET, E_DEVICE, E_UNSUPPORTED = range(8)
ST_SOLVED, ST_BELOW_TAU, ST_CAPPED, ST_REFINED, ST_FACTOR_FAIL, ST_CONVERGED, ST_AXIS_TIE = 1, 2, 4, 8, 16, 32, 64
PREC_FP32, PREC_MIXED, PREC_FP64 = 0, 1, 2

# every entry point include/vgpr.h declares
SYMBOLS = [
    "vgpr_params_default", "vgpr_status_str", "vgpr_create", "vgpr_destroy", "vgpr_set_stream",
    "vgpr_last_error", "vgpr_workspace_bytes", "vgpr_voxelize", "vgpr_fit_predict", "vgpr_fit_predict_noalloc", "vgpr_map_create", "vgpr_map_create_ex", "vgpr_map_export", "vgpr_map_import",
    "vgpr_map_destroy", "vgpr_map_update", "vgpr_map_stats", "vgpr_profile_enable", "vgpr_profile_read",
    "vgpr_set_tuning", "vgpr_get_tuning", "vgpr_fit_graph_create", "vgpr_graph_launch", "vgpr_graph_destroy",
    "vgpr_gauss_init", "vgpr_structure_loss",
]


class Params(C.Structure):
    _fields_ = [
        ("voxel_size", C.c_float), ("max_pts", C.c_int32), ("min_pts", C.c_int32), ("grid_side", C.c_int32),
        ("signal_var", C.c_float), ("length_scale", C.c_float), ("noise_var", C.c_float),
        ("ls_mode", C.c_int32), ("frame_mode", C.c_int32), ("precision", C.c_int32),
        ("refine_threshold", C.c_float), ("converge_var", C.c_float), ("cond_threshold", C.c_float),
    ]

    def replace(self, **kw) -> "Params":
        p = Params()
        C.pointer(p)[0] = self
        for k, v in kw.items():
            setattr(p, k, v)
        return p

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


# stream of each size bucket when the buckets fork (0: the context's stream, 1..3: side streams)
DEFAULT_BUCKET_STREAM = (0, 2, 2, 1, 1, 3, 3)


class Tuning(C.Structure):
    _fields_ = [("fp32_last_bucket", C.c_int32), ("wave_last_bucket", C.c_int32), ("streams", C.c_int32),
                ("grid_scale", C.c_int32 * 7), ("tile_first_bucket", C.c_int32), ("tiled_first", C.c_int32),
                ("bucket_stream", C.c_int32 * 7), ("tiled_merge", C.c_int32)]

    def as_dict(self) -> dict:
        return {"fp32_last_bucket": self.fp32_last_bucket, "wave_last_bucket": self.wave_last_bucket,
                "streams": self.streams, "grid_scale": list(self.grid_scale),
                "tile_first_bucket": self.tile_first_bucket, "tiled_first": self.tiled_first,
                "bucket_stream": list(self.bucket_stream), "tiled_merge": self.tiled_merge}

    @classmethod
    def from_dict(cls, d: dict) -> "Tuning":
        """Entries missing from `d` (older caches) take the library defaults."""
        t = cls()
        t.fp32_last_bucket = d.get("fp32_last_bucket", 0)
        t.wave_last_bucket = d.get("wave_last_bucket", 2)
        t.streams = d.get("streams", 3)
        gs = list(d.get("grid_scale", []))
        for i in range(7):
            t.grid_scale[i] = gs[i] if i < len(gs) else 4
        t.tile_first_bucket = d.get("tile_first_bucket", 5)
        t.tiled_first = d.get("tiled_first", 0)
        bs = list(d.get("bucket_stream", DEFAULT_BUCKET_STREAM))
        for i in range(7):
            t.bucket_stream[i] = bs[i]
        t.tiled_merge = d.get("tiled_merge", 0)
        return t


class VgprError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


_lib = None


def load():
    """Load libvgpr.so and declare its signatures. Raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc for gfx950)")
    # PyTorch ships its own HIP runtime under the same soname as the system's.
    # Importing it first makes libvgpr.so bind to that runtime, the one that owns
    # the tensors and streams passed in; loaded the other way round, the process
    # would hold two HIP runtimes and the second to initialise sees no device.
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    vp, i64, i32, sz = C.c_void_p, C.c_int64, C.c_int32, C.c_size_t
    P = C.POINTER
    sig = {
        "vgpr_params_default": (None, [P(Params)]),
        "vgpr_status_str": (C.c_char_p, [C.c_int]),
        "vgpr_create": (C.c_int, [C.c_int, vp, sz, P(vp)]),
        "vgpr_destroy": (C.c_int, [vp]),
        "vgpr_set_stream": (C.c_int, [vp, vp]),
        "vgpr_last_error": (C.c_char_p, [vp]),
        "vgpr_workspace_bytes": (sz, [vp]),
        "vgpr_voxelize": (C.c_int, [vp, vp, i64, P(i64), i32, P(Params), vp, vp, vp, vp, i64, P(i64), P(i64),
                                    P(i64)]),
        "vgpr_fit_predict": (C.c_int, [vp, vp, i64, vp, vp, vp, vp, i64, vp, P(Params), vp, vp, vp]),
        "vgpr_fit_predict_noalloc": (C.c_int, [vp, vp, i64, vp, vp, vp, vp, i64, vp, P(Params), vp, vp, vp]),
        "vgpr_map_create": (C.c_int, [vp, P(Params), i64, P(vp)]),
        "vgpr_map_create_ex": (C.c_int, [vp, P(Params), i64, C.c_int, P(vp)]),
        "vgpr_map_export": (C.c_int, [vp, vp, sz, P(sz)]),
        "vgpr_map_import": (C.c_int, [vp, vp, sz, i64, P(vp)]),
        "vgpr_map_destroy": (C.c_int, [vp]),
        "vgpr_map_update": (C.c_int, [vp, vp, i64, vp, vp, vp, vp, i64, P(i64)]),
        "vgpr_map_stats": (C.c_int, [vp, P(i64), P(i64), P(i64)]),
        "vgpr_profile_enable": (C.c_int, [vp, C.c_int]),
        "vgpr_profile_read": (C.c_int, [vp, C.c_char_p, P(C.c_double), P(i64)]),
        "vgpr_set_tuning": (C.c_int, [vp, P(Tuning)]),
        "vgpr_get_tuning": (C.c_int, [vp, P(Tuning)]),
        "vgpr_fit_graph_create": (C.c_int, [vp, vp, i64, vp, vp, vp, vp, i64, vp, P(Params), vp, vp, vp, P(vp)]),
        "vgpr_graph_launch": (C.c_int, [vp]),
        "vgpr_graph_destroy": (C.c_int, [vp]),
        "vgpr_gauss_init": (C.c_int, [vp, vp, vp, i64, i32, i32, C.c_float, vp]),
        "vgpr_structure_loss": (C.c_int, [vp, vp, i64, vp, i64, C.c_float, C.c_int, vp, vp, P(C.c_double),
                                          P(i64)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def default_params(**kw) -> Params:
    p = Params()
    load().vgpr_params_default(C.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _f32_dev(t, name: str):
    """The library reads raw device pointers: inputs must be contiguous float32 GPU tensors."""
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous float32 CUDA tensor")
    return t


@dataclass
class Voxels:
    keys: object      # (V,) int64 tensor holding the uint64 key bits
    offsets: object   # (V,) int32
    counts: object    # (V,) int32
    perm: object      # (N,) int32
    n_vox: int
    frame_vox: list
    n_invalid: int


class Context:
    """One vgpr_ctx on a device, enqueuing on a torch stream (default: the current one)."""

    def __init__(self, device: int = 0, stream=None, hbm_budget: int = 0):
        import torch
        self.torch = torch
        self.lib = load()
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        h = C.c_void_p()
        st = self.lib.vgpr_create(device, C.c_void_p(self.stream.cuda_stream), hbm_budget, C.byref(h))
        if st != OK:
            why = (self.lib.vgpr_last_error(None) or b"").decode()
            raise VgprError(st, f"vgpr_create failed: {self.lib.vgpr_status_str(st).decode()} ({why})")
        self.h = h
        self._maps = weakref.WeakSet()
        self._graphs = weakref.WeakSet()

    def close(self):
        if getattr(self, "h", None):
            for m in list(self._maps):
                m.close()
            for g in list(self._graphs):
                g.close()
            self._check(self.lib.vgpr_destroy(self.h), "vgpr_destroy")
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, what):
        if st != OK:
            msg = self.lib.vgpr_last_error(self.h).decode()
            raise VgprError(st, f"{what}: {self.lib.vgpr_status_str(st).decode()}: {msg}")

    def set_stream(self, stream):
        self.stream = stream
        self._check(self.lib.vgpr_set_stream(self.h, C.c_void_p(stream.cuda_stream)), "vgpr_set_stream")

    def workspace_bytes(self) -> int:
        return int(self.lib.vgpr_workspace_bytes(self.h))

    # -- vgpr_voxelize -------------------------------------------------------
    def voxelize(self, xyz, params: Params, frame_offsets=None, cap_vox: int | None = None) -> Voxels:
        torch = self.torch
        _f32_dev(xyz, "xyz")
        n = xyz.numel() // 3
        dev = xyz.device
        cap = n if cap_vox is None else int(cap_vox)
        keys = torch.empty(max(cap, 1), dtype=torch.int64, device=dev)
        offs = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
        cnts = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
        perm = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
        nf = 1 if frame_offsets is None else len(frame_offsets) - 1
        fo = None if frame_offsets is None else (C.c_int64 * (nf + 1))(*[int(x) for x in frame_offsets])
        fv = (C.c_int64 * (nf + 1))()
        nv = C.c_int64()
        ninv = C.c_int64()
        st = self.lib.vgpr_voxelize(self.h, _ptr(xyz), n, fo, nf, C.byref(params), _ptr(keys), _ptr(offs),
                                    _ptr(cnts), _ptr(perm), cap, C.byref(nv), fv, C.byref(ninv))
        self._check(st, "vgpr_voxelize")
        v = nv.value
        return Voxels(keys[:v], offs[:v], cnts[:v], perm[:n], v, list(fv), ninv.value)

    # -- vgpr_fit_predict ----------------------------------------------------
    def fit_predict(self, xyz, vox: Voxels, params: Params, noise_var=None, out=None):
        torch = self.torch
        _f32_dev(xyz, "xyz")
        if noise_var is not None:
            _f32_dev(noise_var, "noise_var")
        m = params.grid_side * params.grid_side
        dev = xyz.device
        v = vox.n_vox
        if out is None:
            out = (torch.empty((max(v, 1), m, 4), dtype=torch.float32, device=dev),
                   torch.empty(max(v, 1), dtype=torch.int8, device=dev),
                   torch.empty(max(v, 1), dtype=torch.uint8, device=dev))
        o, ax, stt = out
        st = self.lib.vgpr_fit_predict(self.h, _ptr(xyz), xyz.numel() // 3, _ptr(vox.keys), _ptr(vox.offsets),
                                       _ptr(vox.counts),
                                       _ptr(vox.perm), v, _ptr(noise_var), C.byref(params), _ptr(o), _ptr(ax),
                                       _ptr(stt))
        self._check(st, "vgpr_fit_predict")
        return o[:v], ax[:v], stt[:v]

    def fit_predict_noalloc(self, xyz, vox: Voxels, params: Params, out, noise_var=None):
        """vgpr_fit_predict_noalloc: the same call on the fixed device scratch. `out` is
        the caller's (out, axis, status) tensors, at least n_vox rows each."""
        _f32_dev(xyz, "xyz")
        if noise_var is not None:
            _f32_dev(noise_var, "noise_var")
        o, ax, stt = out
        v = vox.n_vox
        m = params.grid_side * params.grid_side
        if o.shape[0] < v or ax.shape[0] < v or stt.shape[0] < v or o.shape[1] != m:
            raise ValueError("out tensors hold fewer than n_vox rows or the wrong grid size")
        st = self.lib.vgpr_fit_predict_noalloc(self.h, _ptr(xyz), xyz.numel() // 3, _ptr(vox.keys),
                                               _ptr(vox.offsets), _ptr(vox.counts), _ptr(vox.perm), v,
                                               _ptr(noise_var), C.byref(params), _ptr(o), _ptr(ax), _ptr(stt))
        self._check(st, "vgpr_fit_predict_noalloc")
        return o[:v], ax[:v], stt[:v]

    def fit_graph(self, xyz, vox: Voxels, params: Params, noise_var=None, out=None) -> "Graph":
        """Capture this fit_predict call as a replayable graph (vgpr_fit_graph_create).

        The context must run on a non-default stream. The graph keeps references
        to every tensor it reads or writes; replays read their current contents.
        """
        torch = self.torch
        _f32_dev(xyz, "xyz")
        if noise_var is not None:
            _f32_dev(noise_var, "noise_var")
        m = params.grid_side * params.grid_side
        dev = xyz.device
        v = vox.n_vox
        if out is None:
            out = (torch.empty((max(v, 1), m, 4), dtype=torch.float32, device=dev),
                   torch.empty(max(v, 1), dtype=torch.int8, device=dev),
                   torch.empty(max(v, 1), dtype=torch.uint8, device=dev))
        o, ax, stt = out
        h = C.c_void_p()
        st = self.lib.vgpr_fit_graph_create(self.h, _ptr(xyz), xyz.numel() // 3, _ptr(vox.keys), _ptr(vox.offsets),
                                            _ptr(vox.counts), _ptr(vox.perm), v, _ptr(noise_var), C.byref(params),
                                            _ptr(o), _ptr(ax), _ptr(stt), C.byref(h))
        self._check(st, "vgpr_fit_graph_create")
        g = Graph(self, h, (xyz, vox, noise_var, out), (o[:v], ax[:v], stt[:v]))
        self._graphs.add(g)
        return g

    # -- vgpr_gauss_init -----------------------------------------------------
    def gauss_init(self, out, status, grid_side: int, n_r: int, var_floor: float = 1e-8, gauss=None):
        """Initial 3D Gaussians of each n_r x n_r subgrid: (V, n_s^2, 8) float32."""
        torch = self.torch
        _f32_dev(out, "out")
        v = int(status.shape[0])
        ns = grid_side // n_r if n_r > 0 else 0
        if gauss is None:
            gauss = torch.empty((max(v, 1), max(ns * ns, 1), 8), dtype=torch.float32, device=out.device)
        st = self.lib.vgpr_gauss_init(self.h, _ptr(out), _ptr(status), v, int(grid_side), int(n_r),
                                      float(var_floor), _ptr(gauss))
        self._check(st, "vgpr_gauss_init")
        return gauss[:v]

    def structure_loss(self, pts, gauss, cell_size: float, scale_mode: int = 0, value=None, arg=None):
        """L_p of Eq. (9) for the scan points against Gaussians in the gauss_init
        layout: (loss, n_valid, value (n,) float32, index (n,) int32)."""
        torch = self.torch
        _f32_dev(pts, "pts")
        _f32_dev(gauss, "gauss")
        n = pts.numel() // 3
        g = gauss.reshape(-1, 8) if gauss.numel() else gauss
        ng = gauss.numel() // 8
        if value is None:
            value = torch.empty(max(n, 1), dtype=torch.float32, device=pts.device)
        if arg is None:
            arg = torch.empty(max(n, 1), dtype=torch.int32, device=pts.device)
        loss, nv = C.c_double(), C.c_int64()
        st = self.lib.vgpr_structure_loss(self.h, _ptr(pts), n, _ptr(g) if ng else None, ng, float(cell_size),
                                          int(scale_mode), _ptr(value), _ptr(arg), C.byref(loss), C.byref(nv))
        self._check(st, "vgpr_structure_loss")
        return loss.value, nv.value, value[:n], arg[:n]

    # -- launch tuning ----------------------------------------------------------
    def tuning(self) -> Tuning:
        t = Tuning()
        self._check(self.lib.vgpr_get_tuning(self.h, C.byref(t)), "vgpr_get_tuning")
        return t

    def set_tuning(self, t: Tuning):
        self._check(self.lib.vgpr_set_tuning(self.h, C.byref(t)), "vgpr_set_tuning")

    # -- timing ---------------------------------------------------------------
    def profile(self, on: bool = True):
        self._check(self.lib.vgpr_profile_enable(self.h, 1 if on else 0), "vgpr_profile_enable")

    def profile_read(self, name: str):
        ms = C.c_double()
        cnt = C.c_int64()
        self._check(self.lib.vgpr_profile_read(self.h, name.encode(), C.byref(ms), C.byref(cnt)),
                    "vgpr_profile_read")
        return ms.value, cnt.value


class Graph:
    """A captured fit_predict (vgpr_graph); `outputs` are views of the buffers it writes."""

    def __init__(self, ctx: Context, h, keep, outputs):
        self.ctx = ctx
        self.h = h
        self._keep = keep
        self.outputs = outputs

    def launch(self):
        self.ctx._check(self.ctx.lib.vgpr_graph_launch(self.h), "vgpr_graph_launch")
        return self.outputs

    def close(self):
        if getattr(self, "h", None) and getattr(self.ctx, "h", None):
            self.ctx.lib.vgpr_graph_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Map:
    """A device-resident voxel map (vgpr_map) bound to a Context; feedback=True
    selects update mode 1 (the covariance-centred update of type (c) voxels)."""

    def __init__(self, ctx: Context, params: Params, max_voxels: int, feedback: bool = False, _handle=None):
        self.ctx = ctx
        self.params = params
        self.feedback = bool(feedback)
        if _handle is None:
            h = C.c_void_p()
            ctx._check(ctx.lib.vgpr_map_create_ex(ctx.h, C.byref(params), int(max_voxels), int(self.feedback),
                                                  C.byref(h)), "vgpr_map_create_ex")
            _handle = h
        self.h = _handle
        ctx._maps.add(self)

    def export(self) -> bytes:
        """The map's whole state as bytes (vgpr_map_export)."""
        need = C.c_size_t()
        self.ctx._check(self.ctx.lib.vgpr_map_export(self.h, None, 0, C.byref(need)), "vgpr_map_export")
        buf = C.create_string_buffer(need.value)
        self.ctx._check(self.ctx.lib.vgpr_map_export(self.h, buf, need.value, C.byref(need)), "vgpr_map_export")
        return buf.raw[:need.value]

    @classmethod
    def load(cls, ctx: Context, data: bytes, max_voxels: int) -> "Map":
        """A new map holding a state written by export (vgpr_map_import)."""
        h = C.c_void_p()
        ctx._check(ctx.lib.vgpr_map_import(ctx.h, data, len(data), int(max_voxels), C.byref(h)), "vgpr_map_import")
        prm = Params.from_buffer_copy(data[24:24 + C.sizeof(Params)])  # header: params at byte 24
        mode = int.from_bytes(data[12:16], "little", signed=True)
        return cls(ctx, prm, max_voxels, feedback=mode == 1, _handle=h)

    def close(self):
        if getattr(self, "h", None) and getattr(self.ctx, "h", None):
            self.ctx.lib.vgpr_map_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def update(self, xyz, cap_upd: int | None = None, out=None):
        torch = self.ctx.torch
        _f32_dev(xyz, "xyz")
        n = xyz.numel() // 3
        m = self.params.grid_side ** 2
        cap = n if cap_upd is None else int(cap_upd)
        dev = xyz.device
        if out is None:
            out = (torch.empty(max(cap, 1), dtype=torch.int64, device=dev),
                   torch.empty((max(cap, 1), m, 4), dtype=torch.float32, device=dev),
                   torch.empty(max(cap, 1), dtype=torch.int8, device=dev),
                   torch.empty(max(cap, 1), dtype=torch.uint8, device=dev))
        k, o, ax, st_ = out
        nu = C.c_int64()
        st = self.ctx.lib.vgpr_map_update(self.h, _ptr(xyz), n, _ptr(k), _ptr(o), _ptr(ax), _ptr(st_), cap,
                                          C.byref(nu))
        self.ctx._check(st, "vgpr_map_update")
        u = nu.value
        return k[:u], o[:u], ax[:u], st_[:u]

    def stats(self):
        a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
        self.ctx._check(self.ctx.lib.vgpr_map_stats(self.h, C.byref(a), C.byref(b), C.byref(c)), "vgpr_map_stats")
        return {"voxels": a.value, "points": b.value, "converged": c.value}
