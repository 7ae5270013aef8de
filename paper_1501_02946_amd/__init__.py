"""NEDNER-NUFFT planar photoacoustic reconstruction for AMD MI355X (gfx950).

A thin ctypes binding over ``libnedner.so``: the C-ABI declared in
``include/nedner.h``. Every step of the operator runs in the library's HIP
kernels; PyTorch only supplies device memory and the current stream. The
binding marshals arguments and checks shapes, nothing more, and it raises if
the library is not built (there is no CPU fallback).

    plan = Plan(xy, nt=512, dt=1/512, volume=(128, 128, 256))
    f = plan(g)                       # data (M, Nt) -> image (N1, N2, N3)
    g2 = plan.adjoint(f)              # exact transpose
    f = NednerRecon.apply(g, plan)    # differentiable forward
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

__all__ = ["Plan", "BatchPlan", "NednerRecon", "NednerAdjoint", "NednerQ", "NednerError", "lib", "lsq",
           "mip", "corrcoef", "tenenbaum",
           "power_norm", "PRECISIONS", "KINDS", "FLAGS", "desc_struct", "info_struct",
           "query"]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libnedner.so")

PRECISIONS = {"fp64": 0, "fp32": 1, "fp32c": 2, "fp32_plain": 3, "fp32w": 4}
KINDS = {"volume": 0, "spectrum": 1, "grid": 2}
FLAGS = {"allow_alias": 1, "wrap": 2, "deterministic": 4, "no_autotune": 8, "equispaced": 16}
WINDOWS = {"gaussian": 0, "kaiser_bessel": 1, "kb": 1}
STATUS = {0: "ok", 1: "E_ARG", 2: "E_ALIAS", 3: "E_OOM", 4: "E_WORKSPACE", 5: "E_HIP",
          6: "E_UNSUPPORTED", 7: "E_STATE"}


class NednerError(RuntimeError):
    """A non-OK status from the library; `.status` holds the code."""

    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class desc_struct(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("xy", ctypes.c_void_p), ("h", ctypes.c_void_p),
                ("nt", ctypes.c_int64), ("t0", ctypes.c_double), ("dt", ctypes.c_double),
                ("c", ctypes.c_double), ("n1", ctypes.c_int32), ("n2", ctypes.c_int32),
                ("n3", ctypes.c_int32), ("a1", ctypes.c_double), ("a2", ctypes.c_double),
                ("d1", ctypes.c_double), ("d2", ctypes.c_double), ("d3", ctypes.c_double),
                ("prec", ctypes.c_int32), ("w", ctypes.c_int32), ("sigma", ctypes.c_double),
                ("tau_scale", ctypes.c_double), ("flags", ctypes.c_uint32),
                ("rows_per_wave", ctypes.c_int32), ("time_per_lane", ctypes.c_int32),
                ("window", ctypes.c_int32)]


class info_struct(ctypes.Structure):
    _fields_ = [("n1_os", ctypes.c_int32), ("n2_os", ctypes.c_int32), ("nt_os", ctypes.c_int32),
                ("columns", ctypes.c_int32), ("segments", ctypes.c_int32),
                ("rows_per_wave", ctypes.c_int32), ("time_per_lane", ctypes.c_int32),
                ("pad0", ctypes.c_int32), ("workspace_bytes", ctypes.c_size_t),
                ("table_bytes", ctypes.c_size_t), ("beta", ctypes.c_double),
                ("max_abs_theta", ctypes.c_double), ("list_entries", ctypes.c_int64)]


class tuning_struct(ctypes.Structure):
    _fields_ = [("rows_per_wave", ctypes.c_int32), ("time_per_lane", ctypes.c_int32),
                ("spread_depth", ctypes.c_int32), ("pass_lines", ctypes.c_int32),
                ("pass_threads", ctypes.c_int32), ("pass_inplace", ctypes.c_int32),
                ("gather_rows", ctypes.c_int32), ("pad1", ctypes.c_int32),
                ("ms_spread", ctypes.c_double), ("ms_execute", ctypes.c_double)]


def _tuning_dict(t) -> dict:
    return {k: getattr(t, k) for k, _ in tuning_struct._fields_ if k != "pad1"}


_LIB = None

EXPORTS = ["nedner_desc_init", "nedner_validate", "nedner_query", "nedner_plan_create",
           "nedner_plan_create_many", "nedner_plan_info", "nedner_workspace_size",
           "nedner_set_workspace", "nedner_execute", "nedner_execute_adjoint",
           "nedner_execute_many", "nedner_destroy", "nedner_status_string",
           "nedner_last_error", "nedner_version", "nedner_profile_begin", "nedner_profile_end",
           "nedner_get_tuning", "nedner_set_tuning", "nedner_autotune", "nedner_execute_q",
           "nedner_execute_q_adjoint", "nedner_metrics_workspace_size", "nedner_mip",
           "nedner_corrcoef", "nedner_tenenbaum", "nedner_tenenbaum_mean",
           "nedner_debug_inject_hip_error", "nedner_corrcoef_noalloc"]


def _declare(L):
    vp, i32, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t
    D = ctypes.POINTER(desc_struct)
    L.nedner_desc_init.argtypes = [D]
    L.nedner_desc_init.restype = None
    L.nedner_validate.argtypes = [D]
    L.nedner_query.argtypes = [D, ctypes.POINTER(info_struct)]
    L.nedner_plan_create.argtypes = [D, i32, vp, ctypes.POINTER(vp)]
    L.nedner_plan_create_many.argtypes = [D, i32, i32, vp, ctypes.POINTER(vp)]
    L.nedner_plan_info.argtypes = [vp, ctypes.POINTER(info_struct)]
    L.nedner_workspace_size.argtypes = [vp, ctypes.POINTER(sz)]
    L.nedner_set_workspace.argtypes = [vp, vp, sz]
    L.nedner_execute.argtypes = [vp, vp, vp, i32, vp]
    L.nedner_execute_adjoint.argtypes = [vp, vp, i32, vp, vp]
    L.nedner_execute_many.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), i32, vp]
    L.nedner_execute_q.argtypes = [vp, vp, vp, vp]
    i64 = ctypes.c_int64
    L.nedner_metrics_workspace_size.argtypes = []
    L.nedner_metrics_workspace_size.restype = sz
    L.nedner_mip.argtypes = [vp, i32, i32, i32, i32, i32, vp, vp]
    L.nedner_corrcoef.argtypes = [vp, vp, vp, i64, i32, vp, vp, sz, vp]
    L.nedner_corrcoef_noalloc.argtypes = [vp, vp, vp, i64, i32, vp, vp]
    L.nedner_tenenbaum.argtypes = [vp, i64, i64, i64, i64, i64, i64, i32, vp, vp, sz, vp]
    L.nedner_tenenbaum_mean.argtypes = [vp, i64, i64, i64, i64, i64, i64, i32, vp, vp, sz, vp]
    L.nedner_execute_q_adjoint.argtypes = [vp, vp, vp, vp]
    L.nedner_destroy.argtypes = [vp]
    L.nedner_debug_inject_hip_error.argtypes = [vp, i32]
    L.nedner_status_string.argtypes = [i32]
    L.nedner_status_string.restype = ctypes.c_char_p
    L.nedner_last_error.argtypes = []
    L.nedner_last_error.restype = ctypes.c_char_p
    L.nedner_version.argtypes = []
    L.nedner_profile_begin.argtypes = [vp, i32]
    L.nedner_profile_end.argtypes = [vp, ctypes.POINTER(ctypes.c_double), i32, ctypes.POINTER(i32),
                                     ctypes.POINTER(ctypes.c_char_p)]
    T = ctypes.POINTER(tuning_struct)
    L.nedner_get_tuning.argtypes = [vp, T]
    L.nedner_set_tuning.argtypes = [vp, T]
    L.nedner_autotune.argtypes = [vp, vp, vp, T]
    for name in EXPORTS:
        if name not in ("nedner_desc_init", "nedner_status_string", "nedner_last_error",
                        "nedner_metrics_workspace_size"):
            getattr(L, name).restype = ctypes.c_int


def lib():
    """Load libnedner.so (after torch, so both use one HIP runtime)."""
    global _LIB
    if _LIB is None:
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise NednerError(5, f"{LIB_PATH} is not built; run `python -m paper_1501_02946_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        _declare(L)
        _LIB = L
    return _LIB


def _check(st: int):
    if st != 0:
        msg = lib().nedner_last_error().decode(errors="replace")
        raise NednerError(st, msg)


def _make_desc(xy, h, nt, dt, n1, n2, n3, c=1.0, t0=0.0, a1=0.0, a2=0.0, d1=0.0, d2=0.0,
               d3=0.0, precision="fp32c", w=12, sigma=2.0, tau_scale=1.0, flags=0,
               rows_per_wave=0, time_per_lane=0, window="gaussian"):
    L = lib()
    d = desc_struct()
    L.nedner_desc_init(ctypes.byref(d))
    xy = np.ascontiguousarray(np.asarray(xy, dtype=np.float64).reshape(-1, 2))
    d.m = xy.shape[0]
    d.xy = xy.ctypes.data
    keep = [xy]
    if h is not None:
        harr = np.ascontiguousarray(np.asarray(h, dtype=np.float64).reshape(-1))
        if harr.shape[0] != xy.shape[0]:
            raise ValueError("h must have one entry per sensor")
        d.h = harr.ctypes.data
        keep.append(harr)
    d.nt, d.dt, d.c, d.t0 = int(nt), float(dt), float(c), float(t0)
    d.n1, d.n2, d.n3 = int(n1), int(n2), int(n3)
    d.a1, d.a2 = float(a1), float(a2)
    d.d1 = float(d1) if d1 else 1.0 / int(n1)
    d.d2 = float(d2) if d2 else 1.0 / int(n2)
    d.d3 = float(d3)
    d.prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    d.w, d.sigma, d.tau_scale = int(w), float(sigma), float(tau_scale)
    if isinstance(flags, (list, tuple)):
        flags = sum(FLAGS[f] for f in flags)
    d.flags = int(flags)
    d.rows_per_wave, d.time_per_lane = int(rows_per_wave), int(time_per_lane)
    d.window = WINDOWS[window] if isinstance(window, str) else int(window)
    return d, keep


def query(xy, nt, dt, volume, **kw) -> dict:
    """Host-only: validate a configuration and return the sizes it implies."""
    n1, n2, n3 = volume
    d, keep = _make_desc(xy, kw.pop("h", None), nt, dt, n1, n2, n3, **kw)
    info = info_struct()
    _check(lib().nedner_query(ctypes.byref(d), ctypes.byref(info)))
    del keep
    return {k: getattr(info, k) for k, _ in info_struct._fields_ if k != "pad0"}


class Plan:
    """One reconstruction operator: fixed sensors, time grid and output grid.

    Parameters follow the C descriptor: sensor positions `xy` (M, 2), time
    samples `nt` at t0 + n dt, sound speed `c`, output `volume` = (N1, N2, N3)
    with voxel (i1, i2, i3) at (a1 + i1 d1, a2 + i2 d2, i3 d3); d1, d2 default
    to a unit aperture, d3 to c nt dt / N3. `precision` is one of "fp64",
    "fp32", "fp32c" (compensated float sums), "fp32_plain" (float arguments
    too) or "fp32w" (double spreading sums); `window` is
    "gaussian" (default) or "kaiser_bessel" with `w` taps per axis.
    """

    def __init__(self, xy, nt, dt, volume, c=1.0, h=None, t0=0.0, a1=0.0, a2=0.0, d1=0.0,
                 d2=0.0, d3=0.0, precision="fp32c", w=12, sigma=2.0, tau_scale=1.0, flags=0,
                 rows_per_wave=0, time_per_lane=0, window="gaussian", device=None):
        import torch
        self._torch = torch
        if not torch.cuda.is_available():
            raise NednerError(5, "no GPU: the NEDNER library runs on MI355X only")
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else int(device))
        n1, n2, n3 = (int(v) for v in volume)
        d, keep = _make_desc(xy, h, nt, dt, n1, n2, n3, c=c, t0=t0, a1=a1, a2=a2, d1=d1, d2=d2,
                             d3=d3, precision=precision, w=w, sigma=sigma, tau_scale=tau_scale,
                             flags=flags, rows_per_wave=rows_per_wave, time_per_lane=time_per_lane,
                             window=window)
        self.m, self.nt, self.volume = int(d.m), int(nt), (n1, n2, n3)
        self.precision = precision
        self._w, self._sigma, self._window = int(w), float(sigma), int(d.window)
        self.dtype = torch.float64 if d.prec == 0 else torch.float32
        self._plan = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream(self.device).cuda_stream
            _check(lib().nedner_plan_create(ctypes.byref(d), self.device.index,
                                            ctypes.c_void_p(stream), ctypes.byref(self._plan)))
        del keep
        info = info_struct()
        _check(lib().nedner_plan_info(self._plan, ctypes.byref(info)))
        self.info = {k: getattr(info, k) for k, _ in info_struct._fields_ if k != "pad0"}
        self._ws = None

    # -- plumbing ---------------------------------------------------------
    def _workspace(self):
        if self._ws is None:
            nbytes = int(self.info["workspace_bytes"])
            self._ws = self._torch.empty(max(nbytes, 256), dtype=self._torch.uint8,
                                         device=self.device)
            _check(lib().nedner_set_workspace(self._plan, ctypes.c_void_p(self._ws.data_ptr()),
                                              ctypes.c_size_t(self._ws.numel())))
        return self._ws

    def _stream(self):
        return ctypes.c_void_p(self._torch.cuda.current_stream(self.device).cuda_stream)

    def _check_in(self, t, shape, what):
        torch = self._torch
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{what} must be a torch tensor")
        if t.device != self.device:
            raise ValueError(f"{what} must be on {self.device}")
        if t.dtype != self.dtype:
            raise TypeError(f"{what} must be {self.dtype} for a {self.precision} plan")
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"{what} has shape {tuple(t.shape)}, expected {tuple(shape)}")
        return t.contiguous()

    @property
    def grid_shape(self):
        return (self.info["n1_os"], self.info["n2_os"], self.nt)

    # -- operator ---------------------------------------------------------
    def forward(self, g, kind="volume", out=None):
        """Data (M, Nt) -> volume (N1, N2, N3), spectrum (complex) or spread grid."""
        torch = self._torch
        g = self._check_in(g, (self.m, self.nt), "g")
        k = KINDS[kind]
        if k == 0:
            shape, dt = self.volume, self.dtype
        elif k == 1:
            shape, dt = (*self.volume, 2), self.dtype
        else:
            shape, dt = self.grid_shape, self.dtype
        if out is None:
            out = torch.empty(shape, dtype=dt, device=self.device)
        if k != 2:
            self._workspace()
        with torch.cuda.device(self.device):
            _check(lib().nedner_execute(self._plan, ctypes.c_void_p(g.data_ptr()),
                                        ctypes.c_void_p(out.data_ptr()), k, self._stream()))
        if k == 1:
            return torch.view_as_complex(out)
        return out

    __call__ = forward

    def spectrum(self, g):
        return self.forward(g, kind="spectrum")

    def grid(self, g):
        return self.forward(g, kind="grid")

    def adjoint(self, v, kind="volume", out=None):
        """Transpose: volume (N1, N2, N3) (or spread grid) -> data (M, Nt)."""
        torch = self._torch
        k = KINDS[kind]
        if k == 1:
            raise NednerError(6, "adjoint of the spectrum output is not provided")
        v = self._check_in(v, self.volume if k == 0 else self.grid_shape, "v")
        if out is None:
            out = torch.empty((self.m, self.nt), dtype=self.dtype, device=self.device)
        if k == 0:
            self._workspace()
        with torch.cuda.device(self.device):
            _check(lib().nedner_execute_adjoint(self._plan, ctypes.c_void_p(v.data_ptr()), k,
                                                ctypes.c_void_p(out.data_ptr()), self._stream()))
        return out

    # -- forward operator Q of the wave equation ---------------------------
    def q(self, v, out=None):
        """Forward operator Q: initial pressure (N1, N2, N3) -> the trace of the
        wave equation's solution at the sensors (M, Nt), on the periodic voxel
        grid (per mode cos(c|K|t)); no sensor or inversion weights."""
        torch = self._torch
        v = self._check_in(v, self.volume, "v")
        if out is None:
            out = torch.empty((self.m, self.nt), dtype=self.dtype, device=self.device)
        self._workspace()
        with torch.cuda.device(self.device):
            _check(lib().nedner_execute_q(self._plan, ctypes.c_void_p(v.data_ptr()),
                                          ctypes.c_void_p(out.data_ptr()), self._stream()))
        return out

    def q_adjoint(self, g, out=None):
        """Adjoint of `q` for the real inner products: data (M, Nt) -> volume."""
        torch = self._torch
        g = self._check_in(g, (self.m, self.nt), "g")
        if out is None:
            out = torch.empty(self.volume, dtype=self.dtype, device=self.device)
        self._workspace()
        with torch.cuda.device(self.device):
            _check(lib().nedner_execute_q_adjoint(self._plan, ctypes.c_void_p(g.data_ptr()),
                                                  ctypes.c_void_p(out.data_ptr()), self._stream()))
        return out

    # -- launch shape -------------------------------------------------------
    @property
    def tuning(self) -> dict:
        t = tuning_struct()
        _check(lib().nedner_get_tuning(self._plan, ctypes.byref(t)))
        return _tuning_dict(t)

    def set_tuning(self, tuning: dict):
        """Set the launch shape; fields missing from `tuning` keep their current values."""
        cur = self.tuning
        t = tuning_struct(**{k: tuning.get(k, cur.get(k, 0)) for k, _ in tuning_struct._fields_ if k != "pad1"})
        with self._torch.cuda.device(self.device):
            _check(lib().nedner_set_tuning(self._plan, ctypes.byref(t)))
        self._refresh_info()

    def _refresh_info(self):
        info = info_struct()
        _check(lib().nedner_plan_info(self._plan, ctypes.byref(info)))
        self.info = {k: getattr(info, k) for k, _ in info_struct._fields_ if k != "pad0"}

    def cache_key(self) -> str:
        arch = self._torch.cuda.get_device_properties(self.device).gcnArchName.split(":")[0]
        n1, n2, n3 = self.volume
        return (f"{arch}|{self.precision}|m{self.m}|nt{self.nt}|{n1}x{n2}x{n3}|w{self._w}|s{self._sigma}"
                f"|win{self._window}")

    def autotune(self, g=None, cache: str | None = None) -> dict:
        """Pick the fastest launch shape (sweep length, samples per lane, pass
        shape) by timing candidates on the GPU; results are cached in a JSON
        file keyed by device, precision and problem size (NEDNER_TUNING_CACHE
        or ~/.cache/nedner/tuning.json)."""
        import json
        path = cache or os.environ.get("NEDNER_TUNING_CACHE",
                                       os.path.join(os.path.expanduser("~"), ".cache", "nedner",
                                                    "tuning.json"))
        key = self.cache_key()
        table = {}
        if os.path.exists(path):
            try:
                with open(path) as fh:
                    table = json.load(fh)
            except (OSError, ValueError):
                table = {}
        if key in table:
            self.set_tuning(table[key])
            return table[key]
        torch = self._torch
        if g is None:
            g = torch.zeros((self.m, self.nt), dtype=self.dtype, device=self.device)
        g = self._check_in(g, (self.m, self.nt), "g")
        self._workspace()
        t = tuning_struct()
        with torch.cuda.device(self.device):
            _check(lib().nedner_autotune(self._plan, ctypes.c_void_p(g.data_ptr()), self._stream(),
                                         ctypes.byref(t)))
        self._refresh_info()
        res = _tuning_dict(t)
        table[key] = res
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            with open(path, "w") as fh:
                json.dump(table, fh, indent=1, sort_keys=True)
        except OSError:
            pass
        return res

    def close(self):
        if getattr(self, "_plan", None) is not None and self._plan.value:
            lib().nedner_destroy(self._plan)
            self._plan = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchPlan:
    """Many independent reconstructions run together: one persistent launch
    per pipeline stage for the whole batch (uneven sensor counts, lengths and
    grids are allowed; precision and window width are shared).

    `problems` is a sequence of dicts with the keyword arguments of Plan
    (xy, nt, dt, volume, and optionally c, h, t0, a1, a2, d1, d2, d3).
    """

    def __init__(self, problems, precision="fp32c", w=12, sigma=2.0, tau_scale=1.0, flags=0,
                 time_per_lane=0, window="gaussian", device=None):
        import torch
        self._torch = torch
        if not torch.cuda.is_available():
            raise NednerError(5, "no GPU: the NEDNER library runs on MI355X only")
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else int(device))
        descs = (desc_struct * len(problems))()
        keep = []
        self.shapes = []
        for i, pr in enumerate(problems):
            pr = dict(pr)
            n1, n2, n3 = (int(v) for v in pr.pop("volume"))
            d, k = _make_desc(pr.pop("xy"), pr.pop("h", None), pr.pop("nt"), pr.pop("dt"), n1, n2, n3,
                              precision=precision, w=w, sigma=sigma, tau_scale=tau_scale, flags=flags,
                              time_per_lane=time_per_lane, window=window, **pr)
            descs[i] = d
            keep.append(k)
            self.shapes.append(((int(d.m), int(d.nt)), (n1, n2, n3)))
        self.dtype = torch.float64 if precision == "fp64" else torch.float32
        self.precision = precision
        self._plan = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib().nedner_plan_create_many(descs, len(problems), self.device.index, None,
                                                 ctypes.byref(self._plan)))
        del keep
        info = info_struct()
        _check(lib().nedner_plan_info(self._plan, ctypes.byref(info)))
        self.workspace_bytes = int(info.workspace_bytes)
        self._ws = self._torch.empty(max(self.workspace_bytes, 256), dtype=torch.uint8,
                                     device=self.device)
        _check(lib().nedner_set_workspace(self._plan, ctypes.c_void_p(self._ws.data_ptr()),
                                          ctypes.c_size_t(self._ws.numel())))

    def forward(self, gs, outs=None):
        """Data tensors [(M_i, Nt_i)] -> volumes [(N1_i, N2_i, N3_i)]."""
        torch = self._torch
        if len(gs) != len(self.shapes):
            raise ValueError("one data tensor per problem")
        ins = []
        for g, (gshape, _) in zip(gs, self.shapes):
            if g.device != self.device or g.dtype != self.dtype or tuple(g.shape) != gshape:
                raise ValueError(f"data must be {self.dtype} {gshape} on {self.device}")
            ins.append(g.contiguous())
        if outs is None:
            outs = [torch.empty(vs, dtype=self.dtype, device=self.device) for _, vs in self.shapes]
        n = len(ins)
        gp = (ctypes.c_void_p * n)(*[t.data_ptr() for t in ins])
        op = (ctypes.c_void_p * n)(*[t.data_ptr() for t in outs])
        with torch.cuda.device(self.device):
            stream = ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)
            _check(lib().nedner_execute_many(self._plan, gp, op, KINDS["volume"], stream))
        return outs

    __call__ = forward

    def autotune(self) -> dict:
        """Choose every problem's spreading sweep length by timing it alone."""
        t = tuning_struct()
        with self._torch.cuda.device(self.device):
            stream = ctypes.c_void_p(self._torch.cuda.current_stream(self.device).cuda_stream)
            _check(lib().nedner_autotune(self._plan, None, stream, ctypes.byref(t)))
        return _tuning_dict(t)

    def close(self):
        if getattr(self, "_plan", None) is not None and self._plan.value:
            lib().nedner_destroy(self._plan)
            self._plan = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _autograd():
    import torch

    class _Recon(torch.autograd.Function):
        """f = A g (the reconstruction); backward applies the adjoint A*."""

        @staticmethod
        def forward(ctx, g, plan):
            ctx.plan = plan
            return plan.forward(g)

        @staticmethod
        def backward(ctx, grad):
            return ctx.plan.adjoint(grad.contiguous()), None

    class _Adjoint(torch.autograd.Function):
        """g = A* v; backward applies A."""

        @staticmethod
        def forward(ctx, v, plan):
            ctx.plan = plan
            return plan.adjoint(v)

        @staticmethod
        def backward(ctx, grad):
            return ctx.plan.forward(grad.contiguous()), None

    class _Q(torch.autograd.Function):
        """g = Q v (the wave equation's trace); backward applies Q*."""

        @staticmethod
        def forward(ctx, v, plan):
            ctx.plan = plan
            return plan.q(v)

        @staticmethod
        def backward(ctx, grad):
            return ctx.plan.q_adjoint(grad.contiguous()), None

    return _Recon, _Adjoint, _Q


class _Lazy:
    def __init__(self, idx):
        self._idx = idx
        self._fn = None

    def apply(self, *a):
        if self._fn is None:
            self._fn = _autograd()[self._idx]
        return self._fn.apply(*a)


NednerRecon = _Lazy(0)
NednerAdjoint = _Lazy(1)
NednerQ = _Lazy(2)


def power_norm(plan: Plan, iters: int = 10, seed: int = 0, model: str = "adjoint") -> float:
    """Estimate the squared norm of the least-squares operator by power
    iteration: ||A||^2 (largest eigenvalue of A A*) for model="adjoint",
    ||Q||^2 (largest eigenvalue of Q* Q) for model="q"."""
    torch = plan._torch
    gen = torch.Generator(device=plan.device).manual_seed(seed)
    v = torch.randn(plan.volume, dtype=plan.dtype, device=plan.device, generator=gen)
    lam = 0.0
    for _ in range(iters):
        v = v / torch.linalg.vector_norm(v)
        w = plan.forward(plan.adjoint(v)) if model == "adjoint" else plan.q_adjoint(plan.q(v))
        lam = float(torch.dot(v.reshape(-1), w.reshape(-1)))
        v = w
    return lam


def lsq(plan: Plan, g, iters: int = 20, eta: float | None = None, x0=None, callback=None,
        model: str = "adjoint", sync: bool = True):
    """Projected gradient descent on J(x) = 1/2 ||M x - g||^2 with x >= 0.

    M is the adjoint A* of the reconstruction (model="adjoint") or the forward
    operator Q of the wave equation (model="q"). The gradient M* (M x - g) is
    taken by autograd through NednerAdjoint or NednerQ, so each iteration runs
    the operator and its transpose once. Returns (x, losses): with sync the
    losses are floats read after every iteration (a host synchronisation each);
    without it, and without a callback, they stay 0-d device tensors until the
    caller reads them, so the iterations run back to back on the stream.
    """
    torch = plan._torch
    if model not in ("adjoint", "q"):
        raise ValueError("model must be 'adjoint' or 'q'")
    if eta is None:
        # a step just under 1/L (L = ||M||^2 estimated from below) keeps the
        # projected iteration monotone
        eta = 0.95 / max(power_norm(plan, iters=20, model=model), 1e-300)
    op = NednerAdjoint if model == "adjoint" else NednerQ
    x = torch.zeros(plan.volume, dtype=plan.dtype, device=plan.device) if x0 is None else x0.clone()
    losses = []
    for it in range(iters):
        x.requires_grad_(True)
        r = op.apply(x, plan) - g
        loss = 0.5 * torch.sum(r * r)
        (grad,) = torch.autograd.grad(loss, x)
        losses.append(float(loss.detach()) if (sync or callback is not None) else loss.detach())
        with torch.no_grad():
            x = torch.clamp(x - eta * grad, min=0.0)
        if callback is not None:
            callback(it, x, losses[-1])
    return x.detach(), losses


# ---------------------------------------------------------------- image measures

def _dtype_code(t):
    import torch
    if t.dtype == torch.float32:
        return 0
    if t.dtype == torch.float64:
        return 1
    raise ValueError("float32 or float64 tensors only")


def _metric_buffers(t):
    import torch
    work = torch.empty(int(lib().nedner_metrics_workspace_size()), dtype=torch.uint8, device=t.device)
    res = torch.empty(1, dtype=torch.float64, device=t.device)
    return work, res


def mip(vol, axis: int):
    """Maximum intensity projection of a device volume (N1, N2, N3) along `axis`."""
    import torch
    if vol.dim() != 3 or not vol.is_cuda:
        raise ValueError("a 3-D device tensor is expected")
    v = vol.contiguous()
    shape = [s for k, s in enumerate(v.shape) if k != axis]
    out = torch.empty(shape, dtype=v.dtype, device=v.device)
    with torch.cuda.device(v.device):
        _check(lib().nedner_mip(ctypes.c_void_p(v.data_ptr()), v.shape[0], v.shape[1], v.shape[2], int(axis),
                                _dtype_code(v), ctypes.c_void_p(out.data_ptr()),
                                ctypes.c_void_p(torch.cuda.current_stream(v.device).cuda_stream)))
    return out


def corrcoef(a, b, mask=None) -> float:
    """Correlation coefficient of two device arrays of equal shape (App. B,
    eq. (11)), over the elements where `mask` (bool tensor) is true."""
    import torch
    if a.shape != b.shape or a.dtype != b.dtype or not a.is_cuda:
        raise ValueError("two device tensors of one shape and dtype are expected")
    x, y = a.contiguous(), b.contiguous()
    m = None
    if mask is not None:
        if mask.shape != a.shape:
            raise ValueError("mask shape differs")
        m = mask.to(device=a.device, dtype=torch.uint8).contiguous()
    work, res = _metric_buffers(x)
    with torch.cuda.device(x.device):
        _check(lib().nedner_corrcoef(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                     ctypes.c_void_p(m.data_ptr() if m is not None else 0), x.numel(),
                                     _dtype_code(x), ctypes.c_void_p(res.data_ptr()),
                                     ctypes.c_void_p(work.data_ptr()), work.numel(),
                                     ctypes.c_void_p(torch.cuda.current_stream(x.device).cuda_stream)))
    return float(res.item())


def tenenbaum(img, rect=None, normalized=False) -> float:
    """Tenenbaum sharpness of a device image (rows, cols) (App. B, eqs. (12)-(13))
    over the pixels of rect = (r0, r1, c0, c1) with a full 3x3 neighbourhood;
    with normalized, the paper's F / N, N the element count of the rectangle
    (of the whole image without rect)."""
    import torch
    if img.dim() != 2 or not img.is_cuda:
        raise ValueError("a 2-D device tensor is expected")
    u = img.contiguous()
    rows, cols = u.shape
    r0, r1, c0, c1 = (0, rows, 0, cols) if rect is None else rect
    work, res = _metric_buffers(u)
    fn = lib().nedner_tenenbaum_mean if normalized else lib().nedner_tenenbaum
    with torch.cuda.device(u.device):
        _check(fn(ctypes.c_void_p(u.data_ptr()), rows, cols, r0, r1, c0, c1,
                  _dtype_code(u), ctypes.c_void_p(res.data_ptr()),
                  ctypes.c_void_p(work.data_ptr()), work.numel(),
                  ctypes.c_void_p(torch.cuda.current_stream(u.device).cuda_stream)))
    return float(res.item())
