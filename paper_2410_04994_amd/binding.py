"""ctypes binding of the C ABI in include/shg.h.

Argument marshalling only: every step of the march runs in the HIP library.
Tensors are torch CUDA (HIP) tensors; the binding passes their device pointers
and the current stream.  There is no CPU fallback: if libshg.so is missing or
a tensor is not on the GPU the call raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libshg.so")

SHG_C64, SHG_C128 = 0, 1
SHG_OK, SHG_EINVAL, SHG_EUNSUPPORTED, SHG_ENOMEM, SHG_EDEVICE, SHG_ENONFINITE, SHG_ESTATE = range(7)
SHG_UNDEPLETED = 1 << 0
SHG_NO_GRAPH = 1 << 1
SHG_SPLIT_LNL = 1 << 2
SHG_CHECK_FINITE = 1 << 3
ERROR_NAMES = {0: "SHG_OK", 1: "SHG_EINVAL", 2: "SHG_EUNSUPPORTED", 3: "SHG_ENOMEM",
               4: "SHG_EDEVICE", 5: "SHG_ENONFINITE", 6: "SHG_ESTATE"}


class ShgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


class ShgParams(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("lx", ctypes.c_double), ("ly", ctypes.c_double), ("lcr", ctypes.c_double),
                ("lambda_f", ctypes.c_double), ("n_f", ctypes.c_double), ("n_sh", ctypes.c_double),
                ("d_eff", ctypes.c_double), ("alpha_f", ctypes.c_double),
                ("alpha_sh", ctypes.c_double), ("beta_f", ctypes.c_double),
                ("beta_sh", ctypes.c_double), ("dk0", ctypes.c_double), ("ddk_dT", ctypes.c_double),
                ("dn_dT", ctypes.c_double), ("t_ref", ctypes.c_double), ("flags", ctypes.c_uint32),
                ("checkpoint_every", ctypes.c_int32), ("walkoff_f", ctypes.c_double),
                ("walkoff_sh", ctypes.c_double), ("ddk_dT2", ctypes.c_double),
                ("ddk_dT3", ctypes.c_double), ("grating_period", ctypes.c_double),
                ("grating_a", ctypes.c_double), ("grating_b", ctypes.c_double)]


SHG_FACE_AIR, SHG_FACE_OVEN, SHG_FACE_INSULATED = 0, 1, 2
FACE_NAMES = ("x-", "x+", "y-", "y+", "z-", "z+")
FACE_KINDS = {"air": SHG_FACE_AIR, "oven": SHG_FACE_OVEN, "insulated": SHG_FACE_INSULATED}


class ThermalParams(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("faces", ctypes.c_int32 * 6), ("method", ctypes.c_int32),
                ("lx", ctypes.c_double), ("ly", ctypes.c_double), ("lcr", ctypes.c_double),
                ("k_th", ctypes.c_double), ("h_conv", ctypes.c_double), ("t_inf", ctypes.c_double),
                ("t_oven", ctypes.c_double)]


_VP = ctypes.c_void_p
_I32 = ctypes.c_int32
_F64 = ctypes.c_double
_SIGS = {
    "shg_plan_create": (ctypes.c_int, [ctypes.POINTER(_VP), ctypes.POINTER(ShgParams), ctypes.c_int]),
    "shg_plan_destroy": (ctypes.c_int, [_VP]),
    "shg_workspace_bytes": (ctypes.c_size_t, [_VP, ctypes.c_int]),
    "shg_propagate": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, _I32, _I32, _VP, _VP, _VP]),
    "shg_propagate_noalloc": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, _I32, _I32, _VP, _VP]),
    "shg_propagate_heat": (ctypes.c_int, [_VP] * 9),
    "shg_propagate_adjoint": (ctypes.c_int, [_VP] * 16 + [_VP]),
    "shg_propagate_batch": (ctypes.c_int, [_I32, _VP, _VP, _VP, _VP, _VP, _VP, _VP]),
    "shg_batch_workspace_bytes": (ctypes.c_size_t, [_I32, _VP]),
    "shg_plan_set_schedule": (ctypes.c_int, [_VP, _I32, _I32, _I32, _I32]),
    "shg_plan_describe": (ctypes.c_int, [_VP, ctypes.c_char_p, ctypes.c_size_t]),
    "shg_plan_set_timing": (ctypes.c_int, [_VP, _I32]),
    "shg_plan_set_batch_schedule": (ctypes.c_int, [_VP, _I32, _I32, _I32, _I32]),
    "shg_plan_kernel_times": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_double)]),
    "shg_last_error": (ctypes.c_char_p, []),
    "shg_thermal_create": (ctypes.c_int, [ctypes.POINTER(_VP), ctypes.POINTER(ThermalParams),
                                          ctypes.c_int]),
    "shg_thermal_destroy": (ctypes.c_int, [_VP]),
    "shg_thermal_workspace_bytes": (ctypes.c_size_t, [_VP]),
    "shg_thermal_solve": (ctypes.c_int, [_VP, _VP, _VP, _VP, _F64, _I32, _VP,
                                         ctypes.POINTER(_I32), ctypes.POINTER(_F64), _VP]),
    "shg_self_consistent": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _F64, _I32,
                                           _F64, _I32, _VP, ctypes.POINTER(_I32),
                                           ctypes.POINTER(_F64), _VP]),
}

_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libshg.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library {path} is missing: run `python -m paper_2410_04994_amd.build`")
    # torch ships its own HIP runtime; loading it first makes libshg bind to
    # that same runtime (one runtime per process, shared streams and memory)
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(code: int):
    if code != SHG_OK:
        raise ShgError(code, load_library().shg_last_error().decode())


def _torch():
    import torch
    return torch


def _ptr(t, what: str, dtype=None, numel: Optional[int] = None, nbytes: Optional[int] = None):
    """Device pointer of a contiguous CUDA tensor (None -> NULL).  The kernels
    read and write numel elements (or nbytes bytes) through it, so a smaller
    tensor is refused here."""
    if t is None:
        return None
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{what} must be a CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{what} must have dtype {dtype}, got {t.dtype}")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{what} holds {t.numel()} elements, needs {numel}")
    if nbytes is not None and t.numel() * t.element_size() < nbytes:
        raise ValueError(f"{what} holds {t.numel() * t.element_size()} bytes, needs {nbytes}")
    return t.data_ptr()


def _stream(stream=None):
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


PARAM_KEYS = ("nx", "ny", "nz", "lx", "ly", "lcr", "lambda_f", "n_f", "n_sh", "d_eff", "alpha_f",
              "alpha_sh", "beta_f", "beta_sh", "dk0", "ddk_dT", "dn_dT", "t_ref", "walkoff_f",
              "walkoff_sh", "ddk_dT2", "ddk_dT3", "grating_period", "grating_a", "grating_b")


def make_params(params: dict, flags: int = 0, checkpoint_every: int = 0) -> ShgParams:
    p = ShgParams()
    for k in PARAM_KEYS:
        setattr(p, k, params.get(k, 0.0) if k not in ("nx", "ny", "nz") else int(params[k]))
    f = flags
    if params.get("undepleted"):
        f |= SHG_UNDEPLETED
    split = params.get("split", "NLN")
    if split not in ("NLN", "LNL"):
        raise ValueError(f"unknown split order {split!r}")
    if split == "LNL":
        f |= SHG_SPLIT_LNL
    p.flags = f
    p.checkpoint_every = int(checkpoint_every)
    return p


class Plan:
    """Owns an shg_plan.  `params` uses the keys of workloads.Workload.params()."""

    def __init__(self, params: dict, dtype: str = "c64", flags: int = 0, checkpoint_every: int = 0):
        lib = load_library()
        self.params = dict(params)
        self.dtype = dtype
        self._cp = make_params(params, flags, checkpoint_every)
        h = _VP()
        _check(lib.shg_plan_create(ctypes.byref(h), ctypes.byref(self._cp),
                                   SHG_C64 if dtype == "c64" else SHG_C128))
        self.handle = h
        self._ws = {}

    # ------------------------------------------------------------------ helpers
    @property
    def complex_dtype(self):
        torch = _torch()
        return torch.complex64 if self.dtype == "c64" else torch.complex128

    @property
    def real_dtype(self):
        torch = _torch()
        return torch.float32 if self.dtype == "c64" else torch.float64

    def workspace_bytes(self, adjoint: bool = False) -> int:
        return int(load_library().shg_workspace_bytes(self.handle, 1 if adjoint else 0))

    def workspace(self, adjoint: bool = False, device=None):
        """A cached uint8 device buffer of workspace_bytes(adjoint) bytes."""
        torch = _torch()
        n = self.workspace_bytes(adjoint)
        buf = self._ws.get(adjoint)
        if buf is None or buf.numel() < n:
            buf = torch.empty(max(n, 1), dtype=torch.uint8, device=device or "cuda")
            self._ws[adjoint] = buf
        return buf

    def set_schedule(self, row_e=0, row_wg=0, col_e=0, col_tc=0):
        _check(load_library().shg_plan_set_schedule(self.handle, row_e, row_wg, col_e, col_tc))

    def set_batch_schedule(self, row_e=0, row_wg=0, col_e=0, col_tc=0):
        _check(load_library().shg_plan_set_batch_schedule(self.handle, row_e, row_wg, col_e, col_tc))

    def set_timing(self, enable: bool):
        _check(load_library().shg_plan_set_timing(self.handle, 1 if enable else 0))

    def kernel_times(self) -> dict:
        """Per-kernel event timings since the last query (timing mode only)."""
        out = (ctypes.c_double * 4)()
        _check(load_library().shg_plan_kernel_times(self.handle, out))
        return {"row_ms": out[0], "row_n": int(out[1]), "col_ms": out[2], "col_n": int(out[3])}

    def describe(self) -> str:
        buf = ctypes.create_string_buffer(256)
        _check(load_library().shg_plan_describe(self.handle, buf, 256))
        return buf.value.decode()

    @property
    def cells(self) -> int:
        return int(self.params["nx"]) * int(self.params["ny"])

    @property
    def nz(self) -> int:
        return int(self.params["nz"])

    def _field(self, t, what):
        return _ptr(t, what, self.complex_dtype, numel=self.cells)

    def _dk(self, t):
        return _ptr(t, "dk_z", _torch().float64, numel=self.nz)

    def _temp(self, t):
        return _ptr(t, "temp", self.real_dtype, numel=self.nz * self.cells)

    def _ws_ptr(self, t, adjoint: bool):
        return _ptr(t, "workspace", nbytes=self.workspace_bytes(adjoint) if t is not None else None)

    # ------------------------------------------------------------------ calls
    def propagate(self, a_f, a_sh, dk_z=None, temp=None, s_begin: int = 0, s_end: Optional[int] = None,
                  workspace=None, powers=None, stream=None):
        """March [s_begin, s_end) in place; returns the device double[2] powers."""
        torch = _torch()
        if s_end is None:
            s_end = self.params["nz"]
        if powers is None:
            powers = torch.empty(2, dtype=torch.float64, device=a_f.device)
        _check(load_library().shg_propagate(
            self.handle, self._field(a_f, "a_f"), self._field(a_sh, "a_sh"),
            self._dk(dk_z), self._temp(temp), int(s_begin), int(s_end),
            self._ws_ptr(workspace, False), _ptr(powers, "powers", torch.float64, numel=2),
            _stream(stream)))
        return powers

    def propagate_noalloc(self, a_f, a_sh, powers, dk_z=None, temp=None, s_begin: int = 0,
                          s_end: Optional[int] = None, stream=None):
        """shg_propagate_noalloc: the march of `propagate` with the library's
        static per-GPU workspace; the call allocates nothing (powers is a
        caller-owned device double[2]).  Overlapping calls on one GPU race."""
        torch = _torch()
        if s_end is None:
            s_end = self.params["nz"]
        _check(load_library().shg_propagate_noalloc(
            self.handle, self._field(a_f, "a_f"), self._field(a_sh, "a_sh"),
            self._dk(dk_z), self._temp(temp), int(s_begin), int(s_end),
            _ptr(powers, "powers", torch.float64, numel=2), _stream(stream)))
        return powers

    def propagate_heat(self, a_f, a_sh, dk_z=None, temp=None, heat=None, workspace=None,
                       powers=None, stream=None):
        """Whole march in place, also writing the heat source at the nz + 1 step
        boundaries.  Returns (heat [nz+1, ny, nx], powers)."""
        torch = _torch()
        p = self.params
        if heat is None:
            heat = torch.empty((p["nz"] + 1, p["ny"], p["nx"]), dtype=self.real_dtype,
                               device=a_f.device)
        if powers is None:
            powers = torch.empty(2, dtype=torch.float64, device=a_f.device)
        _check(load_library().shg_propagate_heat(
            self.handle, self._field(a_f, "a_f"), self._field(a_sh, "a_sh"),
            self._dk(dk_z), self._temp(temp),
            _ptr(heat, "heat", self.real_dtype, numel=(self.nz + 1) * self.cells),
            self._ws_ptr(workspace, False), _ptr(powers, "powers", torch.float64, numel=2),
            _stream(stream)))
        return heat, powers

    def adjoint(self, a_f_in, a_sh_in, g_f_out=None, g_sh_out=None, power_weights=None, dk_z=None,
                temp=None, want_dk=False, want_t=False, workspace=None, stream=None, out=None):
        """Forward + reverse march.  Returns a dict with g_f, g_sh (gradients at
        z = 0), a_f, a_sh (exit fields), powers, and g_dk / g_t_moments if asked.
        out: optional dict of preallocated outputs under the same keys."""
        torch = _torch()
        dev = a_f_in.device
        out = out or {}
        g_f = out.get("g_f", None)
        g_f = torch.empty_like(a_f_in) if g_f is None else g_f
        g_sh = out.get("g_sh", None)
        g_sh = torch.empty_like(a_sh_in) if g_sh is None else g_sh
        a_f = out.get("a_f", None)
        a_f = torch.empty_like(a_f_in) if a_f is None else a_f
        a_sh = out.get("a_sh", None)
        a_sh = torch.empty_like(a_sh_in) if a_sh is None else a_sh
        powers = out.get("powers", None)
        powers = torch.empty(2, dtype=torch.float64, device=dev) if powers is None else powers
        g_dk = out.get("g_dk", None)
        if want_dk and g_dk is None:
            g_dk = torch.empty(self.params["nz"], dtype=torch.float64, device=dev)
        g_t = out.get("g_t_moments", None)
        if want_t and g_t is None:
            g_t = torch.empty(2, dtype=torch.float64, device=dev)
        if not want_dk:
            g_dk = None
        if not want_t:
            g_t = None
        if workspace is None:
            workspace = self.workspace(adjoint=True, device=dev)
        _check(load_library().shg_propagate_adjoint(
            self.handle, self._field(a_f_in, "a_f_in"), self._field(a_sh_in, "a_sh_in"),
            self._dk(dk_z), self._temp(temp),
            self._field(g_f_out, "g_f_out"), self._field(g_sh_out, "g_sh_out"),
            _ptr(power_weights, "power_weights", torch.float64, numel=2),
            self._field(g_f, "g_f_in"), self._field(g_sh, "g_sh_in"),
            _ptr(g_dk, "g_dk_z", torch.float64, numel=self.nz),
            _ptr(g_t, "g_t_moments", torch.float64, numel=2),
            self._field(a_f, "a_f_out"), self._field(a_sh, "a_sh_out"),
            _ptr(powers, "powers", torch.float64, numel=2), self._ws_ptr(workspace, True),
            _stream(stream)))
        out = {"g_f": g_f, "g_sh": g_sh, "a_f": a_f, "a_sh": a_sh, "powers": powers}
        if want_dk:
            out["g_dk"] = g_dk
        if want_t:
            out["g_t_moments"] = g_t
        return out

    def close(self):
        if getattr(self, "handle", None):
            load_library().shg_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_workspace_bytes(plans: Sequence[Plan]) -> int:
    arr = (_VP * len(plans))(*[p.handle for p in plans])
    return int(load_library().shg_batch_workspace_bytes(len(plans), arr))


def propagate_batch(plans: Sequence[Plan], a_f: Sequence, a_sh: Sequence, dk_z: Optional[Sequence] = None,
                    workspace=None, powers=None, stream=None):
    """March every instance over its whole crystal; returns [n, 2] powers."""
    torch = _torch()
    n = len(plans)
    if powers is None and n > 0:
        powers = torch.empty((n, 2), dtype=torch.float64, device=a_f[0].device)
    hp = (_VP * n)(*[p.handle for p in plans])
    fa = (_VP * n)(*[p._field(t, "a_f[i]") for p, t in zip(plans, a_f)])
    fs = (_VP * n)(*[p._field(t, "a_sh[i]") for p, t in zip(plans, a_sh)])
    dk = None
    if dk_z is not None:
        dk = (_VP * n)(*[p._dk(d) for p, d in zip(plans, dk_z)])
    ws = None
    if workspace is not None:
        ws = _ptr(workspace, "workspace", nbytes=batch_workspace_bytes(plans))
    _check(load_library().shg_propagate_batch(n, hp, fa, fs, dk, ws,
                                              _ptr(powers, "powers", torch.float64, numel=2 * n),
                                              _stream(stream)))
    return powers


THERMAL_METHODS = {"direct": 0, "cg": 1}


def make_thermal_params(params: dict, k_th: float, h_conv: float, t_inf: float, t_oven: float,
                        faces: dict, method: str = "direct") -> ThermalParams:
    """faces: face name ("x-" .. "z+") -> "oven" | "air" | "insulated" (default air);
    method: "direct" (exact: x-y diagonalisation, tridiagonal solves along z) or "cg"."""
    tp = ThermalParams()
    tp.nx, tp.ny, tp.nz = int(params["nx"]), int(params["ny"]), int(params["nz"])
    for i, f in enumerate(FACE_NAMES):
        tp.faces[i] = FACE_KINDS[faces.get(f, "air")]
    tp.method = THERMAL_METHODS[method]
    tp.lx, tp.ly, tp.lcr = params["lx"], params["ly"], params["lcr"]
    tp.k_th, tp.h_conv, tp.t_inf, tp.t_oven = k_th, h_conv, t_inf, t_oven
    return tp


class Thermal:
    """Owns an shg_thermal: the heat-equation solver on the nodes of a field grid."""

    def __init__(self, params: dict, k_th: float, h_conv: float, t_inf: float, t_oven: float,
                 faces: dict, dtype: str = "c64", method: str = "direct"):
        lib = load_library()
        self.params = dict(params)
        self.dtype = dtype
        self.method = method
        self.t_oven = t_oven
        self._cp = make_thermal_params(params, k_th, h_conv, t_inf, t_oven, faces, method)
        h = _VP()
        _check(lib.shg_thermal_create(ctypes.byref(h), ctypes.byref(self._cp),
                                      SHG_C64 if dtype == "c64" else SHG_C128))
        self.handle = h
        self._ws = None

    @property
    def real_dtype(self):
        torch = _torch()
        return torch.float32 if self.dtype == "c64" else torch.float64

    @property
    def node_shape(self):
        return (self.params["nz"] + 1, self.params["ny"], self.params["nx"])

    def workspace_bytes(self) -> int:
        return int(load_library().shg_thermal_workspace_bytes(self.handle))

    def workspace(self, device=None):
        torch = _torch()
        n = self.workspace_bytes()
        if self._ws is None or self._ws.numel() < n:
            self._ws = torch.empty(n, dtype=torch.uint8, device=device or "cuda")
        return self._ws

    def solve(self, heat, t_nodes=None, t_mid=None, tol: float = 1e-6, max_iter: int = 20000,
              workspace=None, stream=None):
        """Solve k lap T + heat = 0.  t_nodes is the warm start (default T_oven
        everywhere) and receives T.  Returns (t_nodes, t_mid, iterations, residual)."""
        torch = _torch()
        dev = heat.device
        if t_nodes is None:
            t_nodes = torch.full(self.node_shape, self.t_oven, dtype=self.real_dtype, device=dev)
        if t_mid is None:
            n = self.node_shape
            t_mid = torch.empty((n[0] - 1, n[1], n[2]), dtype=self.real_dtype, device=dev)
        it = _I32()
        res = _F64()
        nodes = self.node_shape[0] * self.node_shape[1] * self.node_shape[2]
        mids = nodes - self.node_shape[1] * self.node_shape[2]
        _check(load_library().shg_thermal_solve(
            self.handle, _ptr(heat, "heat", self.real_dtype, numel=nodes),
            _ptr(t_nodes, "t_nodes", self.real_dtype, numel=nodes),
            _ptr(t_mid, "t_mid", self.real_dtype, numel=mids), float(tol), int(max_iter),
            _ptr(workspace if workspace is not None else self.workspace(dev), "workspace",
                 nbytes=self.workspace_bytes()),
            ctypes.byref(it), ctypes.byref(res), _stream(stream)))
        return t_nodes, t_mid, int(it.value), float(res.value)

    def close(self):
        if getattr(self, "handle", None):
            load_library().shg_thermal_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def self_consistent(plan: Plan, thermal: Thermal, a_f0, a_sh0, dk_z=None, t_nodes=None,
                    tol_t: float = 1e-4, max_outer: int = 30, solve_tol: float = 1e-6,
                    max_iter: int = 20000, workspace=None, stream=None):
    """The self-consistent field <-> temperature loop.  Returns a dict with the
    fields of the last march, t_nodes, t_mid, the number of marches and the last
    largest change of T."""
    torch = _torch()
    dev = a_f0.device
    a_f = torch.empty_like(a_f0)
    a_sh = torch.empty_like(a_sh0)
    if t_nodes is None:
        t_nodes = torch.full(thermal.node_shape, thermal.t_oven, dtype=thermal.real_dtype, device=dev)
    n = thermal.node_shape
    t_mid = torch.empty((n[0] - 1, n[1], n[2]), dtype=thermal.real_dtype, device=dev)
    outer = _I32()
    change = _F64()
    nodes = n[0] * n[1] * n[2]
    _check(load_library().shg_self_consistent(
        plan.handle, thermal.handle, plan._field(a_f0, "a_f0"), plan._field(a_sh0, "a_sh0"),
        plan._dk(dk_z), plan._field(a_f, "a_f"), plan._field(a_sh, "a_sh"),
        _ptr(t_nodes, "t_nodes", thermal.real_dtype, numel=nodes),
        _ptr(t_mid, "t_mid", thermal.real_dtype, numel=nodes - n[1] * n[2]),
        float(tol_t), int(max_outer), float(solve_tol), int(max_iter),
        _ptr(workspace if workspace is not None else thermal.workspace(dev), "workspace",
             nbytes=thermal.workspace_bytes()),
        ctypes.byref(outer), ctypes.byref(change), _stream(stream)))
    return {"a_f": a_f, "a_sh": a_sh, "t_nodes": t_nodes, "t_mid": t_mid,
            "outer": int(outer.value), "change": float(change.value)}
