"""Python binding of libfe (the C ABI in include/fe.h): argument marshalling only.

Every step of the expansion runs in the HIP library. PyTorch provides device memory and the
current HIP stream; no computation of the method happens here. If the library has not been
built (``python -m paper_2605_08523_amd.build``) every call raises: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import threading
from dataclasses import dataclass

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libfe.so")

FE_OK = 0
FE_WARN_BETA_CLAMPED = 1
FE_ERR_ARG = -1
FE_ERR_DOMAIN = -2
FE_ERR_HIP = -3
FE_ERR_NONFINITE = -4
FE_ERR_NO_CONVERGENCE = -5
FE_ERR_WORKSPACE = -6
FE_ERR_RANGE = -7

PREC = {"fp64": 0, "fp32": 1, "fp16x2": 2, "bf16x2": 3, "bf16x3": 4}


class FeError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libfe error {code}: {msg}")
        self.code = code


class fe_model(C.Structure):
    _fields_ = [("L", C.c_int32), ("beta0", C.c_double), ("mu0", C.c_double),
                ("theta", C.POINTER(C.c_double))]


class fe_qmodel(C.Structure):
    _fields_ = [("arch", C.c_int32), ("L", C.c_int32), ("k", C.c_int32), ("K", C.c_int32),
                ("beta0", C.c_double), ("mu0", C.c_double), ("coef", C.POINTER(C.c_double))]


class fe_rescale_info(C.Structure):
    _fields_ = [("emin", C.c_double), ("emax", C.c_double), ("mu_p", C.c_double),
                ("beta_p", C.c_double), ("beta_max", C.c_double), ("scale", C.c_double),
                ("shift", C.c_double), ("flipped", C.c_int32), ("clamped", C.c_int32),
                ("degenerate", C.c_int32), ("status", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_P = C.c_void_p
_D = C.c_double
_I32 = C.c_int32
_I64 = C.c_int64

# name -> (restype, argtypes); every symbol declared in include/fe.h
SIGNATURES = {
    "fe_workspace_create": (_I32, [_I64, _I32, _I64, C.POINTER(_P)]),
    "fe_workspace_destroy": (_I32, [_P]),
    "fe_rescale": (_I32, [_P, _I64, _I64, _D, _D, C.POINTER(fe_model), _P, _I64,
                          C.POINTER(fe_rescale_info), _P, _P]),
    "fe_expand_density": (_I32, [_P, _I64, _I64, _D, _D, C.POINTER(fe_model), _I32, _I32, _P, _I32,
                                 _I64, _P, _P, C.POINTER(fe_rescale_info), _P, _P]),
    "fe_expand_density_filling": (_I32, [_P, _I64, _I64, _D, _D, _D, C.POINTER(fe_model), _I32, _D,
                                         _I32, _P, _I32, _I64, _P, _P, C.POINTER(_D),
                                         C.POINTER(_I32), C.POINTER(fe_rescale_info), _P, _P]),
    "fe_observable": (_I32, [_P, _I32, _I64, _P, _I64, _I64, _P, _P, _P]),
    "fe_model_select": (_I32, [_P, _I64, _I64, _D, _D, C.POINTER(fe_model), _I32, C.POINTER(_I32),
                               _P, _P]),
    "fe_free_energy": (_I32, [_P, _I64, _I64, _D, _D, C.POINTER(fe_model), C.POINTER(fe_model), _D,
                              _I32, _P, _I32, _I64, _P, _P, _P, C.POINTER(fe_rescale_info), _P, _P]),
    "fe_expand_entropy": (_I32, [_P, _I64, _I64, _D, _D, C.POINTER(fe_model), _D, _I32, _P,
                                 C.POINTER(fe_rescale_info), _P, _P]),
    "fe_sp2_coeffs": (_I32, [_D, _I32, C.POINTER(_D)]),
    "fe_train_coeffs": (_I32, [_P, _P, _P, _P, _P, _P]),
    "fe_scalar_eval": (_I32, [_P, _I32, _P, _I32, _I32, _D, _D, _P, _P, _P, _P]),
    "fe_scalar_second": (_I32, [_P, _I32, _P, _I32, _I32, _D, _D, _P, _P, _P]),
    "fe_matrix_forward": (_I32, [_P, _I64, _P, _I32, _P, _P]),
    "fe_matrix_backward": (_I32, [_P, _I64, _P, _I32, _P, _P, _P, _I32, _P, _P]),
    "fe_layer_count": (_D, [_D]),
    "fe_batch_plan_retile": (_I32, [_P, _I32]),
    "fe_batch_plan_set_launch": (_I32, [_P, _I32]),
    "fe_batch_plan_get": (_I32, [_P, C.POINTER(_I32), C.POINTER(_I32)]),
    "fe_batch_plan_autotune": (_I32, [_P, _P, C.POINTER(_I32), C.POINTER(_D)]),
    "fe_autotune": (_I32, [C.POINTER(_I64), _I32, _I32, C.POINTER(_I32), C.POINTER(_D), _P, _P]),
    "fe_autotune_input": (_I32, [_P, _I64, _I64, _D, _D, C.POINTER(fe_model), _I32, C.POINTER(_I32),
                                 C.POINTER(_D), _P, _P]),
    "fe_autotune_lookup": (_I32, [_I64, _I32, _P, C.POINTER(_I32)]),
    "fe_autotune_clear": (_I32, []),
    "fe_qmodel_coef_count": (_I32, [_I32, _I32, _I32, _I32, C.POINTER(_I64)]),
    "fe_variant_scratch_bytes": (_I32, [_I64, C.POINTER(fe_qmodel), C.POINTER(_I64)]),
    "fe_expand_density_variant": (_I32, [_P, _I64, _I64, _D, _D, C.POINTER(fe_qmodel), _I32, _P,
                                         _I64, _P, _I32, _I64, _P, _P, C.POINTER(fe_rescale_info),
                                         _P, _P]),
    "fe_embed_mlsp2": (_I32, [C.POINTER(fe_model), _I32, C.POINTER(_D)]),
    "fe_variant_eval": (_I32, [_P, _I32, C.POINTER(fe_qmodel), _P, _P, _P, _P, _P]),
    "fe_train_variant": (_I32, [_P, C.POINTER(fe_qmodel), C.POINTER(_D), _P, _P]),
    "fe_expand_density_noalloc": (_I32, [_P, _I64, _I64, _D, _D, C.POINTER(fe_model), _I32, _I32,
                                         _P, _I32, _I64, _P, _P, C.POINTER(fe_rescale_info), _P]),
    "fe_streamk_segments": (_I32, [_I64, _I32, _I32, _I32, C.POINTER(_I32), C.POINTER(_I32), _I32,
                                   C.POINTER(_I32)]),
    "fe_debug_streamk_giveup": (_I32, [_I32]),
    "fe_debug_batch_queue_giveup": (_I32, [_I32]),
    "fe_batch_queue_layout": (_I32, [_I32, C.POINTER(_I64), C.POINTER(_I32), _I32, _I32,
                                     C.POINTER(_I32), _I64, C.POINTER(_I32), C.POINTER(_I64)]),
    "fe_debug_layer_events": (_I32, [_I32]),
    "fe_debug_layer_events_read": (_I32, [C.POINTER(_D), _I32, C.POINTER(_I32)]),
    "fe_last_error": (C.c_char_p, []),
    "fe_version": (C.c_char_p, []),
}

_lib = None
_lock = threading.Lock()


def lib():
    """Load libfe.so from the package directory (raises if it is missing)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                                   "`python -m paper_2605_08523_amd.build`")
            L = C.CDLL(LIB_PATH)
            for name, (res, args) in SIGNATURES.items():
                f = getattr(L, name)
                f.restype = res
                f.argtypes = args
            _lib = L
    return _lib


def _check(rc: int) -> int:
    if rc < 0:
        raise FeError(rc, lib().fe_last_error().decode())
    return rc


@dataclass
class _ModelRef:
    """Keeps the ctypes struct and its coefficient buffer alive together."""
    struct: fe_model
    theta: np.ndarray


def make_model(theta, beta0: float, mu0: float) -> _ModelRef:
    th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64).reshape(-1, 4))
    m = fe_model(th.shape[0], float(beta0), float(mu0), th.ctypes.data_as(C.POINTER(C.c_double)))
    return _ModelRef(m, th)


def _model_of(model) -> _ModelRef:
    if isinstance(model, _ModelRef):
        return model
    return make_model(model.theta, model.beta0, model.mu0)


def _stream_ptr():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check_H(H):
    import torch
    if not isinstance(H, torch.Tensor) or H.device.type != "cuda" or H.dtype != torch.float64:
        raise TypeError("H must be a float64 tensor on a HIP device")
    if H.dim() != 2 or H.shape[0] != H.shape[1]:
        raise ValueError("H must be square")
    if H.stride(1) != 1:
        raise ValueError("H must be row-major (unit column stride)")
    return H.shape[0], H.stride(0)


class Workspace:
    """Device scratch of the library (fe_workspace_create); sized for matrices up to max_n."""

    def __init__(self, max_n: int, max_batch: int = 0, batch_elems: int = 0):
        p = C.c_void_p()
        _check(lib().fe_workspace_create(int(max_n), int(max_batch), int(batch_elems), C.byref(p)))
        self._p = p
        self.max_n = int(max_n)

    @property
    def handle(self):
        return self._p

    def close(self):
        if self._p:
            lib().fe_workspace_destroy(self._p)
            self._p = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_ws_cache: dict = {}


def workspace(n: int) -> Workspace:
    """A cached workspace large enough for n (grown on demand, per device)."""
    import torch
    dev = torch.cuda.current_device()
    ws = _ws_cache.get(dev)
    if ws is None or ws.max_n < n:
        if ws is not None:
            torch.cuda.synchronize()
            ws.close()
        ws = Workspace(max(n, 128))
        _ws_cache[dev] = ws
    return ws


def rescale(H, mu: float, kT: float, model, want_X0: bool = True, ws: Workspace | None = None):
    """fe_rescale: returns (X0 float32 tensor or None, info dict). Synchronizes."""
    import torch
    n, ldh = _check_H(H)
    ws = ws or workspace(n)
    mr = _model_of(model)
    X0 = torch.empty((n, n), dtype=torch.float32, device=H.device) if want_X0 else None
    info = fe_rescale_info()
    rc = _check(lib().fe_rescale(C.c_void_p(H.data_ptr()), n, ldh, float(mu), float(kT),
                                 C.byref(mr.struct), C.c_void_p(X0.data_ptr() if want_X0 else 0),
                                 n, C.byref(info), ws.handle, _stream_ptr()))
    d = info.as_dict()
    d["rc"] = rc
    return X0, d


def expand_density(H, mu: float, kT: float, model, prec: str = "fp16x2", out=None,
                   out_dtype=None, want_info: bool = False, traces: bool = True,
                   ws: Workspace | None = None, final_correction: bool = False):
    """fe_expand_density. Returns (D, trD, trD2, info): D a tensor (float32 unless out_dtype or
    ``out`` says float64), trD/trD2 0-d float64 device tensors (or None), info a dict or None.
    Asynchronous on the current stream unless want_info."""
    import torch
    n, ldh = _check_H(H)
    ws = ws or workspace(n)
    mr = _model_of(model)
    if out is None:
        out = torch.empty((n, n), dtype=out_dtype or torch.float32, device=H.device)
    if out.dtype not in (torch.float32, torch.float64) or out.stride(1) != 1:
        raise TypeError("out must be a row-major float32/float64 device tensor")
    tr = torch.empty(2, dtype=torch.float64, device=H.device) if traces else None
    info = fe_rescale_info() if want_info else None
    rc = _check(lib().fe_expand_density(
        C.c_void_p(H.data_ptr()), n, ldh, float(mu), float(kT), C.byref(mr.struct), PREC[prec],
        int(bool(final_correction)), C.c_void_p(out.data_ptr()), int(out.dtype == torch.float64),
        out.stride(0),
        C.c_void_p(tr.data_ptr() if traces else 0),
        C.c_void_p(tr.data_ptr() + 8 if traces else 0),
        C.byref(info) if want_info else None, ws.handle, _stream_ptr()))
    d = None
    if want_info:
        d = info.as_dict()
        d["rc"] = rc
    return out, (tr[0] if traces else None), (tr[1] if traces else None), d


def expand_density_noalloc(H, mu: float, kT: float, model, prec: str = "fp16x2", out=None,
                           out_dtype=None, want_info: bool = False, final_correction: bool = False):
    """fe_expand_density_noalloc (no workspace; the library's static scratch). Returns
    (D, trD, trD2, info) as expand_density."""
    import torch
    n, ldh = _check_H(H)
    mr = _model_of(model)
    if out is None:
        out = torch.empty((n, n), dtype=out_dtype or torch.float32, device=H.device)
    if out.dtype not in (torch.float32, torch.float64) or out.stride(1) != 1:
        raise TypeError("out must be a row-major float32/float64 device tensor")
    tr = torch.empty(2, dtype=torch.float64, device=H.device)
    info = fe_rescale_info() if want_info else None
    rc = _check(lib().fe_expand_density_noalloc(
        C.c_void_p(H.data_ptr()), n, ldh, float(mu), float(kT), C.byref(mr.struct), PREC[prec],
        int(bool(final_correction)), C.c_void_p(out.data_ptr()), int(out.dtype == torch.float64),
        out.stride(0),
        C.c_void_p(tr.data_ptr()), C.c_void_p(tr.data_ptr() + 8),
        C.byref(info) if want_info else None, _stream_ptr()))
    d = None
    if want_info:
        d = info.as_dict()
        d["rc"] = rc
    return out, tr[0], tr[1], d


def expand_density_filling(H, n_occ: float, kT: float, model, prec: str = "fp16x2",
                           mu_init: float | None = None, tol: float | None = None,
                           max_iter: int = 50, out=None, out_dtype=None,
                           ws: Workspace | None = None):
    """fe_expand_density_filling. Returns (D, mu, iters, trD, trD2, info): the density matrix at
    the chemical potential mu with Tr D = n_occ, found by safeguarded Newton iterations.
    Default tol: 1e-6 n in the 16-bit and FP32 modes (the trace's own rounding noise is of that
    order), 1e-10 n in FP64. Synchronizes the stream once per iterate."""
    import torch
    n, ldh = _check_H(H)
    ws = ws or workspace(n)
    mr = _model_of(model)
    if out is None:
        out = torch.empty((n, n), dtype=out_dtype or torch.float32, device=H.device)
    if out.dtype not in (torch.float32, torch.float64) or out.stride(1) != 1:
        raise TypeError("out must be a row-major float32/float64 device tensor")
    tr = torch.empty(2, dtype=torch.float64, device=H.device)
    info = fe_rescale_info()
    mu = C.c_double()
    iters = C.c_int32()
    _check(lib().fe_expand_density_filling(
        C.c_void_p(H.data_ptr()), n, ldh, float(n_occ), float(kT),
        float("nan") if mu_init is None else float(mu_init), C.byref(mr.struct), PREC[prec],
        float((1e-10 if prec == "fp64" else 1e-6) * n if tol is None else tol), int(max_iter),
        C.c_void_p(out.data_ptr()), int(out.dtype == torch.float64), out.stride(0),
        C.c_void_p(tr.data_ptr()), C.c_void_p(tr.data_ptr() + 8), C.byref(mu), C.byref(iters),
        C.byref(info), ws.handle, _stream_ptr()))
    return out, mu.value, iters.value, tr[0], tr[1], info.as_dict()


def select_model(H, mu: float, kT: float, bank, ws: Workspace | None = None) -> int:
    """fe_model_select: index in `bank` (a list of models) of the model with the fewest layers
    valid for H at (mu, kT). Synchronizes the stream."""
    n, ldh = _check_H(H)
    ws = ws or workspace(n)
    refs = [_model_of(x) for x in bank]
    structs = (fe_model * len(refs))(*[r.struct for r in refs])
    idx = C.c_int32()
    _check(lib().fe_model_select(C.c_void_p(H.data_ptr()), n, ldh, float(mu), float(kT), structs,
                                 len(refs), C.byref(idx), ws.handle, _stream_ptr()))
    return idx.value


SCHEDULES = {0: "dp128", 1: "sk256", 2: "sk2x128"}


def autotune(sizes, prec: str = "fp16x2", ws: Workspace | None = None):
    """fe_autotune: per size, the chosen schedule name and each candidate's ms per expansion."""
    sizes = [int(x) for x in sizes]
    ws = ws or workspace(max(sizes))
    arr = (C.c_int64 * len(sizes))(*sizes)
    choice = (C.c_int32 * len(sizes))()
    ms = (C.c_double * (3 * len(sizes)))()
    _check(lib().fe_autotune(arr, len(sizes), PREC[prec], choice, ms, ws.handle, _stream_ptr()))
    return [{"n": n, "schedule": SCHEDULES[choice[i]],
             "ms": {SCHEDULES[c]: ms[3 * i + c] for c in range(3) if ms[3 * i + c] == ms[3 * i + c]}}
            for i, n in enumerate(sizes)]


def autotune_input(H, mu: float, kT: float, model, prec: str = "fp16x2",
                   ws: Workspace | None = None):
    """fe_autotune_input: the schedule choice made on this input; returns {n, schedule, ms}."""
    n, ldh = _check_H(H)
    ws = ws or workspace(n)
    ref = _model_of(model)
    choice = C.c_int32()
    ms = (C.c_double * 3)()
    _check(lib().fe_autotune_input(C.c_void_p(H.data_ptr()), n, ldh, float(mu), float(kT),
                                   C.byref(ref.struct), PREC[prec], C.byref(choice), ms, ws.handle,
                                   _stream_ptr()))
    return {"n": n, "schedule": SCHEDULES[choice.value],
            "ms": {SCHEDULES[c]: ms[c] for c in range(3) if ms[c] == ms[c]}}


def autotune_lookup(n: int, prec: str = "fp16x2", ws: Workspace | None = None) -> str:
    ws = ws or workspace(n)
    out = C.c_int32()
    _check(lib().fe_autotune_lookup(int(n), PREC[prec], ws.handle, C.byref(out)))
    return SCHEDULES[out.value]


def autotune_clear() -> None:
    _check(lib().fe_autotune_clear())


def observable(D, A, ws: Workspace | None = None):
    """fe_observable: <A> = 2 Tr(D A) as a 0-d float64 device tensor (asynchronous)."""
    import torch
    n = D.shape[0]
    if D.dim() != 2 or D.shape[1] != n or D.stride(1) != 1 or D.dtype not in (torch.float32, torch.float64):
        raise TypeError("D must be a square row-major float32/float64 device tensor")
    if A.shape != D.shape or A.dtype != torch.float64 or A.stride(1) != 1 or not A.is_cuda:
        raise TypeError("A must be a row-major float64 device tensor of D's shape")
    ws = ws or workspace(n)
    out = torch.empty((), dtype=torch.float64, device=D.device)
    _check(lib().fe_observable(C.c_void_p(D.data_ptr()), int(D.dtype == torch.float64), D.stride(0),
                               C.c_void_p(A.data_ptr()), A.stride(0), n, C.c_void_p(out.data_ptr()),
                               ws.handle, _stream_ptr()))
    return out


def free_energy(H, mu: float, kT: float, model, model_s=None, alpha: float = 1.0,
                prec: str = "fp16x2", out=None, want_D: bool = False, out_dtype=None,
                ws: Workspace | None = None):
    """fe_free_energy. Returns (G, S, trD, D): 0-d float64 device tensors G = 2 Tr[D (H - mu I)]
    - 2 kT S, S and Tr D, and D (``out``, or a new tensor of out_dtype, float32 by default, when
    want_D). Tr[D H] is formed from D as stored (float32 D rounds it)."""
    import torch
    n, ldh = _check_H(H)
    ws = ws or workspace(n)
    mr = _model_of(model)
    ms = _model_of(model_s) if model_s is not None else None
    if out is None and want_D:
        out = torch.empty((n, n), dtype=out_dtype or torch.float32, device=H.device)
    if out is not None and (out.dtype not in (torch.float32, torch.float64) or out.stride(1) != 1):
        raise TypeError("out must be a row-major float32/float64 device tensor")
    sc = torch.empty(3, dtype=torch.float64, device=H.device)
    _check(lib().fe_free_energy(
        C.c_void_p(H.data_ptr()), n, ldh, float(mu), float(kT), C.byref(mr.struct),
        C.byref(ms.struct) if ms is not None else None, float(alpha), PREC[prec],
        C.c_void_p(out.data_ptr() if out is not None else 0),
        int(out is not None and out.dtype == torch.float64), out.stride(0) if out is not None else 0,
        C.c_void_p(sc.data_ptr()), C.c_void_p(sc.data_ptr() + 8), C.c_void_p(sc.data_ptr() + 16),
        None, ws.handle, _stream_ptr()))
    return sc[0], sc[1], sc[2], out


def expand_entropy(H, mu: float, kT: float, model_s, alpha: float, prec: str = "fp16x2",
                   want_info: bool = False, ws: Workspace | None = None):
    """fe_expand_entropy. Returns (S 0-d float64 device tensor, info dict or None)."""
    import torch
    n, ldh = _check_H(H)
    ws = ws or workspace(n)
    mr = _model_of(model_s)
    S = torch.empty((), dtype=torch.float64, device=H.device)
    info = fe_rescale_info() if want_info else None
    rc = _check(lib().fe_expand_entropy(
        C.c_void_p(H.data_ptr()), n, ldh, float(mu), float(kT), C.byref(mr.struct), float(alpha),
        PREC[prec], C.c_void_p(S.data_ptr()), C.byref(info) if want_info else None, ws.handle,
        _stream_ptr()))
    d = None
    if want_info:
        d = info.as_dict()
        d["rc"] = rc
    return S, d


def sp2_coeffs(mu_p: float, L: int) -> np.ndarray:
    out = np.zeros((L, 4))
    _check(lib().fe_sp2_coeffs(float(mu_p), int(L), out.ctypes.data_as(C.POINTER(C.c_double))))
    return out


def layer_count(beta_p: float) -> float:
    return float(lib().fe_layer_count(float(beta_p)))


def version() -> str:
    return lib().fe_version().decode()


def streamk_segments(np_: int, schedule: int, grid: int, w: int):
    """fe_streamk_segments: (geometry dict, int32 array of w's segments, one row (pass, tile,
    kb0, kb1, jlo) each), computed on the host."""
    geom = (C.c_int32 * 6)()
    cnt = C.c_int32()
    _check(lib().fe_streamk_segments(int(np_), int(schedule), int(grid), int(w), geom, None, 0,
                                     C.byref(cnt)))
    segs = np.zeros((max(cnt.value, 1), 5), dtype=np.int32)
    _check(lib().fe_streamk_segments(int(np_), int(schedule), int(grid), int(w), geom,
                                     segs.ctypes.data_as(C.POINTER(C.c_int32)), cnt.value,
                                     C.byref(cnt)))
    g = dict(zip(("T", "ntiles", "nk", "dp_tiles", "groups", "grid"), list(geom)))
    return g, segs[:cnt.value]


def layer_events(enable: bool) -> None:
    """fe_debug_layer_events: time each layer launch of the split path with HIP events."""
    _check(lib().fe_debug_layer_events(1 if enable else 0))


def layer_events_read():
    """fe_debug_layer_events_read: ms per layer launch of the most recent expansion (numpy)."""
    cnt = C.c_int32()
    _check(lib().fe_debug_layer_events_read(None, 0, C.byref(cnt)))
    out = np.zeros(max(cnt.value, 1))
    _check(lib().fe_debug_layer_events_read(out.ctypes.data_as(C.POINTER(C.c_double)), cnt.value,
                                            C.byref(cnt)))
    return out[:cnt.value]


def debug_streamk_giveup(enable: bool) -> None:
    """fe_debug_streamk_giveup: make every stream-K wait give up (failure-handling tests)."""
    _check(lib().fe_debug_streamk_giveup(1 if enable else 0))


def batch_queue_layout(np_list, L_list, tile: int, nq: int):
    """fe_batch_queue_layout: the queue launch's work items for matrices of padded sizes np_list
    running L_list layers (batch order). Returns (items int32 [n, 4]: matrix, tile, layer, need;
    qoff int32 [nq + 1])."""
    count = len(np_list)
    npa = (C.c_int64 * count)(*[int(v) for v in np_list])
    La = (C.c_int32 * count)(*[int(v) for v in L_list])
    qoff = np.zeros(nq + 1, dtype=np.int32)
    n = C.c_int64()
    _check(lib().fe_batch_queue_layout(count, npa, La, int(tile), int(nq), None, 0,
                                       qoff.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(n)))
    items = np.zeros((max(n.value, 1), 4), dtype=np.int32)
    _check(lib().fe_batch_queue_layout(count, npa, La, int(tile), int(nq),
                                       items.ctypes.data_as(C.POINTER(C.c_int32)), n.value,
                                       qoff.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(n)))
    return items[:n.value], qoff


def debug_batch_queue_giveup(enable: bool) -> None:
    """fe_debug_batch_queue_giveup: batch plans built while enabled make every queue-launch wait
    give up (failure-handling tests)."""
    _check(lib().fe_debug_batch_queue_giveup(1 if enable else 0))


# ---- batches -----------------------------------------------------------------------------

class fe_batch_item(C.Structure):
    _fields_ = [("H", C.c_void_p), ("n", C.c_int64), ("ldh", C.c_int64), ("mu", C.c_double),
                ("kT", C.c_double), ("D", C.c_void_p), ("ldd", C.c_int64),
                ("d_is_fp64", C.c_int32), ("trD", C.c_void_p), ("trD2", C.c_void_p),
                ("S", C.c_void_p)]


SIGNATURES.update({
    "fe_batch_plan_create": (_I32, [C.POINTER(fe_batch_item), _I32, C.POINTER(fe_model),
                                    C.POINTER(fe_model), _D, _I32, _P, _P, C.POINTER(_P)]),
    "fe_batch_plan_create_bank": (_I32, [C.POINTER(fe_batch_item), _I32, C.POINTER(fe_model), _I32,
                                         _I32, _D, _I32, _P, C.POINTER(_I32), _P, C.POINTER(_P)]),
    "fe_batch_plan_launch": (_I32, [_P, _P]),
    "fe_batch_plan_destroy": (_I32, [_P]),
    "fe_batched_expand": (_I32, [C.POINTER(fe_batch_item), _I32, C.POINTER(fe_model),
                                 C.POINTER(fe_model), _D, _I32, _P, _P, _P]),
})


BATCH_LAUNCH = {"layers": 0, "queue": 1}   # FE_BATCH_LAUNCH_*


def _batch_outputs(mats, want_D, d_dtype, with_S):
    """The fe_batch_item array for `mats` (dicts with H, mu, kT) and the output tensors it points
    to: D list, tr [count, 2] (Tr D, sum D_ij^2), S [count], status [count]; plus the sum of the
    padded sizes squared (arena elements)."""
    import torch
    count = len(mats)
    dev = mats[0]["H"].device
    d_dtype = d_dtype or torch.float32
    D_list = []
    tr = torch.zeros((count, 2), dtype=torch.float64, device=dev)
    S = torch.zeros(count, dtype=torch.float64, device=dev)
    status = torch.zeros(count, dtype=torch.int32, device=dev)
    arr = (fe_batch_item * count)()
    elems = 0
    for b, m in enumerate(mats):
        n, ldh = _check_H(m["H"])
        D = torch.empty((n, n), dtype=d_dtype, device=dev) if want_D else None
        D_list.append(D)
        arr[b] = fe_batch_item(m["H"].data_ptr(), n, ldh, float(m["mu"]), float(m["kT"]),
                               D.data_ptr() if want_D else None, n if want_D else 0,
                               int(d_dtype == torch.float64),
                               tr.data_ptr() + 16 * b, tr.data_ptr() + 16 * b + 8,
                               S.data_ptr() + 8 * b if with_S else None)
        np_ = -(-n // 128) * 128
        elems += np_ * np_
    return arr, D_list, tr, S, status, elems


def batched_expand(mats, model, prec="fp16x2", model_s=None, alpha=1.0, ws=None, d_dtype=None):
    """fe_batched_expand: one-shot batch (plan, launch, wait, destroy) on the current stream.
    Returns (D list, tr [count, 2], S [count] (with model_s), status [count])."""
    arr, D, tr, S, status, elems = _batch_outputs(mats, True, d_dtype, model_s is not None)
    if prec == "bf16x3":   # 20 instead of 16 bytes of the arena per padded element
        elems = -(-elems * 20 // 16)
    ws = ws or Workspace(128, max_batch=len(mats), batch_elems=elems)
    m = _model_of(model)
    ms = _model_of(model_s) if model_s is not None else None
    _check(lib().fe_batched_expand(arr, len(mats), C.byref(m.struct),
                                   C.byref(ms.struct) if ms else None, float(alpha), PREC[prec],
                                   C.c_void_p(status.data_ptr()), ws.handle, _stream_ptr()))
    return D, tr, S, status


class BatchPlan:
    """A captured batch (fe_batch_plan_create): `launch()` replays it on the current stream.
    By default every layer of every matrix runs in one queue launch (`set_launch`).

    Each entry of `mats` is a dict with keys H (float64 device tensor), mu, kT. Outputs are
    allocated here: D (float32, or float64 with d_dtype), traces tr[b] = (Tr D, sum D_ij^2), S[b]
    (entropy, when model_s is given or with_entropy with a bank) and status[b] (int32 rescale
    status).

    `model` is one model, or a list of models (a bank, fe_batch_plan_create_bank): then every
    matrix runs the bank model with the fewest layers whose region of validity contains its
    (beta', mu'), and `chosen[b]` is that model's index in the list."""

    def __init__(self, mats, model, prec="fp16x2", model_s=None, alpha=1.0, ws=None,
                 want_D=True, d_dtype=None, with_entropy=False):
        self.count = len(mats)
        self.H = [m["H"] for m in mats]
        arr, self.D, self.tr, self.S, self.status, elems = _batch_outputs(
            mats, want_D, d_dtype, model_s is not None or with_entropy)
        self._items = arr
        if prec == "bf16x3":   # 20 instead of 16 bytes of the arena per padded element
            elems = -(-elems * 20 // 16)
        self.ws = ws or Workspace(128, max_batch=self.count, batch_elems=elems)
        p = C.c_void_p()
        self.chosen = None
        if isinstance(model, (list, tuple)):
            self._bank = [_model_of(x) for x in model]
            structs = (fe_model * len(self._bank))(*[x.struct for x in self._bank])
            self._bank_structs = structs
            chosen = (C.c_int32 * self.count)()
            _check(lib().fe_batch_plan_create_bank(
                arr, self.count, structs, len(self._bank), int(bool(with_entropy)), float(alpha),
                PREC[prec], C.c_void_p(self.status.data_ptr()), chosen, self.ws.handle,
                C.byref(p)))
            self.chosen = np.array(chosen[:], dtype=np.int32)
        else:
            self._m = _model_of(model)
            self._ms = _model_of(model_s) if model_s is not None else None
            _check(lib().fe_batch_plan_create(arr, self.count, C.byref(self._m.struct),
                                              C.byref(self._ms.struct) if self._ms else None,
                                              float(alpha), PREC[prec],
                                              C.c_void_p(self.status.data_ptr()), self.ws.handle,
                                              C.byref(p)))
        self._p = p

    def launch(self):
        _check(lib().fe_batch_plan_launch(self._p, _stream_ptr()))

    def retile(self, tile: int):
        """fe_batch_plan_retile: rebuild with 128 x 128 or 64 x 64 layer tiles."""
        _check(lib().fe_batch_plan_retile(self._p, int(tile)))

    def set_launch(self, launch: str):
        """fe_batch_plan_set_launch: "layers" (one grouped launch per layer) or "queue" (every
        layer of every matrix in one launch)."""
        _check(lib().fe_batch_plan_set_launch(self._p, BATCH_LAUNCH[launch]))

    @property
    def launch_form(self) -> str:
        """fe_batch_plan_get: "queue" or "layers"."""
        launch = C.c_int32()
        _check(lib().fe_batch_plan_get(self._p, None, C.byref(launch)))
        return {v: k for k, v in BATCH_LAUNCH.items()}[launch.value]

    @property
    def tile(self) -> int:
        """fe_batch_plan_get: the layer tile size (128 or 64)."""
        tile = C.c_int32()
        _check(lib().fe_batch_plan_get(self._p, C.byref(tile), None))
        return tile.value

    def autotune(self):
        """fe_batch_plan_autotune: keeps the fastest tile size and launch form; returns
        (tile, {tile: ms of its faster launch form}); `launch_form` holds the chosen form."""
        tile = C.c_int32()
        ms = (C.c_double * 2)()
        _check(lib().fe_batch_plan_autotune(self._p, _stream_ptr(), C.byref(tile), ms))
        return tile.value, {t: v for t, v in ((128, ms[0]), (64, ms[1])) if v == v}

    def close(self):
        if self._p:
            lib().fe_batch_plan_destroy(self._p)
            self._p = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
