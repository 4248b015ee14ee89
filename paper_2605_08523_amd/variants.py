"""Skip-SP2 and Max-SP2 through the HIP library (argument marshalling only; Sec. III.A, App. C).

* ``QModel``: a model of either family (shape + host coefficients in the layout of fe_qmodel).
* ``embed_mlsp2``: fe_embed_mlsp2, an MLSP2 model as Skip-SP2 (k = K = 1) or Max-SP2.
* ``expand_density_variant``: fe_expand_density_variant on a resident Hamiltonian.
* ``variant_eval``: fe_variant_eval, the scalar model and its Jacobian on device points.
* ``train_variant``: fe_train_variant, Levenberg-Marquardt from an initial model.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np

from . import api
from .training import SAMPLING, fe_train_report, fe_train_spec

ARCH = {"max": 1, "skip": 2}


def coef_count(arch: str, L: int, k: int = 1, K: int = 1) -> int:
    out = C.c_int64()
    api._check(api.lib().fe_qmodel_coef_count(ARCH[arch], int(L), int(k), int(K), C.byref(out)))
    return out.value


@dataclass
class QModel:
    arch: str
    L: int
    coef: np.ndarray
    beta0: float
    mu0: float
    k: int = 1
    K: int = 1

    def __post_init__(self):
        self.coef = np.ascontiguousarray(np.asarray(self.coef, dtype=np.float64).ravel())
        want = coef_count(self.arch, self.L, self.k, self.K)
        if self.coef.size != want:
            raise ValueError(f"{self.arch} model with L={self.L} needs {want} coefficients")
        self.struct = api.fe_qmodel(ARCH[self.arch], int(self.L), int(self.k), int(self.K),
                                    float(self.beta0), float(self.mu0),
                                    self.coef.ctypes.data_as(C.POINTER(C.c_double)))


def embed_mlsp2(model, arch: str) -> QModel:
    """The MLSP2 model (anything with theta, beta0, mu0) as a Skip-SP2 (k = K = 1) or Max-SP2
    model with the same function (App. C)."""
    mr = api._model_of(model)
    L = mr.struct.L
    out = np.zeros(coef_count(arch, L, 1, 1))
    api._check(api.lib().fe_embed_mlsp2(C.byref(mr.struct), ARCH[arch],
                                        out.ctypes.data_as(C.POINTER(C.c_double))))
    return QModel(arch, L, out, mr.struct.beta0, mr.struct.mu0)


def scratch_bytes(n: int, qm: QModel) -> int:
    out = C.c_int64()
    api._check(api.lib().fe_variant_scratch_bytes(int(n), C.byref(qm.struct), C.byref(out)))
    return out.value


def expand_density_variant(H, mu: float, kT: float, qm: QModel, prec: str = "fp16x2", out=None,
                           out_dtype=None, want_info: bool = False, scratch=None,
                           ws: api.Workspace | None = None):
    """Returns (D, trD, trD2, info) like api.expand_density. ``scratch`` (a uint8 device tensor
    of at least scratch_bytes(n, qm)) is allocated if not given."""
    import torch
    n, ldh = api._check_H(H)
    ws = ws or api.workspace(n)
    nbytes = scratch_bytes(n, qm)
    if scratch is None:
        scratch = torch.empty(nbytes, dtype=torch.uint8, device=H.device)
    if out is None:
        out = torch.empty((n, n), dtype=out_dtype or torch.float32, device=H.device)
    if out.dtype not in (torch.float32, torch.float64) or out.stride(1) != 1:
        raise TypeError("out must be a row-major float32/float64 device tensor")
    tr = torch.empty(2, dtype=torch.float64, device=H.device)
    info = api.fe_rescale_info() if want_info else None
    rc = api._check(api.lib().fe_expand_density_variant(
        C.c_void_p(H.data_ptr()), n, ldh, float(mu), float(kT), C.byref(qm.struct), api.PREC[prec],
        C.c_void_p(scratch.data_ptr()), scratch.numel(), C.c_void_p(out.data_ptr()),
        int(out.dtype == torch.float64), out.stride(0), C.c_void_p(tr.data_ptr()),
        C.c_void_p(tr.data_ptr() + 8), C.byref(info) if want_info else None, ws.handle,
        api._stream_ptr()))
    d = None
    if want_info:
        d = info.as_dict()
        d["rc"] = rc
    return out, tr[0], tr[1], d


def variant_eval(y, qm: QModel, tgt=None, jacobian: bool = True):
    """y: float64 device tensor. Returns (r, JT) device tensors (JT: coefficients x points)."""
    import torch
    coef = torch.from_numpy(qm.coef).to(y.device)
    n = y.numel()
    r = torch.empty(n, dtype=torch.float64, device=y.device)
    JT = torch.empty((qm.coef.size, n), dtype=torch.float64, device=y.device) if jacobian else None
    api._check(api.lib().fe_variant_eval(
        C.c_void_p(y.data_ptr()), n, C.byref(qm.struct), C.c_void_p(coef.data_ptr()),
        C.c_void_p(tgt.data_ptr()) if tgt is not None else None, C.c_void_p(r.data_ptr()),
        C.c_void_p(JT.data_ptr()) if jacobian else None, api._stream_ptr()))
    torch.cuda.current_stream().synchronize()   # coef is a temporary
    return r, JT


def train_variant(init: QModel, beta0: float, mu0: float, n_points: int = 8192,
                  sampling: str = "deriv", max_iter: int = 200, tol: float = 1e-8):
    """Returns (QModel with the fitted coefficients at (beta0, mu0), report dict, converged)."""
    spec = fe_train_spec(0, int(init.L), float(beta0), float(mu0), 1.0, int(n_points),
                         SAMPLING[sampling], int(max_iter), float(tol))
    out = np.zeros_like(init.coef)
    rep = fe_train_report()
    rc = api.lib().fe_train_variant(C.byref(spec), C.byref(init.struct),
                                    out.ctypes.data_as(C.POINTER(C.c_double)), C.byref(rep),
                                    api._stream_ptr())
    if rc < 0 and rc != api.FE_ERR_NO_CONVERGENCE:
        api._check(rc)
    fitted = QModel(init.arch, init.L, out, beta0, mu0, init.k, init.K)
    return fitted, rep.as_dict(), rc == api.FE_OK
