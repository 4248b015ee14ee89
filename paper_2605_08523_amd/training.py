"""Coefficient training through the HIP library (argument marshalling only).

* ``train_coeffs``: fe_train_coeffs, Levenberg-Marquardt with geodesic acceleration on scalar
  sample points of the model coordinate (Sec. III.C), Jacobians on the GPU.
* ``scalar_eval``: fe_scalar_eval, the scalar model, residuals and Jacobian on the GPU.
* ``MatrixRecursion``: a torch.autograd.Function whose forward (fe_matrix_forward) and
  backward (fe_matrix_backward) are the library's FP32 kernels, for fitting on matrices.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import api

TARGET = {"fermi": 0, "entropy": 1}
SAMPLING = {"uniform": 0, "deriv": 1, "arclen": 2}


class fe_train_spec(C.Structure):
    _fields_ = [("target", C.c_int32), ("L", C.c_int32), ("beta0", C.c_double),
                ("mu0", C.c_double), ("alpha", C.c_double), ("n_points", C.c_int32),
                ("sampling", C.c_int32), ("max_iter", C.c_int32), ("tol", C.c_double),
                ("n_mats", C.c_int32), ("mat_iters", C.c_int32), ("mat_n", C.c_int64),
                ("X0s", C.POINTER(C.c_void_p)), ("Drefs", C.POINTER(C.c_void_p)),
                ("mat_weight", C.c_double)]


class fe_train_report(C.Structure):
    _fields_ = [("iters", C.c_int32), ("rms", C.c_double), ("max_err_points", C.c_double),
                ("max_err_grid", C.c_double), ("lambda_", C.c_double), ("mat_iters", C.c_int32),
                ("mat_accepted", C.c_int32), ("mat_loss_start", C.c_double),
                ("mat_loss_end", C.c_double)]

    def as_dict(self):
        return {"iters": self.iters, "rms": self.rms, "max_err_points": self.max_err_points,
                "max_err_grid": self.max_err_grid, "lambda": self.lambda_,
                "mat_iters": self.mat_iters, "mat_accepted": self.mat_accepted,
                "mat_loss_start": self.mat_loss_start, "mat_loss_end": self.mat_loss_end}


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def train_coeffs(L: int, beta0: float, mu0: float, target: str = "fermi", alpha: float = 1.0,
                 n_points: int = 8192, sampling: str = "deriv", max_iter: int = 500,
                 tol: float = 1e-8, theta_init=None, mats=None, mat_iters: int = 20,
                 mat_weight: float = 1.0):
    """Returns (theta L x 4, report dict, converged flag). mats: optional list of (X0, Dref)
    device tensors (float32 and float64, n x n, n a multiple of 64) for the matrix-set
    refinement of fe_train_coeffs."""
    spec = fe_train_spec(TARGET[target], int(L), float(beta0), float(mu0), float(alpha),
                         int(n_points), SAMPLING[sampling], int(max_iter), float(tol))
    keep = None
    if mats:
        n = int(mats[0][0].shape[0])
        X0s = (C.c_void_p * len(mats))(*[C.c_void_p(x.data_ptr()) for x, _ in mats])
        Drefs = (C.c_void_p * len(mats))(*[C.c_void_p(dd.data_ptr()) for _, dd in mats])
        keep = (X0s, Drefs, mats)
        spec.n_mats, spec.mat_iters, spec.mat_n = len(mats), int(mat_iters), n
        spec.X0s = C.cast(X0s, C.POINTER(C.c_void_p))
        spec.Drefs = C.cast(Drefs, C.POINTER(C.c_void_p))
        spec.mat_weight = float(mat_weight)
    out = np.zeros((L, 4))
    init = None if theta_init is None else np.ascontiguousarray(theta_init, dtype=np.float64)
    rep = fe_train_report()
    rc = api.lib().fe_train_coeffs(C.byref(spec), _dp(init) if init is not None else None,
                                   _dp(out), C.byref(rep), None, api._stream_ptr())
    del keep
    if rc < 0 and rc != api.FE_ERR_NO_CONVERGENCE:
        api._check(rc)
    return out, rep.as_dict(), rc == api.FE_OK


def scalar_eval(y, theta, target: str = "fermi", mu0: float = 1.0 / 3.0, alpha: float = 1.0,
                tgt=None, jacobian: bool = True):
    """y: float64 device tensor. Returns (r, JT) device tensors (JT is 4L x n or None)."""
    import torch
    th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64).reshape(-1, 4))
    L = th.shape[0]
    n = y.numel()
    r = torch.empty(n, dtype=torch.float64, device=y.device)
    JT = torch.empty((4 * L, n), dtype=torch.float64, device=y.device) if jacobian else None
    api._check(api.lib().fe_scalar_eval(
        C.c_void_p(y.data_ptr()), n, _dp(th), L, TARGET[target], float(mu0), float(alpha),
        C.c_void_p(tgt.data_ptr()) if tgt is not None else None, C.c_void_p(r.data_ptr()),
        C.c_void_p(JT.data_ptr()) if jacobian else None, api._stream_ptr()))
    return r, JT


def scalar_second(y, theta, v, target: str = "fermi", mu0: float = 1.0 / 3.0,
                  alpha: float = 1.0):
    """fe_scalar_second: d^2/dt^2 of the scalar model at theta + t v (y: float64 device tensor;
    theta, v: L x 4). Returns a device tensor."""
    import torch
    th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64).reshape(-1, 4))
    vd = torch.from_numpy(np.ascontiguousarray(np.asarray(v, dtype=np.float64).reshape(-1, 4))).to(y.device)
    r2 = torch.empty(y.numel(), dtype=torch.float64, device=y.device)
    api._check(api.lib().fe_scalar_second(
        C.c_void_p(y.data_ptr()), y.numel(), _dp(th), th.shape[0], TARGET[target], float(mu0),
        float(alpha), C.c_void_p(vd.data_ptr()), C.c_void_p(r2.data_ptr()), api._stream_ptr()))
    return r2


def _autograd_fn():
    import torch

    class MatrixRecursion(torch.autograd.Function):
        """P = A_L + X_L of the layer recursion on X0 (FP32 kernels), differentiable in theta.

        theta: CPU float64 tensor L x 4 (requires_grad); X0: device float32 n x n symmetric,
        n a multiple of 64."""

        @staticmethod
        def forward(ctx, theta, X0):
            n = X0.shape[0]
            L = theta.shape[0]
            th = np.ascontiguousarray(theta.detach().cpu().numpy(), dtype=np.float64)
            hist = torch.empty((L + 1, n, n), dtype=torch.float32, device=X0.device)
            hist[0].copy_(X0)
            P = torch.empty((n, n), dtype=torch.float32, device=X0.device)
            api._check(api.lib().fe_matrix_forward(C.c_void_p(hist.data_ptr()), n, _dp(th), L,
                                                   C.c_void_p(P.data_ptr()), api._stream_ptr()))
            ctx.save_for_backward(hist)
            ctx.th = th
            return P

        @staticmethod
        def backward(ctx, G):
            (hist,) = ctx.saved_tensors
            th = ctx.th
            L = th.shape[0]
            n = hist.shape[1]
            G = G.contiguous().float()
            work = torch.empty((3, n, n), dtype=torch.float32, device=G.device)
            nblocks = 256
            part = torch.empty((nblocks, 4), dtype=torch.float64, device=G.device)
            grad = torch.empty((L, 4), dtype=torch.float64, device=G.device)
            api._check(api.lib().fe_matrix_backward(
                C.c_void_p(hist.data_ptr()), n, _dp(th), L, C.c_void_p(G.data_ptr()),
                C.c_void_p(work.data_ptr()), C.c_void_p(part.data_ptr()), nblocks,
                C.c_void_p(grad.data_ptr()), api._stream_ptr()))
            return grad.cpu(), None

    return MatrixRecursion


_MR = None


def matrix_recursion(theta, X0):
    global _MR
    if _MR is None:
        _MR = _autograd_fn()
    return _MR.apply(theta, X0)
