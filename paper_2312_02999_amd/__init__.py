"""MI355X-native PD+IPC quasi-static solver (Li, Yang, Solenthaler 2023).

Python front-end of the C ABI in ``include/pdipc.h``.  torch is used only for
device memory and streams: every step of a frame runs in the HIP kernels of
``libpdipc.so``.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib
from ._lib import FrameStats, IterTrace, MeshDesc, Options, PdipcError, check, lib

__all__ = ["Solver", "PdipcError", "FP64", "MIXED_FP32", "host_factor_solve", "actuation_rows", "PDIPCFrame",
           "dense_spd", "dense_spd_noalloc", "GSTEP_SCHUR_WOODBURY", "GSTEP_PCG",
           "GSTEP_SCHUR"]

FP64, MIXED_FP32 = 0, 1
# global steps (Table 1): Schur complement + low-rank update (the method), the
# conjugate-gradient baseline, the Schur complement alone
GSTEP_SCHUR_WOODBURY, GSTEP_PCG, GSTEP_SCHUR = 0, 1, 2


def _dev(t: torch.Tensor, shape=None) -> int:
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
        raise TypeError("expected a contiguous float64 CUDA (ROCm) tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"expected shape {shape}, got {tuple(t.shape)}")
    return t.data_ptr()


def actuation_rows(A: np.ndarray) -> np.ndarray:
    """(m, 3, 3) symmetric -> (m, 6) rows (xx, yy, zz, xy, yz, zx)."""
    return np.stack([A[:, 0, 0], A[:, 1, 1], A[:, 2, 2], A[:, 0, 1], A[:, 1, 2], A[:, 2, 0]], axis=1)


class Solver:
    """One mesh, its constant factor and its device state.

    Arguments follow ``pdipc_mesh_desc`` / ``pdipc_options``; ``scene`` may be
    any object with the attributes of ``meshgen.Scene``.
    """

    def __init__(self, scene=None, *, X=None, tets=None, dirichlet=None, surf_tris=None, region=None,
                 youngs=None, poisson=None, dhat=None, kappa=None, iters=30, tol=0.0, precision=FP64,
                 ccd_eta=0.1, ccd_steps=16, ls_max_halvings=20, cinv_updates_max=16,
                 fp32_reduced_min=8192, hinv_rows_mb=4096, device="cuda", stream=None, W=None,
                 global_method=0, cg_tol=1e-12, cg_max_iters=2000, barrier_form=0, kappa_adapt=False):
        # material and barrier parameters: explicit arguments, else the
        # scene's, else E = 1e4, nu = 0.45, dhat = 5e-4, kappa = 1e3
        defaults = {"youngs": 1e4, "poisson": 0.45, "dhat": 5e-4, "kappa": 1e3}
        given = {"youngs": youngs, "poisson": poisson, "dhat": dhat, "kappa": kappa}
        if scene is not None:
            X, tets, dirichlet, surf_tris = scene.X, scene.tets, scene.dirichlet, scene.surf_tris
            region = scene.region
            defaults = {k: getattr(scene, k) for k in defaults}
            if W is None:
                W = getattr(scene, "W", None)
        youngs, poisson, dhat, kappa = (given[k] if given[k] is not None else defaults[k]
                                        for k in ("youngs", "poisson", "dhat", "kappa"))
        self.device = torch.device(device)
        self._X = np.ascontiguousarray(X, dtype=np.float64)
        self._tets = np.ascontiguousarray(tets, dtype=np.int32)
        self._dir = np.ascontiguousarray(dirichlet, dtype=np.uint8)
        self._tris = np.ascontiguousarray(surf_tris, dtype=np.int32).reshape(-1, 3)
        self._reg = None if region is None else np.ascontiguousarray(region, dtype=np.uint8)
        self.n, self.m = self._X.shape[0], self._tets.shape[0]
        md = MeshDesc(self.n, self.m, self._X.ctypes.data, self._tets.ctypes.data, self._dir.ctypes.data,
                      self._tris.shape[0], self._tris.ctypes.data if self._tris.size else None,
                      self._reg.ctypes.data if self._reg is not None else None, float(youngs), float(poisson))
        if W is not None:
            # proxy embedding s = W x as CSR (rowptr, col, val or None); the
            # triangles then index proxy vertices (rows of W)
            rowptr, col, val = W
            self._W = (np.ascontiguousarray(rowptr, dtype=np.int32), np.ascontiguousarray(col, dtype=np.int32),
                       None if val is None else np.ascontiguousarray(val, dtype=np.float64))
            md.n_surf_verts = self._W[0].size - 1
            md.W_rowptr = self._W[0].ctypes.data
            md.W_col = self._W[1].ctypes.data
            md.W_val = self._W[2].ctypes.data if self._W[2] is not None else None
        with torch.cuda.device(self.device):
            st = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.stream = st
        op = Options(float(dhat), float(kappa), int(iters), float(tol), int(precision), float(ccd_eta),
                     int(ccd_steps), int(ls_max_halvings), int(cinv_updates_max),
                     int(fp32_reduced_min), int(hinv_rows_mb), C.c_void_p(st.cuda_stream), int(global_method),
                     float(cg_tol), int(cg_max_iters), int(barrier_form), int(bool(kappa_adapt)))
        h = C.c_void_p()
        check(lib().pdipc_init_mesh(C.byref(md), C.byref(op), C.byref(h)), None)
        self._h = h
        self.iters = iters

    # ------------------------------------------------------------------ API
    def close(self):
        if getattr(self, "_h", None):
            lib().pdipc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sizes(self):
        a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
        check(lib().pdipc_get_sizes(self._h, C.byref(a), C.byref(b), C.byref(c)), self._h)
        return {"n1": a.value, "n2": b.value, "factor_nnz": c.value}

    def device_bytes(self) -> int:
        b = C.c_int64()
        check(lib().pdipc_device_bytes(self._h, C.byref(b)), self._h)
        return b.value

    def set_actuation(self, A: torch.Tensor):
        check(lib().pdipc_set_actuation(self._h, _dev(A, (self.m, 6))), self._h)

    def set_actuation_scalar(self, a: torch.Tensor, R: torch.Tensor | None = None):
        rp = _dev(R, (self.m, 9)) if R is not None else None
        check(lib().pdipc_set_actuation_scalar(self._h, _dev(a, (self.m,)), rp), self._h)

    def solve_frame(self, x_in: torch.Tensor, x_out: torch.Tensor | None = None, stats: bool = False):
        if x_out is None:
            x_out = torch.empty_like(x_in)
        fs = FrameStats()
        rc = lib().pdipc_solve_frame(self._h, _dev(x_in, (self.n, 3)), _dev(x_out, (self.n, 3)),
                                     C.byref(fs) if stats else None)
        check(rc, self._h)
        self.last_status = rc
        return (x_out, fs.as_dict()) if stats else x_out

    def solve_frame_backward(self, dL_dx: torch.Tensor) -> torch.Tensor:
        out = torch.empty(self.m, dtype=torch.float64, device=self.device)
        check(lib().pdipc_solve_frame_backward(self._h, _dev(dL_dx, (self.n, 3)), _dev(out)), self._h)
        return out

    def kernel_timer(self, which: int = -1):
        """Return (total_ms, launches) since the last call and arm the timer for ``which``."""
        t, c = C.c_double(), C.c_int64()
        check(lib().pdipc_kernel_timer(self._h, int(which), C.byref(t), C.byref(c)), self._h)
        return t.value, c.value

    # ------------------------------------------------------------ debug taps
    def debug_local(self, x: torch.Tensor):
        R = torch.empty(self.m, 9, dtype=torch.float64, device=self.device)
        E = torch.empty(self.m, dtype=torch.float64, device=self.device)
        g = torch.empty(self.n, 3, dtype=torch.float64, device=self.device)
        check(lib().pdipc_debug_local(self._h, _dev(x, (self.n, 3)), _dev(R), _dev(E), _dev(g)), self._h)
        return R, E, g

    def debug_contacts(self, x: torch.Tensor, cap: int = 1 << 20):
        cnt = C.c_int32()
        check(lib().pdipc_debug_contacts(self._h, _dev(x, (self.n, 3)), None, 0, C.byref(cnt)), self._h)
        k = cnt.value
        buf = torch.empty(max(k, 1) * 3, dtype=torch.int32, device=self.device)
        check(lib().pdipc_debug_contacts(self._h, _dev(x, (self.n, 3)), buf.data_ptr(), k, C.byref(cnt)), self._h)
        return buf[: 3 * k].reshape(k, 3).cpu().numpy()

    def trace(self):
        """Per-iteration records of the last frame (list of dicts)."""
        cnt = C.c_int32()
        check(lib().pdipc_debug_trace(self._h, None, 0, C.byref(cnt)), self._h)
        buf = (IterTrace * max(cnt.value, 1))()
        check(lib().pdipc_debug_trace(self._h, buf, cnt.value, C.byref(cnt)), self._h)
        return [buf[i].as_dict() for i in range(cnt.value)]

    def debug_step(self, x: torch.Tensor):
        dx = torch.empty(self.n, 3, dtype=torch.float64, device=self.device)
        am, a = C.c_double(), C.c_double()
        check(lib().pdipc_debug_step(self._h, _dev(x, (self.n, 3)), _dev(dx), C.byref(am), C.byref(a)), self._h)
        return dx, am.value, a.value


class PDIPCFrame(torch.autograd.Function):
    """x* = frame(a; x_init) as a differentiable function of the per-tet
    actuation scalars a (frames R fixed).  The backward pass is the adjoint of
    the converged quasi-static solve (``pdipc_solve_frame_backward``); the
    gradient with respect to x_init is None because an equilibrium does not
    depend on its initial guess.  The solver must not run another frame
    between forward and backward."""

    @staticmethod
    def forward(ctx, a, x_init, solver, R):
        solver.set_actuation_scalar(a.detach().contiguous(), R)
        x = solver.solve_frame(x_init.detach().contiguous())
        ctx.solver = solver
        return x

    @staticmethod
    def backward(ctx, gx):
        return ctx.solver.solve_frame_backward(gx.contiguous()), None, None, None


def dense_spd(A: torch.Tensor, b: torch.Tensor | None = None, inverse: bool = False, precision: int = FP64):
    """Dense SPD kernels on device data: returns (x or None, A^-1 or None)."""
    n = A.shape[0]
    x = None if b is None else b.clone().contiguous()
    nrhs = 0 if x is None else (1 if x.dim() == 1 else x.shape[1])
    inv = torch.empty_like(A) if inverse else None
    check(lib().pdipc_debug_dense(_dev(A, (n, n)), n, _dev(x) if x is not None else None, nrhs,
                                  _dev(inv) if inv is not None else None, int(precision)), None)
    return x, inv


def dense_spd_noalloc(A: torch.Tensor, b: torch.Tensor | None = None, inverse: bool = False,
                      precision: int = FP64, stream=None):
    """pdipc_dense_spd_noalloc on device data: returns (x or None, A^-1 or
    None, info).  The library allocates nothing; the output tensors here are
    the caller's.  The work is queued on ``stream`` (default: the current
    stream); info (a one-element int32 device tensor) is 0 on success."""
    n = A.shape[0]
    x = None if b is None else b.clone().contiguous()
    nrhs = 0 if x is None else (1 if x.dim() == 1 else x.shape[1])
    inv = torch.empty_like(A) if inverse else None
    info = torch.empty(1, dtype=torch.int32, device=A.device)
    st = stream if stream is not None else torch.cuda.current_stream(A.device)
    check(lib().pdipc_dense_spd_noalloc(_dev(A, (n, n)), n, _dev(x) if x is not None else None, nrhs,
                                        _dev(inv) if inv is not None else None, int(precision), info.data_ptr(),
                                        C.c_void_p(st.cuda_stream)), None)
    return x, inv, info


def host_factor_solve(n1: int, n2: int, coords1, ptr, col, val, b=None, leaf: int = 96):
    """Host-only factor check (no GPU): returns (x, Sigma_s, factor_nnz)."""
    coords1 = np.ascontiguousarray(coords1, dtype=np.float64)
    ptr = np.ascontiguousarray(ptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    val = np.ascontiguousarray(val, dtype=np.float64)
    N = n1 + n2
    sig = np.zeros((n2, n2))
    nnz = C.c_int64()
    x = None
    bp = xp = None
    if b is not None:
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.zeros(N)
        bp, xp = b.ctypes.data, x.ctypes.data
    rc = lib().pdipc_debug_host_factor(n1, n2, coords1.ctypes.data, ptr.ctypes.data, col.ctypes.data,
                                       val.ctypes.data, leaf, bp, xp, sig.ctypes.data if n2 else None,
                                       C.byref(nnz))
    check(rc, None)
    return x, sig, nnz.value
