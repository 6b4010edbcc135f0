"""Python binding of libvie.so: argument marshalling only.

Every step of the method runs in the HIP library; this module converts torch
device tensors to pointers and forwards the calls of include/vie.h.  If the
library has not been built the import of ``lib()`` raises -- there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvie.so")

VIE_OK, VIE_EINVAL, VIE_ENOMEM, VIE_EDEVICE, VIE_ENOCONV, VIE_ENUMERIC, VIE_ESTATE, VIE_ENOTIMPL = \
    0, -1, -2, -3, -4, -5, -6, -7
VIE_FP64, VIE_WITH_FP32, VIE_NO_AUTOTUNE = 0, 1, 2

_lib = None


class VieError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"vie error {code}: {msg}")
        self.code = code


class SolveOpts(ctypes.Structure):
    _fields_ = [("restart", ctypes.c_int), ("maxit", ctypes.c_int), ("use_x0", ctypes.c_int),
                ("precision", ctypes.c_int), ("inner_restart", ctypes.c_int), ("inner_tol", ctypes.c_double),
                ("use_graph", ctypes.c_int), ("stall_restarts", ctypes.c_int)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("inner_iters", ctypes.c_int), ("restarts", ctypes.c_int),
                ("matvecs", ctypes.c_int), ("status", ctypes.c_int), ("rel_res_true", ctypes.c_double),
                ("rel_res_est", ctypes.c_double), ("seconds", ctypes.c_double), ("fallback", ctypes.c_int),
                ("stalled", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class CirculantInfo(ctypes.Structure):
    _fields_ = [("support_columns", ctypes.c_int), ("block_size", ctypes.c_int), ("blocks", ctypes.c_int),
                ("first_slice", ctypes.c_int), ("fp64", ctypes.c_int), ("bytes", ctypes.c_size_t),
                ("seconds", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def lib() -> ctypes.CDLL:
    """Load libvie.so (built by paper_1803_06237_amd.build); raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} not built: run python -m paper_1803_06237_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        ip = ctypes.POINTER(ctypes.c_int)
        L.vie_version.restype = ctypes.c_char_p
        L.vie_last_error.restype = ctypes.c_char_p
        L.vie_last_error.argtypes = [vp]
        L.vie_green_table.argtypes = [ip, ctypes.c_double, vp, ctypes.c_int]
        L.vie_plan.argtypes = [ctypes.POINTER(vp), ip, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                               ctypes.c_uint, vp]
        L.vie_set_contrast.argtypes = [vp, vp]
        L.vie_rhs.argtypes = [vp, vp, vp]
        L.vie_get_contrast.argtypes = [vp, vp]
        L.vie_matvec.argtypes = [vp, vp, vp]
        L.vie_matvec_c64.argtypes = [vp, vp, vp]
        L.vie_residual.argtypes = [vp, vp, vp, vp]
        L.vie_solve.argtypes = [vp, vp, vp, ctypes.c_double, ctypes.POINTER(SolveOpts),
                                ctypes.POINTER(SolveInfo)]
        L.vie_solve_noalloc.argtypes = [vp, vp, vp, ctypes.c_double, ctypes.POINTER(SolveOpts),
                                ctypes.POINTER(SolveInfo)]
        L.vie_profile_matvec.argtypes = [vp, ctypes.c_int, vp, vp, ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
        L.vie_solve_batch.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.c_int,
                                      ctypes.c_double, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveInfo)]
        L.vie_destroy.argtypes = [vp]
        L.vie_destroy.restype = None
        L.vie_net_create.argtypes = [ctypes.POINTER(vp), ip, ctypes.c_uint, vp]
        L.vie_net_destroy.argtypes = [vp]
        L.vie_net_destroy.restype = None
        L.vie_net_num_params.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
        L.vie_net_get_params.argtypes = [vp, vp, ctypes.c_size_t]
        L.vie_net_set_params.argtypes = [vp, vp, ctypes.c_size_t]
        L.vie_net_get_state.argtypes = [vp, vp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_int)]
        L.vie_net_set_state.argtypes = [vp, vp, ctypes.c_size_t, ctypes.c_int]
        L.vie_net_apply.argtypes = [vp, vp, vp, vp]
        L.vie_net_train_step.argtypes = [vp, ctypes.c_int, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                         ctypes.POINTER(vp), ctypes.c_float, ctypes.POINTER(ctypes.c_double)]
        L.vie_set_preconditioner.argtypes = [vp, vp]
        L.vie_circulant_build.argtypes = [vp, ctypes.c_uint, ctypes.POINTER(CirculantInfo)]
        L.vie_get_tune.argtypes = [vp, ctypes.c_int, ip, ip]
        L.vie_set_tune.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.vie_circulant_apply.argtypes = [vp, vp, vp]
        L.vie_nn_conv_test.argtypes = [ctypes.c_int, ip, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, vp, vp,
                                       ctypes.c_int, vp]
        L.vie_net_get_grads.argtypes = [vp, vp, ctypes.c_size_t]
        L.vie_net_apply_base.argtypes = [vp, vp, vp, vp, vp]
        L.vie_net_train_step_base.argtypes = [vp, ctypes.c_int, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                              ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.c_float,
                                              ctypes.POINTER(ctypes.c_double)]
        L.vie_nn_op_test.argtypes = [ctypes.c_int, ip, ctypes.c_int, vp, vp, vp, vp, vp]
        L.vie_nn_adam_test.argtypes = [ctypes.c_long, vp, vp, vp, vp, ctypes.c_int, ctypes.c_float, vp]
        L.vie_net_last_error.restype = ctypes.c_char_p
        L.vie_net_last_error.argtypes = [vp]
        L.vie_curl_table.argtypes = [ip, ctypes.c_double, vp, ctypes.c_int]
        L.vie_jm_enable.argtypes = [vp]
        L.vie_jm_set_permeability.argtypes = [vp, vp]
        L.vie_jm_set_route.argtypes = [vp, ctypes.c_int, ctypes.c_int]
        L.vie_jm_get_route.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
        L.vie_jm_rhs.argtypes = [vp, vp, vp, vp]
        L.vie_jm_matvec.argtypes = [vp, vp, vp]
        L.vie_jm_matvec_c64.argtypes = [vp, vp, vp]
        L.vie_jm_residual.argtypes = [vp, vp, vp, vp]
        L.vie_jm_solve.argtypes = [vp, vp, vp, ctypes.c_double, ctypes.POINTER(SolveOpts),
                                   ctypes.POINTER(SolveInfo)]
        _lib = L
    return _lib


def _check(code: int, plan=None):
    if code != VIE_OK:
        msg = lib().vie_last_error(plan).decode()
        raise VieError(code, msg)


def _grid(n: Sequence[int]):
    return (ctypes.c_int * 3)(*[int(v) for v in n])


def green_table(grid: Sequence[int], kappa: float, nthreads: int = 0) -> np.ndarray:
    """Host FP64 Toeplitz table N^{ab}(m), shape (6, n1, n2, n3), components xx xy xz yy yz zz."""
    out = np.empty((6,) + tuple(int(v) for v in grid), dtype=np.complex128)
    _check(lib().vie_green_table(_grid(grid), float(kappa), out.ctypes.data, int(nthreads)))
    return out


def curl_table(grid: Sequence[int], kappa: float, nthreads: int = 0) -> np.ndarray:
    """Host FP64 table of K = curl S, shape (3, n1, n2, n3), components xy xz yz (vie_curl_table)."""
    out = np.empty((3,) + tuple(int(v) for v in grid), dtype=np.complex128)
    _check(lib().vie_curl_table(_grid(grid), float(kappa), out.ctypes.data, int(nthreads)))
    return out


def _ptr(t, dtype, numel: int, name: str):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
    return ctypes.c_void_p(t.data_ptr())


class Plan:
    """Operator I - M_eps N on one grid (see include/vie.h)."""

    def __init__(self, grid: Sequence[int], h: float, k0: float, eps_b: float, fp32: bool = True,
                 stream=None):
        import torch
        self.n = tuple(int(v) for v in grid)
        self.N = self.n[0] * self.n[1] * self.n[2]
        self.h, self.k0, self.eps_b = float(h), float(k0), float(eps_b)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        handle = ctypes.c_void_p()
        flags = VIE_WITH_FP32 if fp32 else VIE_FP64
        code = lib().vie_plan(ctypes.byref(handle), _grid(self.n), self.h, self.k0, self.eps_b, flags,
                              ctypes.c_void_p(stream.cuda_stream))
        _check(code, None)
        self._h = handle

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            lib().vie_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_contrast(self, eps):
        import torch
        _check(lib().vie_set_contrast(self._h, _ptr(eps, torch.complex128, self.N, "eps")), self._h)

    def contrast(self, out=None):
        import torch
        if out is None:
            out = torch.empty(self.n, dtype=torch.complex128, device="cuda")
        _check(lib().vie_get_contrast(self._h, _ptr(out, torch.complex128, self.N, "chi")), self._h)
        return out

    def rhs(self, e_inc, out=None):
        import torch
        if out is None:
            out = torch.empty_like(e_inc)
        _check(lib().vie_rhs(self._h, _ptr(e_inc, torch.complex128, 3 * self.N, "e_inc"),
                             _ptr(out, torch.complex128, 3 * self.N, "b")), self._h)
        return out

    def matvec(self, x, y=None):
        import torch
        if y is None:
            y = torch.empty_like(x)
        _check(lib().vie_matvec(self._h, _ptr(x, torch.complex128, 3 * self.N, "x"),
                                _ptr(y, torch.complex128, 3 * self.N, "y")), self._h)
        return y

    def matvec_c64(self, x, y=None):
        import torch
        if y is None:
            y = torch.empty_like(x)
        _check(lib().vie_matvec_c64(self._h, _ptr(x, torch.complex64, 3 * self.N, "x"),
                                    _ptr(y, torch.complex64, 3 * self.N, "y")), self._h)
        return y

    def residual(self, x, b, r=None):
        import torch
        if r is None:
            r = torch.empty_like(b)
        _check(lib().vie_residual(self._h, _ptr(x, torch.complex128, 3 * self.N, "x"),
                                  _ptr(b, torch.complex128, 3 * self.N, "b"),
                                  _ptr(r, torch.complex128, 3 * self.N, "r")), self._h)
        return r

    def profile_matvec(self, x, y, reps: int, precision: int = 0):
        """Average per-pass and per-product durations (ms) over reps products, HIP events."""
        import torch
        dt = torch.complex128 if precision == 0 else torch.complex64
        ms = (ctypes.c_double * 3)()
        tot = ctypes.c_double()
        _check(lib().vie_profile_matvec(self._h, int(precision), _ptr(x, dt, 3 * self.N, "x"),
                                        _ptr(y, dt, 3 * self.N, "y"), int(reps), ms, ctypes.byref(tot)),
               self._h)
        return list(ms), tot.value

    def set_preconditioner(self, net):
        _check(lib().vie_set_preconditioner(self._h, net.handle if net is not None else None), self._h)
        self._net = net

    def tune(self, precision: int = 0) -> dict:
        """Launch shapes in use (vie_get_tune)."""
        xv, zp = ctypes.c_int(), ctypes.c_int()
        _check(lib().vie_get_tune(self._h, int(precision), ctypes.byref(xv), ctypes.byref(zp)), self._h)
        return {"xy_variant": xv.value, "z_pencils": zp.value}

    def set_tune(self, precision: int, xy_variant: int, z_pencils: int = 0):
        """Force launch shapes (vie_set_tune)."""
        _check(lib().vie_set_tune(self._h, int(precision), int(xy_variant), int(z_pencils)), self._h)

    def build_circulant(self, fp64: bool = False) -> dict:
        """Block-circulant preconditioner of the current contrast (vie_circulant_build)."""
        info = CirculantInfo()
        _check(lib().vie_circulant_build(self._h, 1 if fp64 else 0, ctypes.byref(info)), self._h)
        return info.as_dict()

    def apply_circulant(self, r, z=None):
        """z = W^{-1} r (vie_circulant_apply)."""
        import torch
        if z is None:
            z = torch.empty_like(r)
        _check(lib().vie_circulant_apply(self._h, _ptr(r, torch.complex128, 3 * self.N, "r"),
                                         _ptr(z, torch.complex128, 3 * self.N, "z")), self._h)
        return z

    def solve(self, b, x=None, tol: float = 1e-8, restart: int = 50, maxit: int = 10000,
              precision: int = 0, use_x0: bool = False, inner_restart: int = 20,
              inner_tol: float = 1e-4, raise_on_noconv: bool = False, stall_restarts: int = 0):
        """GMRES(restart) (precision 0), FP32-inner / FP64-outer FGMRES (1), learned (2),
        circulant-preconditioned FGMRES (3, after build_circulant) or the network
        correcting the circulant (4, after build_circulant and set_preconditioner).
        stall_restarts = k > 0 stops once k restarts in a row gain less than 0.1 % of
        the true residual (the mixed tiers hand over to FP64 GMRES first).

        Returns (x, info dict).  info['status'] is VIE_OK or VIE_ENOCONV."""
        import torch
        if x is None:
            x = torch.zeros_like(b)
        opts = SolveOpts(int(restart), int(maxit), int(bool(use_x0)), int(precision), int(inner_restart),
                         float(inner_tol), 0, int(stall_restarts))
        info = SolveInfo()
        code = lib().vie_solve(self._h, _ptr(b, torch.complex128, 3 * self.N, "b"),
                               _ptr(x, torch.complex128, 3 * self.N, "x"), float(tol), ctypes.byref(opts),
                               ctypes.byref(info))
        if code not in (VIE_OK, VIE_ENOCONV) or (raise_on_noconv and code != VIE_OK):
            _check(code, self._h)
        return x, info.as_dict()

    def solve_noalloc(self, b, x=None, tol: float = 1e-8, restart: int = 50, maxit: int = 10000,
                      precision: int = 0, use_x0: bool = False):
        """vie_solve_noalloc: the same solve with no allocation during the call (precision 0
        or 3), its workspace in the library's static scratch array.  Returns (x, info dict)."""
        import torch
        if x is None:
            x = torch.zeros_like(b)
        opts = SolveOpts(int(restart), int(maxit), int(bool(use_x0)), int(precision), 20, 1e-4, 0)
        info = SolveInfo()
        code = lib().vie_solve_noalloc(self._h, _ptr(b, torch.complex128, 3 * self.N, "b"),
                                       _ptr(x, torch.complex128, 3 * self.N, "x"), float(tol), ctypes.byref(opts),
                                       ctypes.byref(info))
        if code not in (VIE_OK, VIE_ENOCONV):
            _check(code, self._h)
        return x, info.as_dict()

    # ---- JM-VIE: electric and magnetic currents, 6N values (see include/vie.h)
    def jm_enable(self):
        """Spectrum of K = curl S and the JM buffers; mu_r = 1 (vie_jm_enable)."""
        _check(lib().vie_jm_enable(self._h), self._h)

    def jm_route(self, precision: int = 0) -> bool:
        """True when the JM cross-section pass runs fused in LDS (vie_jm_get_route)."""
        v = ctypes.c_int()
        _check(lib().vie_jm_get_route(self._h, int(precision), ctypes.byref(v)), self._h)
        return bool(v.value)

    def set_jm_route(self, precision: int, fused: bool):
        """Force the fused or the through-HBM cross-section pass (vie_jm_set_route)."""
        _check(lib().vie_jm_set_route(self._h, int(precision), int(bool(fused))), self._h)

    def set_permeability(self, mu_r):
        """Relative permeability per voxel, device complex128 of N values."""
        import torch
        _check(lib().vie_jm_set_permeability(self._h, _ptr(mu_r, torch.complex128, self.N, "mu_r")), self._h)

    def jm_rhs(self, e_inc, etah_inc, out=None):
        """b = h^{3/2} (M_eps e_inc, M_mu eta h_inc), 6N values (vie_jm_rhs)."""
        import torch
        if out is None:
            out = torch.empty(6 * self.N, dtype=torch.complex128, device=e_inc.device)
        _check(lib().vie_jm_rhs(self._h, _ptr(e_inc, torch.complex128, 3 * self.N, "e_inc"),
                                _ptr(etah_inc, torch.complex128, 3 * self.N, "etah_inc"),
                                _ptr(out, torch.complex128, 6 * self.N, "b")), self._h)
        return out

    def jm_matvec(self, x, y=None):
        import torch
        if y is None:
            y = torch.empty_like(x)
        _check(lib().vie_jm_matvec(self._h, _ptr(x, torch.complex128, 6 * self.N, "x"),
                                   _ptr(y, torch.complex128, 6 * self.N, "y")), self._h)
        return y

    def jm_matvec_c64(self, x, y=None):
        import torch
        if y is None:
            y = torch.empty_like(x)
        _check(lib().vie_jm_matvec_c64(self._h, _ptr(x, torch.complex64, 6 * self.N, "x"),
                                       _ptr(y, torch.complex64, 6 * self.N, "y")), self._h)
        return y

    def jm_residual(self, x, b, r=None):
        import torch
        if r is None:
            r = torch.empty_like(b)
        _check(lib().vie_jm_residual(self._h, _ptr(x, torch.complex128, 6 * self.N, "x"),
                                     _ptr(b, torch.complex128, 6 * self.N, "b"),
                                     _ptr(r, torch.complex128, 6 * self.N, "r")), self._h)
        return r

    def jm_solve(self, b, x=None, tol: float = 1e-8, restart: int = 50, maxit: int = 10000, precision: int = 0,
                 use_x0: bool = False, inner_restart: int = 20, inner_tol: float = 1e-4):
        """GMRES(restart) (precision 0) or FP32-inner / FP64-outer FGMRES (1) on the 6N
        unknowns (vie_jm_solve).  Returns (x, info dict)."""
        import torch
        if x is None:
            x = torch.zeros_like(b)
        opts = SolveOpts(int(restart), int(maxit), int(bool(use_x0)), int(precision), int(inner_restart),
                         float(inner_tol), 0)
        info = SolveInfo()
        code = lib().vie_jm_solve(self._h, _ptr(b, torch.complex128, 6 * self.N, "b"),
                                  _ptr(x, torch.complex128, 6 * self.N, "x"), float(tol), ctypes.byref(opts),
                                  ctypes.byref(info))
        if code not in (VIE_OK, VIE_ENOCONV):
            _check(code, self._h)
        return x, info.as_dict()


def solve_batch(plans, bs, xs=None, tol: float = 1e-8, restart: int = 50, maxit: int = 10000,
                precision: int = 0, use_x0: bool = False, inner_restart: int = 20, inner_tol: float = 1e-4,
                use_graph: bool = True):
    """Solve len(plans) systems together (vie_solve_batch).  Returns (xs, infos, status)."""
    import torch
    n = len(plans)
    if xs is None:
        xs = [torch.zeros_like(b) for b in bs]
    P = (ctypes.c_void_p * n)(*[p.handle for p in plans])
    Bp = (ctypes.c_void_p * n)(*[_ptr(b, torch.complex128, 3 * p.N, "b").value for b, p in zip(bs, plans)])
    Xp = (ctypes.c_void_p * n)(*[_ptr(x, torch.complex128, 3 * p.N, "x").value for x, p in zip(xs, plans)])
    opts = SolveOpts(int(restart), int(maxit), int(bool(use_x0)), int(precision), int(inner_restart),
                     float(inner_tol), int(bool(use_graph)))
    infos = (SolveInfo * n)()
    code = lib().vie_solve_batch(P, Bp, Xp, n, float(tol), ctypes.byref(opts), infos)
    if code not in (VIE_OK, VIE_ENOCONV):
        raise VieError(code, "vie_solve_batch failed")
    return xs, [i.as_dict() for i in infos], code


class Net:
    """The learned preconditioner network (see vie_net_* in include/vie.h)."""

    def __init__(self, grid: Sequence[int], seed: int = 0, stream=None):
        import torch
        self.n = tuple(int(v) for v in grid)
        self.N = self.n[0] * self.n[1] * self.n[2]
        if stream is None:
            stream = torch.cuda.current_stream()
        h = ctypes.c_void_p()
        code = lib().vie_net_create(ctypes.byref(h), _grid(self.n), int(seed), ctypes.c_void_p(stream.cuda_stream))
        if code != VIE_OK:
            raise VieError(code, "vie_net_create failed")
        self._h = h

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            lib().vie_net_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def num_params(self) -> int:
        c = ctypes.c_size_t()
        lib().vie_net_num_params(self._h, ctypes.byref(c))
        return c.value

    def get_params(self) -> np.ndarray:
        out = np.empty(self.num_params(), dtype=np.float32)
        if lib().vie_net_get_params(self._h, out.ctypes.data, out.size) != VIE_OK:
            raise VieError(VIE_EDEVICE, "vie_net_get_params failed")
        return out

    def set_params(self, w: np.ndarray):
        w = np.ascontiguousarray(w, dtype=np.float32)
        if lib().vie_net_set_params(self._h, w.ctypes.data, w.size) != VIE_OK:
            raise VieError(VIE_EINVAL, "vie_net_set_params failed")

    def get_state(self):
        """Training state (vie_net_get_state): (weights, Adam m, Adam v, step)."""
        n = self.num_params()
        buf = np.empty(3 * n, dtype=np.float32)
        step = ctypes.c_int()
        if lib().vie_net_get_state(self._h, buf.ctypes.data, n, ctypes.byref(step)) != VIE_OK:
            raise VieError(VIE_EDEVICE, "vie_net_get_state failed")
        return buf[:n].copy(), buf[n:2 * n].copy(), buf[2 * n:].copy(), step.value

    def set_state(self, w: np.ndarray, m: np.ndarray, v: np.ndarray, step: int):
        """Restore a training state (vie_net_set_state)."""
        n = self.num_params()
        buf = np.concatenate([np.asarray(a, dtype=np.float32).ravel() for a in (w, m, v)])
        if buf.size != 3 * n:
            raise VieError(VIE_EINVAL, "state of the wrong size")
        code = lib().vie_net_set_state(self._h, buf.ctypes.data, n, int(step))
        if code != VIE_OK:
            raise VieError(code, (lib().vie_net_last_error(self._h) or b"").decode())

    def get_grads(self) -> np.ndarray:
        """FP32 weight gradients of the last train_step (vie_net_get_grads)."""
        out = np.empty(self.num_params(), dtype=np.float32)
        if lib().vie_net_get_grads(self._h, out.ctypes.data, out.size) != VIE_OK:
            raise VieError(VIE_EDEVICE, "vie_net_get_grads failed")
        return out

    def apply(self, r, chi, z=None):
        import torch
        if z is None:
            z = torch.empty_like(r)
        code = lib().vie_net_apply(self._h, _ptr(r, torch.complex128, 3 * self.N, "r"),
                                   _ptr(chi, torch.complex128, self.N, "chi"),
                                   _ptr(z, torch.complex128, 3 * self.N, "z"))
        if code != VIE_OK:
            raise VieError(code, "vie_net_apply failed")
        return z

    def apply_base(self, r, w, chi, z=None):
        """z = w + net(r, chi, w) (vie_net_apply_base): the network's correction of w."""
        import torch
        if z is None:
            z = torch.empty_like(r)
        code = lib().vie_net_apply_base(self._h, _ptr(r, torch.complex128, 3 * self.N, "r"),
                                        _ptr(w, torch.complex128, 3 * self.N, "w"),
                                        _ptr(chi, torch.complex128, self.N, "chi"),
                                        _ptr(z, torch.complex128, 3 * self.N, "z"))
        if code != VIE_OK:
            raise VieError(code, "vie_net_apply_base failed")
        return z

    def train_step_base(self, rs, ws, chis, targets, lr: float) -> float:
        """One Adam step on the base-vector form (vie_net_train_step_base)."""
        import torch
        n = len(rs)
        R = (ctypes.c_void_p * n)(*[_ptr(r, torch.complex128, 3 * self.N, "r").value for r in rs])
        Wb = (ctypes.c_void_p * n)(*[_ptr(w, torch.complex128, 3 * self.N, "w").value for w in ws])
        C = (ctypes.c_void_p * n)(*[_ptr(c, torch.complex128, self.N, "chi").value for c in chis])
        T = (ctypes.c_void_p * n)(*[_ptr(t, torch.complex128, 3 * self.N, "target").value for t in targets])
        loss = ctypes.c_double()
        code = lib().vie_net_train_step_base(self._h, n, R, Wb, C, T, float(lr), ctypes.byref(loss))
        if code != VIE_OK:
            raise VieError(code, "vie_net_train_step_base failed")
        return loss.value

    def train_step(self, rs, chis, targets, lr: float) -> float:
        import torch
        n = len(rs)
        R = (ctypes.c_void_p * n)(*[_ptr(r, torch.complex128, 3 * self.N, "r").value for r in rs])
        C = (ctypes.c_void_p * n)(*[_ptr(c, torch.complex128, self.N, "chi").value for c in chis])
        T = (ctypes.c_void_p * n)(*[_ptr(t, torch.complex128, 3 * self.N, "target").value for t in targets])
        loss = ctypes.c_double()
        code = lib().vie_net_train_step(self._h, n, R, C, T, float(lr), ctypes.byref(loss))
        if code != VIE_OK:
            raise VieError(code, "vie_net_train_step failed")
        return loss.value


def conv_test(mode: int, dims, taps: int, cin: int, cout: int, x, w, relu: bool = False):
    """Diagnostic single convolution layer (vie_nn_conv_test) on FP32 device tensors."""
    import torch
    V = int(np.prod(dims))
    if mode == 0:
        out = torch.empty((V, cout), dtype=torch.float32, device=x.device)
    elif mode == 1:
        out = torch.empty((V, cin), dtype=torch.float32, device=x.device)
    else:
        out = torch.empty((taps, cout, cin), dtype=torch.float32, device=x.device)
    code = lib().vie_nn_conv_test(int(mode), _grid(dims), int(taps), int(cin), int(cout),
                                  ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(w.data_ptr()),
                                  ctypes.c_void_p(out.data_ptr()), int(bool(relu)),
                                  ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    if code != VIE_OK:
        raise VieError(code, "vie_nn_conv_test failed")
    return out


def nn_op_test(op: int, fine_dims, C: int, x, mask=None, acc=None):
    """Diagnostic pooling (0) / pooling gradient (1) / upsampling (2) / upsampling
    gradient (3) kernel on FP32 device tensors (vie_nn_op_test)."""
    import torch
    Vf = int(np.prod(fine_dims))
    nout = (Vf // 8 if op in (0, 3) else Vf) * C
    out = torch.empty(nout, dtype=torch.float32, device=x.device)
    ptr = lambda t: ctypes.c_void_p(t.data_ptr() if t is not None else 0)
    code = lib().vie_nn_op_test(int(op), _grid(fine_dims), int(C), ptr(x), ptr(mask), ptr(acc), ptr(out),
                                ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    if code != VIE_OK:
        raise VieError(code, "vie_nn_op_test failed")
    return out


def nn_adam_test(w, m, v, g, t: int, lr: float):
    """Diagnostic Adam step t on FP32 device tensors, in place (vie_nn_adam_test)."""
    import torch
    code = lib().vie_nn_adam_test(ctypes.c_long(w.numel()), ctypes.c_void_p(w.data_ptr()),
                                  ctypes.c_void_p(m.data_ptr()), ctypes.c_void_p(v.data_ptr()),
                                  ctypes.c_void_p(g.data_ptr()), int(t), ctypes.c_float(lr),
                                  ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    if code != VIE_OK:
        raise VieError(code, "vie_nn_adam_test failed")
