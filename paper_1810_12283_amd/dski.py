"""Python binding of libdski.so (ctypes; argument marshalling only).

Every computation runs in the HIP library.  PyTorch supplies device memory
(tensor data pointers) and the current HIP stream, nothing else.  Blocks of R
N-vectors are torch tensors of shape (R, N), contiguous: row r is vector r,
i.e. the column-major N x R layout of the C ABI with ld = N.

If the library is missing or cannot be loaded every call raises: there is no
fallback.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from typing import Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdski.so")

OK, NOT_CONVERGED, RANK_TRUNCATED = 0, 1, 2
INTERP = {"cubic": 0, "quintic": 1}   # DSKI_INTERP_CUBIC, DSKI_INTERP_QUINTIC
KERNEL = {"se": 0, "spline": 1}       # DSKI_KERNEL_SE, DSKI_KERNEL_SPLINE
SCATTER_VARIANTS = 7                  # 0-5 bitwise equal; 6 the grouped 3-D form
GATHER_VARIANTS = 3
_STATUS = {0: "OK", 1: "NOT_CONVERGED", 2: "RANK_TRUNCATED", -1: "EINVAL", -2: "ENOMEM",
           -3: "EHIP", -4: "EBREAKDOWN", -5: "ENOTSUP"}


class DSKIError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None

vp = C.c_void_p
ip = C.POINTER(C.c_int)
dp = C.POINTER(C.c_double)
_SIGS = {
    "dski_last_error": (C.c_char_p, []),
    "dski_version": (C.c_char_p, []),
    "dski_plan_create": (C.c_int, [C.POINTER(vp), C.c_int, C.c_int, vp, ip, dp, dp, C.c_int, vp]),
    "dski_plan_destroy": (C.c_int, [vp]),
    "dskip_plan_create": (C.c_int, [C.POINTER(vp), C.c_int, C.c_int, vp, C.c_int, C.c_int, C.c_uint64,
                                    dp, dp, dp, vp]),
    "dskip_plan_info": (C.c_int, [vp, ip, ip, ip, ip]),
    "dski_plan_info": (C.c_int, [vp, ip, ip, ip, C.POINTER(C.c_longlong), ip, ip, dp, dp]),
    "dski_set_hypers": (C.c_int, [vp, dp, C.c_double, C.c_double, C.c_double, vp]),
    "dski_mvm": (C.c_int, [vp, C.c_int, vp, C.c_int, vp, C.c_int, vp]),
    "dski_mvm_dtheta": (C.c_int, [vp, C.c_int, C.c_int, vp, C.c_int, vp, C.c_int, vp]),
    "dski_predict_grid": (C.c_int, [vp, vp, vp, vp]),
    "dski_predict": (C.c_int, [vp, vp, C.c_int, vp, vp, vp]),
    "dski_predict_var": (C.c_int, [vp, vp, C.c_int, vp, vp, vp]),
    "dski_expected_improvement": (C.c_int, [C.c_int, vp, C.c_int, vp, C.c_double, C.c_double, vp, ip, vp, vp]),
    "dski_active_subspace": (C.c_int, [C.c_int, C.c_int, vp, C.c_int, C.c_int, vp, vp, vp]),
    "dski_active_project": (C.c_int, [C.c_int, C.c_int, C.c_int, vp, vp, C.c_int, vp, vp, vp, vp]),
    "dski_predict_var_probes": (C.c_int, [vp, vp, C.c_int, vp, C.c_int, vp, C.c_double, C.c_int, vp, vp]),
    "dski_permute": (C.c_int, [vp, C.c_int, C.c_int, vp, C.c_int, vp, C.c_int, vp]),
    "dski_tile_order": (C.c_int, [vp, ip]),
    "dski_mvm_tiled": (C.c_int, [vp, C.c_int, vp, C.c_int, vp, C.c_int, vp]),
    "dski_mvm_tiled_noalloc": (C.c_int, [vp, C.c_int, vp, C.c_int, vp, C.c_int, vp]),
    "pivchol_build": (C.c_int, [vp, C.c_int, C.POINTER(vp), ip, ip, vp]),
    "pivchol_build_forced": (C.c_int, [vp, C.c_int, ip, C.POINTER(vp), ip, ip, vp]),
    "dski_precond_destroy": (C.c_int, [vp]),
    "dski_precond_apply": (C.c_int, [vp, C.c_int, vp, C.c_int, vp, C.c_int, vp]),
    "dski_precond_logdet": (C.c_int, [vp, dp]),
    "dski_precond_factor": (C.c_int, [vp, vp, C.c_int, vp]),
    "pcg_solve": (C.c_int, [vp, vp, C.c_int, vp, C.c_int, vp, C.c_int, dp, C.c_int, ip, dp, vp, vp]),
    "slq_logdet": (C.c_int, [vp, vp, C.c_int, C.c_int, C.c_double, C.c_int, C.c_uint64, dp, dp, vp]),
    "mll_and_grad": (C.c_int, [vp, vp, C.c_int, vp, C.c_int, C.c_uint64, C.c_double, C.c_int,
                               dp, dp, dp, ip, vp]),
    "dski_rademacher": (C.c_int, [C.c_uint64, C.c_int, C.c_int, C.c_int, vp, C.c_int, vp]),
    "dski_lanczos_quad_log": (C.c_double, [dp, dp, C.c_int, ip]),
    "dski_plan_set_precision": (C.c_int, [vp, C.c_int]),
    "dski_set_kernel": (C.c_int, [vp, C.c_int, vp]),
    "dski_mvm_stage": (C.c_int, [vp, C.c_int, C.c_int, vp, C.c_int, vp, C.c_int, vp]),
    "dski_autotune": (C.c_int, [vp, C.c_int, dp, vp]),
    "dski_autotune_cached": (C.c_int, [vp, C.c_int, C.c_char_p, ip, dp, vp]),
    "dski_set_variants": (C.c_int, [vp, C.c_int, C.c_int]),
    "dski_set_graph": (C.c_int, [vp, C.c_int]),
    "dski_set_kuu_variant": (C.c_int, [vp, C.c_int, C.c_int]),
    "mlp_create": (C.c_int, [C.POINTER(vp), C.c_int, C.c_int, C.c_int, vp, vp]),
    "mlp_destroy": (C.c_int, [vp]),
    "mlp_num_params": (C.c_int, [vp, ip]),
    "mlp_get_params": (C.c_int, [vp, vp, vp]),
    "mlp_forward": (C.c_int, [vp, C.c_int, vp, vp, vp]),
    "mlp_jvp": (C.c_int, [vp, C.c_int, vp, vp, vp, vp]),
    "mlp_backward": (C.c_int, [vp, C.c_int, vp, vp, vp, C.c_float, dp, vp]),
    "mlp_step": (C.c_int, [vp, C.c_float, C.c_float, C.c_float, C.c_float, vp]),
    "dski_mvm_f64": (C.c_int, [vp, C.c_int, vp, C.c_int, vp, C.c_int, vp]),
    "dski_mvm_dtheta_f64": (C.c_int, [vp, C.c_int, C.c_int, vp, C.c_int, vp, C.c_int, vp]),
    "dski_permute_f64": (C.c_int, [vp, C.c_int, C.c_int, vp, C.c_int, vp, C.c_int, vp]),
    "dski_mvm_tiled_f64": (C.c_int, [vp, C.c_int, vp, C.c_int, vp, C.c_int, vp]),
    "dski_precond_apply_f64": (C.c_int, [vp, C.c_int, vp, C.c_int, vp, C.c_int, vp]),
    "pcg_solve_f64": (C.c_int, [vp, vp, C.c_int, vp, C.c_int, vp, C.c_int, dp, C.c_int, ip, dp, vp, vp]),
    "mll_and_grad_f64": (C.c_int, [vp, vp, C.c_int, vp, C.c_int, C.c_uint64, C.c_double, C.c_int,
                                   dp, dp, dp, ip, vp]),
    "mll_and_grad_warm": (C.c_int, [vp, vp, C.c_int, vp, C.c_int, C.c_uint64, C.c_double, C.c_int, vp, vp,
                                    dp, dp, dp, ip, vp]),
}

EXPORTS = tuple(_SIGS)


def lib():
    """Load libdski.so (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built: run `python -m paper_1810_12283_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def last_error() -> str:
    return lib().dski_last_error().decode()


def _check(status, what):
    if status < 0:
        raise DSKIError(status, f"{what}: {last_error()}")
    return status


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return vp(stream.cuda_stream)


def _dptr(t: torch.Tensor):
    return vp(t.data_ptr())


def _fn(name, V):
    """The FP32 entry point or its *_f64 twin, by the tensor's dtype."""
    return getattr(lib(), name + ("_f64" if V.dtype == torch.float64 else ""))


def _arr(vals, ctype):
    a = (ctype * len(vals))(*vals)
    return a


def _block(V: torch.Tensor, N: int, name: str) -> torch.Tensor:
    if not V.is_cuda or V.dtype not in (torch.float32, torch.float64):
        raise TypeError(f"{name} must be a CUDA float32 or float64 tensor")
    if V.dim() == 1:
        V = V[None, :]
    if V.shape[-1] != N or not V.is_contiguous():
        raise ValueError(f"{name} must be contiguous with shape (R, {N})")
    return V


class Plan:
    """A D-SKI operator on fixed points and grid (owns a dski_plan)."""

    def __init__(self, X: torch.Tensor, grid_m: Sequence[int], lo=None, hi=None, stream=None,
                 interp: str = "cubic", kernel: str = "se"):
        """interp: "cubic" (Keys, 4 nodes per axis) or "quintic" (Meijering,
        6 nodes per axis); kernel: "se" (squared exponential) or "spline"
        (thin-plate spline, multi-level Toeplitz K_UU)."""
        L = lib()
        if interp not in INTERP:
            raise ValueError(f"interp must be one of {sorted(INTERP)}")
        if kernel not in KERNEL:
            raise ValueError(f"kernel must be one of {sorted(KERNEL)}")
        if not X.is_cuda or X.dtype != torch.float64 or X.dim() != 2:
            raise TypeError("X must be a CUDA float64 tensor of shape (n, d)")
        X = X.contiguous()
        n, d = X.shape
        self.n, self.d, self.N = n, d, n * (d + 1)
        h = vp()
        m = _arr([int(v) for v in grid_m], C.c_int)
        lo_a = _arr([float(v) for v in lo], C.c_double) if lo is not None else None
        hi_a = _arr([float(v) for v in hi], C.c_double) if hi is not None else None
        _check(L.dski_plan_create(C.byref(h), n, d, _dptr(X), m, lo_a, hi_a, INTERP[interp], _stream(stream)),
               "dski_plan_create")
        self.interp = interp
        self._h = h
        if kernel != "se":
            _check(L.dski_set_kernel(h, KERNEL[kernel], _stream(stream)), "dski_set_kernel")
        self.kernel = kernel
        self._h = h
        self._info()

    def _info(self):
        L = lib()
        if getattr(self, "kind", "dski") == "dskip":
            m1, r, ka, kb = C.c_int(), C.c_int(), C.c_int(), C.c_int()
            _check(L.dskip_plan_info(self._h, C.byref(m1), C.byref(r), C.byref(ka), C.byref(kb)),
                   "dskip_plan_info")
            self.m_1d, self.rank_r, self.root_ranks = m1.value, r.value, (ka.value, kb.value)
            self.grid_nodes = 0
            return
        n, d, N = C.c_int(), C.c_int(), C.c_int()
        M = C.c_longlong()
        m = (C.c_int * 3)()
        Lf = (C.c_int * 3)()
        h = (C.c_double * 3)()
        lo = (C.c_double * 3)()
        _check(L.dski_plan_info(self._h, C.byref(n), C.byref(d), C.byref(N), C.byref(M), m, Lf, h, lo),
               "dski_plan_info")
        self.grid_nodes = M.value
        self.grid_m = [m[i] for i in range(self.d)]
        self.fft_len = [Lf[i] for i in range(self.d)]
        self.h = [h[i] for i in range(self.d)]
        self.grid_lo = [lo[i] for i in range(self.d)]

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().dski_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    kind = "dski"

    def set_hypers(self, log_ell, log_s, log_sigma_f, log_sigma_g, stream=None):
        le = np.broadcast_to(np.asarray(log_ell, dtype=np.float64), (self.d,))
        a = _arr([float(v) for v in le], C.c_double)
        _check(lib().dski_set_hypers(self._h, a, float(log_s), float(log_sigma_f), float(log_sigma_g),
                                     _stream(stream)), "dski_set_hypers")

    def mvm(self, V: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        V = _block(V, self.N, "V")
        Y = torch.empty_like(V) if out is None else out
        _check(_fn("dski_mvm", V)(self._h, V.shape[0], _dptr(V), self.N, _dptr(Y), self.N, _stream(stream)),
               "dski_mvm")
        return Y

    def mvm_tiled(self, V: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        V = _block(V, self.N, "V")
        Y = torch.empty_like(V) if out is None else out
        _check(_fn("dski_mvm_tiled", V)(self._h, V.shape[0], _dptr(V), self.N, _dptr(Y), self.N,
                                    _stream(stream)), "dski_mvm_tiled")
        return Y

    def mvm_tiled_noalloc(self, V: torch.Tensor, out: torch.Tensor, stream=None) -> torch.Tensor:
        """dski_mvm_tiled with the library's fixed grid workspace (no device
        allocation inside the call): FP32 tile-ordered V (R x N) into out."""
        V = _block(V, self.N, "V")
        if V.dtype != torch.float32 or out.dtype != torch.float32 or out.shape != V.shape or not out.is_cuda:
            raise TypeError("V and out must be CUDA float32 tensors of the same shape (R, N)")
        _check(lib().dski_mvm_tiled_noalloc(self._h, V.shape[0], _dptr(V), self.N, _dptr(out), self.N,
                                            _stream(stream)), "dski_mvm_tiled_noalloc")
        return out

    def mvm_stage(self, stage: int, V: torch.Tensor, Y: Optional[torch.Tensor] = None, stream=None):
        """One stage of the tile-ordered MVM (0 scatter, 1 K_UU, 2 gather into Y)."""
        V = _block(V, self.N, "V")
        yp = _dptr(Y) if Y is not None else None
        _check(lib().dski_mvm_stage(self._h, int(stage), V.shape[0], _dptr(V), self.N, yp, self.N,
                                    _stream(stream)), "dski_mvm_stage")
        return Y

    def predict_grid(self, alpha: torch.Tensor, stream=None) -> torch.Tensor:
        """Grid vector g = K_UU S^T alpha (M doubles) for the posterior mean;
        alpha = K~^{-1} y, an FP64 CUDA N-vector in user order."""
        if not alpha.is_cuda or alpha.dtype != torch.float64 or alpha.numel() != self.N:
            raise TypeError("alpha must be a CUDA float64 tensor with N entries")
        alpha = alpha.contiguous()
        # D-SKIP plans have no single grid; the library refuses them (DSKI_ENOTSUP)
        m = getattr(self, "grid_m", None)
        g = torch.empty(int(np.prod(m)) if m is not None else 1, dtype=torch.float64, device=alpha.device)
        _check(lib().dski_predict_grid(self._h, _dptr(alpha), _dptr(g), _stream(stream)), "dski_predict_grid")
        return g

    def predict(self, g: torch.Tensor, Xs: torch.Tensor, stream=None) -> torch.Tensor:
        """Posterior means at the test points Xs (n* x d, FP64, CUDA): n* x (d + 1),
        column 0 the value, column 1 + p the derivative along axis p."""
        if not Xs.is_cuda or Xs.dtype != torch.float64 or Xs.dim() != 2 or Xs.shape[1] != self.d:
            raise TypeError("Xs must be a CUDA float64 tensor of shape (n*, d)")
        if not isinstance(g, torch.Tensor) or not g.is_cuda or g.dtype != torch.float64:
            raise TypeError("g must be the CUDA float64 grid vector of predict_grid")
        if self.grid_nodes and g.numel() != self.grid_nodes:
            raise ValueError(f"g has {g.numel()} entries; this plan's grid has {self.grid_nodes} nodes")
        Xs = Xs.contiguous()
        out = torch.empty((Xs.shape[0], self.d + 1), dtype=torch.float64, device=Xs.device)
        _check(lib().dski_predict(self._h, _dptr(g.contiguous()), Xs.shape[0], _dptr(Xs), _dptr(out),
                                  _stream(stream)), "dski_predict")
        return out

    def predict_var(self, pc: "Precond", Xs: torch.Tensor, stream=None) -> torch.Tensor:
        """Predictive variance of f at the test points Xs (n* x d, FP64, CUDA) with
        the preconditioner pc (built on this plan) standing in for K~: n* values."""
        if not Xs.is_cuda or Xs.dtype != torch.float64 or Xs.dim() != 2 or Xs.shape[1] != self.d:
            raise TypeError("Xs must be a CUDA float64 tensor of shape (n*, d)")
        Xs = Xs.contiguous()
        out = torch.empty(Xs.shape[0], dtype=torch.float64, device=Xs.device)
        _check(lib().dski_predict_var(self._h, pc.handle, Xs.shape[0], _dptr(Xs), _dptr(out), _stream(stream)),
               "dski_predict_var")
        return out

    def predict_var_probes(self, pc: "Precond", Xs: torch.Tensor, Zp: torch.Tensor, tol: float = 1e-8,
                           max_iter: int = 10000, stream=None):
        """Randomized predictive variance of f at Xs with the pivoted-Cholesky
        estimate as control variate; Zp (R x n*, FP64, CUDA) holds the probes.
        Returns (n* values, status): status 1 if a solve reached max_iter."""
        if not Xs.is_cuda or Xs.dtype != torch.float64 or Xs.dim() != 2 or Xs.shape[1] != self.d:
            raise TypeError("Xs must be a CUDA float64 tensor of shape (n*, d)")
        if not Zp.is_cuda or Zp.dtype != torch.float64 or Zp.dim() != 2 or Zp.shape[1] != Xs.shape[0]:
            raise TypeError("Zp must be a CUDA float64 tensor of shape (R, n*)")
        Xs, Zp = Xs.contiguous(), Zp.contiguous()
        out = torch.empty(Xs.shape[0], dtype=torch.float64, device=Xs.device)
        st = _check(lib().dski_predict_var_probes(self._h, pc.handle, Xs.shape[0], _dptr(Xs), Zp.shape[0],
                                                  _dptr(Zp), float(tol), int(max_iter), _dptr(out),
                                                  _stream(stream)), "dski_predict_var_probes")
        return out, st

    def mvm_dtheta(self, which: int, V: torch.Tensor, stream=None) -> torch.Tensor:
        V = _block(V, self.N, "V")
        Y = torch.empty_like(V)
        _check(_fn("dski_mvm_dtheta", V)(self._h, int(which), V.shape[0], _dptr(V), self.N, _dptr(Y), self.N,
                                     _stream(stream)), "dski_mvm_dtheta")
        return Y

    def permute(self, V: torch.Tensor, direction: int, stream=None) -> torch.Tensor:
        V = _block(V, self.N, "V")
        Y = torch.empty_like(V)
        _check(_fn("dski_permute", V)(self._h, int(direction), V.shape[0], _dptr(V), self.N, _dptr(Y), self.N,
                                  _stream(stream)), "dski_permute")
        return Y

    def autotune(self, R: int, stream=None, cache: Optional[str] = None) -> dict:
        """Time the kernel variants for this shape and keep the fastest; with
        cache (a file path) reuse the choice stored for this shape if there is
        one (the result then has cached=True and no timings)."""
        t = (C.c_double * 16)()
        if cache is None:
            _check(lib().dski_autotune(self._h, int(R), t, _stream(stream)), "dski_autotune")
            hit = False
        else:
            h = C.c_int()
            _check(lib().dski_autotune_cached(self._h, int(R), str(cache).encode(), C.byref(h), t, _stream(stream)),
                   "dski_autotune_cached")
            hit = bool(h.value)
        return {"scatter_us": [t[i] for i in range(SCATTER_VARIANTS)], "gather_us": [t[7], t[8], t[9]],
                "kuu_us": [[t[10 + 2 * a], t[11 + 2 * a]] for a in range(min(self.d, 3))], "cached": hit}

    def set_variants(self, scatter: int, gather: int = 0):
        _check(lib().dski_set_variants(self._h, int(scatter), int(gather)), "dski_set_variants")

    def set_kuu_variant(self, axis: int, variant: int):
        """K_UU factor of one axis: 0 FFT, 1 dense matrix-core product."""
        _check(lib().dski_set_kuu_variant(self._h, int(axis), int(variant)), "dski_set_kuu_variant")

    def set_graph(self, on: bool):
        """Replay PCG iterations from a captured HIP graph (default) or launch directly."""
        _check(lib().dski_set_graph(self._h, int(bool(on))), "dski_set_graph")

    def set_precision(self, bits: int):
        """Storage precision of the vectors slq_logdet creates (32 or 64)."""
        _check(lib().dski_plan_set_precision(self._h, int(bits)), "dski_plan_set_precision")

    def tile_order(self) -> np.ndarray:
        perm = (C.c_int * self.n)()
        _check(lib().dski_tile_order(self._h, perm), "dski_tile_order")
        return np.frombuffer(perm, dtype=np.int32).copy()

    def pivchol(self, k: int, stream=None, forced=None) -> "Precond":
        return Precond(self, k, stream, forced=forced)

    def pcg(self, B: torch.Tensor, precond: Optional["Precond"] = None, tol=1e-4, max_iter=10000,
            history=False, stream=None):
        """Returns (X, iters, relres, status, alpha_beta or None)."""
        B = _block(B, self.N, "B")
        R = B.shape[0]
        X = torch.empty(B.shape, dtype=torch.float64, device=B.device)
        tols = _arr([float(t) for t in np.broadcast_to(np.asarray(tol, dtype=np.float64), (R,))], C.c_double)
        iters = (C.c_int * R)()
        relres = (C.c_double * R)()
        ab = torch.zeros(2 * max_iter * R, dtype=torch.float64, device=B.device) if history else None
        st = _check(_fn("pcg_solve", B)(self._h, precond.handle if precond else None, R, _dptr(B), self.N,
                                    _dptr(X), self.N, tols, int(max_iter), iters, relres,
                                    _dptr(ab) if ab is not None else None, _stream(stream)), "pcg_solve")
        return X, list(iters), list(relres), st, ab

    def slq_logdet(self, precond: Optional["Precond"], num_probes: int, lanczos_steps: int = 0,
                   tol: float = 1e-4, max_iter: int = 10000, seed: int = 0x181012283, stream=None):
        ld, se = C.c_double(), C.c_double()
        _check(lib().slq_logdet(self._h, precond.handle if precond else None, int(num_probes),
                                int(lanczos_steps), float(tol), int(max_iter), C.c_uint64(seed),
                                C.byref(ld), C.byref(se), _stream(stream)), "slq_logdet")
        return ld.value, se.value

    def mll_and_grad(self, y: torch.Tensor, precond: Optional["Precond"] = None, k: int = 50,
                     num_probes: int = 16, seed: int = 0x181012283, tol: float = 1e-4,
                     max_iter: int = 10000, stream=None, x0: Optional[torch.Tensor] = None,
                     want_alpha: bool = False):
        """x0 (CUDA FP64, N values, user order) warm-starts the data solve and
        want_alpha returns alpha (as "alpha") for the next warm start; both
        need FP32 y (mll_and_grad_warm)."""
        y = _block(y, self.N, "y")
        mll, ld = C.c_double(), C.c_double()
        grad = (C.c_double * (self.d + 3))()
        iters = (C.c_int * (1 + num_probes))()
        alpha = None
        if x0 is not None or want_alpha:
            if y.dtype != torch.float32:
                raise TypeError("warm starts take an FP32 y")
            if x0 is not None and (not x0.is_cuda or x0.dtype != torch.float64 or x0.numel() != self.N):
                raise TypeError("x0 must be a CUDA float64 tensor with N entries")
            alpha = torch.empty(self.N, dtype=torch.float64, device=y.device) if want_alpha else None
            st = _check(lib().mll_and_grad_warm(self._h, precond.handle if precond else None, int(k), _dptr(y),
                                                int(num_probes), C.c_uint64(seed), float(tol), int(max_iter),
                                                _dptr(x0.contiguous()) if x0 is not None else None,
                                                _dptr(alpha) if alpha is not None else None, C.byref(mll), grad,
                                                C.byref(ld), iters, _stream(stream)), "mll_and_grad_warm")
        else:
            st = _check(_fn("mll_and_grad", y)(self._h, precond.handle if precond else None, int(k), _dptr(y),
                                           int(num_probes), C.c_uint64(seed), float(tol), int(max_iter),
                                           C.byref(mll), grad, C.byref(ld), iters, _stream(stream)),
                        "mll_and_grad")
        out = dict(mll=mll.value, grad=np.array(list(grad)), logdet=ld.value, iters=list(iters), status=st)
        if alpha is not None:
            out["alpha"] = alpha
        return out


class DskipPlan(Plan):
    """A D-SKIP operator (Hadamard product of Lanczos-compressed 1-D D-SKI
    factors, Sec. 3.2) on fixed points; works with the same solver calls."""

    kind = "dskip"

    def __init__(self, X: torch.Tensor, m_1d: int, rank_r: int, seed: int, log_ell, lo=None, hi=None,
                 stream=None):
        L = lib()
        if not X.is_cuda or X.dtype != torch.float64 or X.dim() != 2:
            raise TypeError("X must be a CUDA float64 tensor of shape (n, d)")
        X = X.contiguous()
        n, d = X.shape
        self.n, self.d, self.N = n, d, n * (d + 1)
        h = vp()
        le = np.broadcast_to(np.asarray(log_ell, dtype=np.float64), (d,))
        le_a = _arr([float(v) for v in le], C.c_double)
        lo_a = _arr([float(v) for v in lo], C.c_double) if lo is not None else None
        hi_a = _arr([float(v) for v in hi], C.c_double) if hi is not None else None
        _check(L.dskip_plan_create(C.byref(h), n, d, _dptr(X), int(m_1d), int(rank_r), int(seed) & (2**64 - 1),
                                   lo_a, hi_a, le_a, _stream(stream)), "dskip_plan_create")
        self._h = h
        self._info()


class MarginalLikelihood(torch.autograd.Function):
    """mll(theta) with theta = (log ell_1..log ell_d, log s, log sigma_f,
    log sigma_g) as a float64 tensor; the forward pass sets the hyper-parameters
    of `plan`, builds a rank-k preconditioner and calls mll_and_grad (adjoint
    MVMs on the device); the backward pass returns grad_output times the
    gradient computed there (eq. (1) and its derivatives).

        mll = MarginalLikelihood.apply(theta, plan, y, k, num_probes, seed, tol, max_iter)
    """

    @staticmethod
    def forward(ctx, theta, plan, y, k=50, num_probes=16, seed=0x181012283, tol=1e-4, max_iter=10000):
        th = theta.detach().double().cpu().numpy()
        d = plan.d
        if th.shape != (d + 3,):
            raise ValueError(f"theta must have d + 3 = {d + 3} entries")
        plan.set_hypers(th[:d], th[d], th[d + 1], th[d + 2])
        res = plan.mll_and_grad(y, None, k=k, num_probes=num_probes, seed=seed, tol=tol, max_iter=max_iter)
        ctx.save_for_backward(torch.tensor(res["grad"], dtype=theta.dtype, device=theta.device))
        return torch.tensor(res["mll"], dtype=theta.dtype, device=theta.device)

    @staticmethod
    def backward(ctx, grad_output):
        (g,) = ctx.saved_tensors
        return (grad_output * g,) + (None,) * 7


class Precond:
    """Pivoted-Cholesky preconditioner (owns a dski_precond)."""

    def __init__(self, plan: Plan, k: int, stream=None, forced=None):
        """forced: optional pivot sequence (k user-order N-indices) that replaces
        the greedy choice (pivchol_build_forced)."""
        self.plan = plan
        h = vp()
        rank = C.c_int()
        piv = (C.c_int * max(k, 1))()
        if forced is None:
            self.status = _check(lib().pivchol_build(plan.handle, int(k), C.byref(h), C.byref(rank), piv,
                                                     _stream(stream)), "pivchol_build")
        else:
            f = [int(v) for v in forced]
            if len(f) != k:
                raise ValueError(f"forced holds {len(f)} pivots, k = {k}")
            self.status = _check(lib().pivchol_build_forced(plan.handle, int(k), _arr(f, C.c_int), C.byref(h),
                                                            C.byref(rank), piv, _stream(stream)),
                                 "pivchol_build_forced")
        self._h = h
        self.rank = rank.value
        self.pivots = np.array([piv[i] for i in range(self.rank)], dtype=np.int64)

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().dski_precond_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def logdet(self) -> float:
        v = C.c_double()
        _check(lib().dski_precond_logdet(self._h, C.byref(v)), "dski_precond_logdet")
        return v.value

    def apply(self, Rm: torch.Tensor, stream=None) -> torch.Tensor:
        Rm = _block(Rm, self.plan.N, "R")
        Z = torch.empty_like(Rm)
        _check(_fn("dski_precond_apply", Rm)(self._h, Rm.shape[0], _dptr(Rm), self.plan.N, _dptr(Z), self.plan.N,
                                        _stream(stream)), "dski_precond_apply")
        return Z

    def factor(self, stream=None) -> torch.Tensor:
        """L as a (rank, N) float64 tensor (row j = column j of L, user order)."""
        out = torch.zeros((max(self.rank, 1), self.plan.N), dtype=torch.float64, device="cuda")
        _check(lib().dski_precond_factor(self._h, _dptr(out), self.plan.N, _stream(stream)),
               "dski_precond_factor")
        return out[: self.rank]


class Mlp:
    """The surrogate network on the device (owns a dski_mlp); parameters packed
    row-major as W1, b1, W2, b2, w3, b3 (FP32)."""

    def __init__(self, params: np.ndarray, F: int = 8, H: int = 128, J: int = 5, stream=None):
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != H * F + H * H + 3 * H + 1:
            raise ValueError("packed parameter vector has the wrong length")
        h = vp()
        _check(lib().mlp_create(C.byref(h), int(F), int(H), int(J), p.ctypes.data_as(vp), _stream(stream)),
               "mlp_create")
        self._h, self.F, self.H, self.J, self.n = h, F, H, J, p.size

    @staticmethod
    def pack(W1, b1, W2, b2, w3, b3) -> np.ndarray:
        return np.concatenate([np.ravel(W1), np.ravel(b1), np.ravel(W2), np.ravel(b2), np.ravel(w3),
                               np.ravel(b3)]).astype(np.float32)

    def params(self) -> np.ndarray:
        out = np.empty(self.n, dtype=np.float32)
        _check(lib().mlp_get_params(self._h, out.ctypes.data_as(vp), None), "mlp_get_params")
        return out

    def grad(self) -> np.ndarray:
        out = np.empty(self.n, dtype=np.float32)
        _check(lib().mlp_get_params(self._h, None, out.ctypes.data_as(vp)), "mlp_get_params")
        return out

    def forward(self, X: torch.Tensor, stream=None) -> torch.Tensor:
        X = X.contiguous()
        y = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
        _check(lib().mlp_forward(self._h, X.shape[0], _dptr(X), _dptr(y), _stream(stream)), "mlp_forward")
        return y

    def jvp(self, X: torch.Tensor, stream=None):
        X = X.contiguous()
        y = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
        dy = torch.empty((X.shape[0], self.J), dtype=torch.float32, device=X.device)
        _check(lib().mlp_jvp(self._h, X.shape[0], _dptr(X), _dptr(y), _dptr(dy), _stream(stream)), "mlp_jvp")
        return y, dy

    def backward(self, X: torch.Tensor, t: torch.Tensor, g: torch.Tensor, lam: float = 1.0, stream=None) -> float:
        X, t, g = X.contiguous(), t.contiguous(), g.contiguous()
        loss = C.c_double()
        _check(lib().mlp_backward(self._h, X.shape[0], _dptr(X), _dptr(t), _dptr(g), float(lam), C.byref(loss),
                                  _stream(stream)), "mlp_backward")
        return loss.value

    def step(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        _check(lib().mlp_step(self._h, float(lr), float(beta1), float(beta2), float(eps), _stream(stream)),
               "mlp_step")

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def expected_improvement(mu: torch.Tensor, var: torch.Tensor, f_best: float, xi: float = 0.0, stream=None):
    """EI of every candidate (minimisation) and the best one: (ei tensor, index,
    value).  mu: CUDA FP64, n_cand values or dski_predict's n_cand x (d + 1)
    output (its value column is used); var: CUDA FP64, n_cand."""
    if not mu.is_cuda or mu.dtype != torch.float64 or not var.is_cuda or var.dtype != torch.float64:
        raise TypeError("mu and var must be CUDA float64 tensors")
    mu, var = mu.contiguous(), var.contiguous()
    stride = 1 if mu.dim() == 1 else mu.shape[1]
    n = var.numel()
    if mu.shape[0] != n:
        raise ValueError("mu and var hold different numbers of candidates")
    ei = torch.empty(n, dtype=torch.float64, device=var.device)
    idx = C.c_int()
    best = C.c_double()
    _check(lib().dski_expected_improvement(n, _dptr(mu), stride, _dptr(var), float(f_best), float(xi), _dptr(ei),
                                           C.byref(idx), C.byref(best), _stream(stream)), "dski_expected_improvement")
    return ei, idx.value, best.value


def active_subspace(G: torch.Tensor, d: int, stream=None):
    """Active subspace from gradient samples G (CUDA FP64, D x n: row p holds
    component p of every sample): (P as a D x d numpy array, the D eigenvalues
    of C = (1/n) sum g g^T in decreasing order)."""
    if not G.is_cuda or G.dtype != torch.float64 or G.dim() != 2:
        raise TypeError("G must be a CUDA float64 tensor of shape (D, n)")
    G = G.contiguous()
    D, n = G.shape
    P = np.zeros((D, d), dtype=np.float64)
    lam = np.zeros(D, dtype=np.float64)
    _check(lib().dski_active_subspace(n, D, _dptr(G), n, int(d), P.ctypes.data_as(vp), lam.ctypes.data_as(vp),
                                      _stream(stream)), "dski_active_subspace")
    return P, lam


def active_project(X: torch.Tensor, G: Optional[torch.Tensor], P, stream=None):
    """Reduced data: U = X P (n x d) and, if G (D x n) is given, the reduced
    gradients as a d x n tensor (row j = P[:, j]^T g_i); CUDA FP64."""
    if not X.is_cuda or X.dtype != torch.float64 or X.dim() != 2:
        raise TypeError("X must be a CUDA float64 tensor of shape (n, D)")
    X = X.contiguous()
    n, D = X.shape
    Pt = torch.as_tensor(np.ascontiguousarray(P, dtype=np.float64), device=X.device)
    if Pt.dim() != 2 or Pt.shape[0] != D or not 1 <= Pt.shape[1] <= D:
        raise ValueError(f"P must be a (D, d) matrix with D = {D} and 1 <= d <= D, got {tuple(Pt.shape)}")
    d = Pt.shape[1]
    U = torch.empty((n, d), dtype=torch.float64, device=X.device)
    Gu = None
    if G is not None:
        if not G.is_cuda or G.dtype != torch.float64 or G.dim() != 2 or tuple(G.shape) != (D, n):
            raise ValueError(f"G must be a CUDA float64 tensor of shape (D, n) = ({D}, {n}), "
                             f"got {tuple(G.shape)}")
        G = G.contiguous()
        Gu = torch.empty((d, n), dtype=torch.float64, device=X.device)
    _check(lib().dski_active_project(n, D, d, _dptr(X), _dptr(G) if G is not None else None, n, _dptr(Pt),
                                     _dptr(U), _dptr(Gu) if Gu is not None else None, _stream(stream)),
           "dski_active_project")
    return U, Gu


def rademacher(seed: int, col0: int, ncols: int, N: int, device="cuda", stream=None) -> torch.Tensor:
    out = torch.empty((ncols, N), dtype=torch.float32, device=device)
    _check(lib().dski_rademacher(C.c_uint64(seed), int(col0), int(ncols), int(N), _dptr(out), N,
                                 _stream(stream)), "dski_rademacher")
    return out


def lanczos_quad_log(alpha: Sequence[float], beta: Sequence[float]) -> float:
    J = len(alpha)
    a = _arr([float(v) for v in alpha], C.c_double)
    b = _arr([float(v) for v in beta] + [0.0], C.c_double)
    ok = C.c_int()
    v = lib().dski_lanczos_quad_log(a, b, J, C.byref(ok))
    if not ok.value:
        raise DSKIError(-4, "quadrature failed (non-positive Ritz value)")
    return v


def version() -> str:
    return lib().dski_version().decode()
