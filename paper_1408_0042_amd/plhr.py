"""Python interface to the HIP block PLHR solver.

PyTorch supplies device memory and the stream; every step of the method
runs in libplhr.so.  There is no CPU fallback: constructing a solver
without the built library or without a HIP device raises.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib as L


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _require_cuda(t: torch.Tensor, name: str, dtype=torch.float64):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


@dataclass
class SolveResult:
    eigvals: torch.Tensor      # (k,) device
    V: torch.Tensor            # (n, k) device, point-major
    rel_res: np.ndarray        # (k,)
    iters: int
    converged: bool


class Solver:
    """Block PLHR for the k eigenpairs of A v = lambda v nearest sigma.

    kind: "fd5_2d" or "fd7_3d"; dims: interior grid points; h: spacing;
    scale: factor on the negative Laplacian; potential: optional (n,) float64
    device tensor added to the diagonal; precond: None (T = I) or a dict
    {"levels", "nu", "omega"} for the multigrid V-cycle.
    """

    def __init__(self, kind: str, dims: Sequence[int], h: float, sigma: float, k: int,
                 scale: float = 1.0, potential: Optional[torch.Tensor] = None,
                 precond: Optional[dict] = None, tol: float = 1e-8, max_iters: int = 10000,
                 k_extra: int = 1, lock: bool = True, check_every: int = 1,
                 drop_tol: float = 1e-12, precision: str = "fp64",
                 stream: Optional[torch.cuda.Stream] = None):
        self.lib = L.load()
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device available")
        dims = tuple(int(d) for d in dims)
        a = L.OpDesc()
        if kind == "fd5_2d":
            assert len(dims) == 2
            a.kind, a.nx, a.ny, a.nz = L.OP_FD5_2D, dims[0], dims[1], 1
        elif kind == "fd7_3d":
            assert len(dims) == 3
            a.kind, a.nx, a.ny, a.nz = L.OP_FD7_3D, dims[0], dims[1], dims[2]
        else:
            raise ValueError(f"unknown operator kind {kind}")
        a.dtype = L.F64
        a.h = float(h)
        a.scale = float(scale)
        self.potential = potential
        if potential is not None:
            _require_cuda(potential, "potential")
            a.potential = potential.data_ptr()
        self.n = int(np.prod(dims))
        self.dims = dims
        self.k = int(k)
        self.kint = int(k) + int(k_extra)
        self.sigma = float(sigma)
        t = None
        if precond is not None:
            t = L.PrecDesc()
            t.kind = L.PREC_MG_VCYCLE
            t.levels = int(precond.get("levels", 5))
            t.nu_pre = t.nu_post = int(precond.get("nu", 2))
            t.omega = float(precond.get("omega", 2.0 / 3.0))
        o = L.default_options()
        o.tol, o.max_iters, o.k_extra = float(tol), int(max_iters), int(k_extra)
        o.lock, o.check_every, o.drop_tol = int(bool(lock)), int(check_every), float(drop_tol)
        if precision not in ("fp64", "mixed"):
            raise ValueError("precision must be 'fp64' or 'mixed'")
        o.precision = L.PRECISION_MIXED if precision == "mixed" else L.PRECISION_FP64
        self.opts = o
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._a, self._t = a, t
        ctx = C.c_void_p()
        L.check(self.lib.plhr_create(C.byref(a), None, C.byref(t) if t is not None else None,
                                     self.sigma, self.k, C.byref(o),
                                     C.c_void_p(self.stream.cuda_stream), None, 0,
                                     C.byref(ctx)))
        self.ctx = ctx
        self.finished = False

    # -- lifecycle
    def close(self):
        if getattr(self, "ctx", None):
            self.lib.plhr_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _v0(self, V0: torch.Tensor):
        _require_cuda(V0, "V0")
        if tuple(V0.shape) != (self.n, self.kint):
            raise ValueError(f"V0 must have shape {(self.n, self.kint)}")

    # -- the C ABI, one call each
    def start(self, V0: torch.Tensor):
        self._v0(V0)
        self._V0 = V0
        L.check(self.lib.plhr_start(self.ctx, C.c_void_p(V0.data_ptr())))

    def iterate(self, n_steps: int) -> L.IterInfo:
        info = L.IterInfo()
        L.check(self.lib.plhr_iterate(self.ctx, int(n_steps), C.byref(info)))
        return info

    def finish(self):
        ev = torch.empty(self.k, dtype=torch.float64, device="cuda")
        V = torch.empty((self.n, self.k), dtype=torch.float64, device="cuda")
        rr = (C.c_double * self.k)()
        L.check(self.lib.plhr_finish(self.ctx, C.c_void_p(ev.data_ptr()),
                                     C.c_void_p(V.data_ptr()), rr))
        self.finished = True
        return ev, V, np.array(rr[:])

    def solve(self, V0: torch.Tensor, allow_unconverged: bool = False) -> SolveResult:
        self._v0(V0)
        ev = torch.empty(self.k, dtype=torch.float64, device="cuda")
        V = torch.empty((self.n, self.k), dtype=torch.float64, device="cuda")
        rr = (C.c_double * self.k)()
        it = C.c_int32()
        code = self.lib.plhr_solve(self.ctx, C.c_void_p(V0.data_ptr()), C.c_void_p(ev.data_ptr()),
                                   C.c_void_p(V.data_ptr()), rr, C.byref(it))
        converged = code == L.OK
        if not (converged or (allow_unconverged and code == L.ERR_NOT_CONVERGED)):
            L.check(code)
        self.finished = True
        return SolveResult(ev, V, np.array(rr[:]), int(it.value), converged)

    def backward(self, dL_dlam: torch.Tensor, out: Optional[torch.Tensor] = None,
                 accumulate: bool = False) -> torch.Tensor:
        _require_cuda(dL_dlam, "dL_dlam")
        if out is None:
            out = torch.empty(self.n, dtype=torch.float64, device="cuda")
        L.check(self.lib.plhr_eigvals_backward(self.ctx, C.c_void_p(dL_dlam.data_ptr()),
                                               C.c_void_p(out.data_ptr()), int(accumulate)))
        return out

    def apply(self, which: str, X: torch.Tensor) -> torch.Tensor:
        _require_cuda(X, "X")
        w = {"A": 0, "A-sigma": 1, "T": 2}[which]
        ncols = 1 if X.dim() == 1 else X.shape[1]
        Y = torch.empty_like(X)
        L.check(self.lib.plhr_apply(self.ctx, w, C.c_void_p(X.data_ptr()),
                                    C.c_void_p(Y.data_ptr()), int(ncols)))
        return Y

    def profile_start(self, category: int = -1, max_launches: int = 100000):
        L.check(self.lib.plhr_profile_start(self.ctx, int(category), int(max_launches)))

    def profile_stop(self) -> dict:
        pr = L.Profile()
        L.check(self.lib.plhr_profile_stop(self.ctx, C.byref(pr)))
        out = {}
        for i, name in enumerate(L.KCAT_NAMES):
            out[name] = {"launches": pr.launches[i], "ms": pr.total_ms[i],
                         "bytes": pr.bytes[i], "flops": pr.flops[i]}
        out["truncated"] = bool(pr.truncated)
        return out

    def debug_read(self, which: int, count: int) -> np.ndarray:
        buf = (C.c_double * count)()
        L.check(self.lib.plhr_debug_read(self.ctx, int(which), buf, int(count)))
        return np.array(buf[:])

    def state(self):
        lam = (C.c_double * self.kint)()
        V = torch.empty((self.n, self.kint), dtype=torch.float64, device="cuda")
        L.check(self.lib.plhr_get_state(self.ctx, lam, C.c_void_p(V.data_ptr())))
        return np.array(lam[:]), V


def eigvals(potential: torch.Tensor, V0: torch.Tensor, **opts) -> torch.Tensor:
    """Differentiable eigenvalues of scale*(-Laplacian) + diag(potential)
    nearest sigma (opts as for Solver).  backward() returns dL/dpotential
    from the library's Hellmann-Feynman kernel, d lambda_j / d pot_x =
    v_j(x)^2 / (v_j^T v_j)."""
    return _EigvalsWithStart.apply(potential, V0, opts)


class _EigvalsWithStart(torch.autograd.Function):
    @staticmethod
    def forward(ctx, potential, V0, opts):
        S = Solver(potential=potential.detach().contiguous(), **opts)
        r = S.solve(V0.detach().contiguous())
        ctx.solver = S
        ctx.result = r
        return r.eigvals.clone()

    @staticmethod
    def backward(ctx, grad_lam):
        S = ctx.solver
        g = S.backward(grad_lam.detach().contiguous().to(torch.float64))
        S.close()
        return g, None, None
