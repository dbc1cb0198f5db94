"""Python interface to the HIP block PLHR solver.

PyTorch supplies device memory and the stream; every step of the method
runs in libplhr.so.  There is no CPU fallback: constructing a solver
without the built library or without a HIP device raises.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import List, NamedTuple, Optional, Sequence

import numpy as np
import torch

from . import _lib as L


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _csr_fields(desc, csr, n: int, name: str):
    """Fill the CSR fields of an operator descriptor from device tensors."""
    rp, ci, v = csr
    _require_cuda(rp, name + " row_ptr", torch.int32)
    _require_cuda(ci, name + " col_idx", torch.int32)
    _require_cuda(v, name + " values", torch.float64)
    if rp.numel() != n + 1 or ci.numel() != v.numel():
        raise ValueError(f"{name}: row_ptr needs n + 1 entries and col_idx/values nnz each")
    desc.row_ptr, desc.col_idx, desc.values = rp.data_ptr(), ci.data_ptr(), v.data_ptr()
    desc.nnz = int(v.numel())
    return (rp, ci, v)


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
    """Block PLHR for the k eigenpairs of A v = lambda B v nearest sigma.

    kind: "fd5_2d", "fd7_3d" (finite differences) or "q1_2d", "q1_3d"
    (bilinear/trilinear finite elements, interior nodes); dims: interior
    grid points (nodes); h: spacing (element size); scale: factor on the
    negative Laplacian (on the stiffness); potential: optional (n,) float64
    device tensor added to the diagonal; mass: None (B = I), an (n,)
    float64 positive device tensor (B = diag(mass), finite differences),
    or "q1" (B = the consistent finite-element mass); precond: None (T = I)
    or a dict {"levels", "nu", "omega"} for the multigrid V-cycle, with
    "kind": "av" (AV-MG, Appendix A Algorithm 4; "delta", "degree") or
    "inv" (INV-MG, Algorithm 5) for the preconditioners of Section 6.2;
    extraction: "tharmonic" (eq. 3.5) or "harmonic" (T -> I in the
    projection); use_graph: replay each iteration from a captured HIP graph.
    precond {"kind": "dense", "matrix": T} takes T as an (n, n) float64
    device tensor (symmetric positive definite, kept referenced).
    algorithm: "block" (Algorithm 3), "single" (Algorithm 1 in complex
    arithmetic, k = 1; the start block is (n, 2): real and imaginary parts)
    or "plmr" (PLMR of Section 3.3, k = 1, start block (n, 1)).
    kind "csr": a general sparse symmetric A given as csr = (row_ptr int32,
    col_idx int32, values float64) device tensors, dims = (n,); mass may
    then be a CSR triple for B; T must be the identity.
    kind "bloch7_3d": the complex Hermitian Bloch operator
    scale (-Laplacian_theta) + diag(potential) on a periodic box with phases
    `thetas`, solved by the block iteration in complex arithmetic
    (Algorithm 2); B = I, T the identity or {"levels", "nu", "omega"} for
    its V-cycle; V0 is an (n, k + k_extra) complex128 tensor and the
    vectors come back as (n, k) complex128.
    workspace: optional device tensor of at least `workspace_bytes` bytes
    (256-byte aligned) that the context uses instead of allocating.
    """

    def __init__(self, kind: str, dims: Sequence[int], h: float, sigma: float, k: int,
                 scale: float = 1.0, potential: Optional[torch.Tensor] = None,
                 mass=None, csr=None,
                 precond: Optional[dict] = None, tol: float = 1e-8, max_iters: int = 10000,
                 k_extra: int = 1, lock: bool = True, check_every: int = 1,
                 drop_tol: float = 1e-10, precision: str = "fp64", ortho_passes: int = 0,
                 extraction: str = "tharmonic", use_graph: bool = False,
                 algorithm: str = "block", stream: Optional[torch.cuda.Stream] = None,
                 thetas: Sequence[float] = (0.0, 0.0, 0.0),
                 workspace: Optional[torch.Tensor] = None):
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
        elif kind == "q1_2d":
            assert len(dims) == 2
            a.kind, a.nx, a.ny, a.nz = L.OP_Q1_2D, dims[0], dims[1], 1
        elif kind == "q1_3d":
            assert len(dims) == 3
            a.kind, a.nx, a.ny, a.nz = L.OP_Q1_3D, dims[0], dims[1], dims[2]
        elif kind == "csr":
            assert len(dims) == 1 and csr is not None
            a.kind, a.nx, a.ny, a.nz = L.OP_CSR, dims[0], 1, 1
            self._csr = _csr_fields(a, csr, dims[0], "csr")
        elif kind == "bloch7_3d":
            assert len(dims) == 3
            a.kind, a.nx, a.ny, a.nz = L.OP_BLOCH7_3D, dims[0], dims[1], dims[2]
            for d in range(3):
                a.theta[d] = float(thetas[d])
        else:
            raise ValueError(f"unknown operator kind {kind}")
        self.cplx = kind == "bloch7_3d"
        a.dtype = L.C128 if self.cplx else L.F64
        a.h = float(h)
        a.scale = float(scale)
        self.potential = potential
        if potential is not None:
            _require_cuda(potential, "potential")
            a.potential = potential.data_ptr()
        self.n = int(np.prod(dims))
        self.dims = dims
        self.mass = mass
        bdesc = None
        if isinstance(mass, (tuple, list)):
            bdesc = L.OpDesc()
            bdesc.kind, bdesc.dtype = L.OP_CSR, L.F64
            bdesc.nx, bdesc.ny, bdesc.nz = a.nx, 1, 1
            self._bcsr = _csr_fields(bdesc, mass, a.nx, "mass")
        elif isinstance(mass, str):
            if mass != "q1":
                raise ValueError("mass must be None, a tensor or 'q1'")
            bdesc = L.OpDesc()
            bdesc.kind, bdesc.dtype = L.OP_Q1_MASS, L.F64
            bdesc.nx, bdesc.ny, bdesc.nz = a.nx, a.ny, a.nz
            bdesc.h, bdesc.scale = a.h, 1.0
        elif mass is not None:
            _require_cuda(mass, "mass")
            if tuple(mass.shape) != (self.n,):
                raise ValueError(f"mass must have shape {(self.n,)}")
            bdesc = L.OpDesc()
            bdesc.kind, bdesc.dtype = L.OP_DIAG, L.F64
            bdesc.nx, bdesc.ny, bdesc.nz = a.nx, a.ny, a.nz
            bdesc.h, bdesc.scale = 1.0, 1.0
            bdesc.potential = mass.data_ptr()
        self.k = int(k)
        if algorithm not in ("block", "single", "plmr"):
            raise ValueError("algorithm must be 'block', 'single' or 'plmr'")
        self.kint = {"single": 2, "plmr": 1}.get(algorithm, int(k) + int(k_extra))
        # columns of the start block (complex ones for the Bloch operator)
        self.kcols = self.kint
        self.sigma = float(sigma)
        t = None
        if precond is not None:
            t = L.PrecDesc()
            kinds = {"vcycle": L.PREC_MG_VCYCLE, "av": L.PREC_AV_MG, "inv": L.PREC_INV_MG,
                     "dense": L.PREC_DENSE}
            t.kind = kinds[precond.get("kind", "vcycle")]
            if t.kind == L.PREC_DENSE:
                Tm = precond["matrix"]
                _require_cuda(Tm, "precond matrix")
                if tuple(Tm.shape) != (self.n, self.n) or not Tm.is_contiguous():
                    raise ValueError(f"precond matrix must be a contiguous {(self.n, self.n)} tensor")
                self._tmat = Tm
                t.matrix = Tm.data_ptr()
            t.levels = int(precond.get("levels", 5))
            t.nu_pre = t.nu_post = int(precond.get("nu", 2))
            t.omega = float(precond.get("omega", 2.0 / 3.0))
            t.delta = float(precond.get("delta", 0.6))
            t.degree = int(precond.get("degree", 10))
        o = L.default_options()
        o.tol, o.max_iters, o.k_extra = float(tol), int(max_iters), int(k_extra)
        o.lock, o.check_every, o.drop_tol = int(bool(lock)), int(check_every), float(drop_tol)
        o.ortho_passes = int(ortho_passes)
        o.extraction = {"tharmonic": L.EXTRACT_T_HARMONIC, "harmonic": L.EXTRACT_HARMONIC}[extraction]
        o.use_graph = int(bool(use_graph))
        o.algorithm = {"block": L.ALG_BLOCK, "single": L.ALG_SINGLE, "plmr": L.ALG_PLMR}[algorithm]
        if precision not in ("fp64", "mixed"):
            raise ValueError("precision must be 'fp64' or 'mixed'")
        o.precision = L.PRECISION_MIXED if precision == "mixed" else L.PRECISION_FP64
        self.opts = o
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._a, self._t, self._b = a, t, bdesc
        sz = C.c_size_t()
        L.check(self.lib.plhr_workspace_size(C.byref(a),
                                             C.byref(bdesc) if bdesc is not None else None,
                                             C.byref(t) if t is not None else None, self.sigma,
                                             self.k, C.byref(o), C.byref(sz)))
        self.workspace_bytes = int(sz.value)
        ws_ptr, ws_len = None, 0
        if workspace is not None:
            # a caller workspace: the context allocates no device memory
            if not workspace.is_cuda or workspace.numel() * workspace.element_size() < sz.value:
                raise ValueError(f"workspace must be a device tensor of >= {sz.value} bytes")
            self._ws = workspace
            ws_ptr, ws_len = C.c_void_p(workspace.data_ptr()), workspace.numel() * workspace.element_size()
        ctx = C.c_void_p()
        L.check(self.lib.plhr_create(C.byref(a), C.byref(bdesc) if bdesc is not None else None,
                                     C.byref(t) if t is not None else None,
                                     self.sigma, self.k, C.byref(o),
                                     C.c_void_p(self.stream.cuda_stream), ws_ptr, ws_len,
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
        _require_cuda(V0, "V0", torch.complex128 if self.cplx else torch.float64)
        if tuple(V0.shape) != (self.n, self.kcols):
            raise ValueError(f"V0 must have shape {(self.n, self.kcols)}")

    def _vout(self):
        return torch.empty((self.n, self.k), dtype=torch.complex128 if self.cplx else torch.float64,
                           device="cuda")

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
        V = self._vout()
        rr = (C.c_double * self.k)()
        L.check(self.lib.plhr_finish(self.ctx, C.c_void_p(ev.data_ptr()),
                                     C.c_void_p(V.data_ptr()), rr))
        self.finished = True
        return ev, V, np.array(rr[:])

    def solve(self, V0: torch.Tensor, allow_unconverged: bool = False) -> SolveResult:
        self._v0(V0)
        ev = torch.empty(self.k, dtype=torch.float64, device="cuda")
        V = self._vout()
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
        _require_cuda(X, "X", torch.complex128 if self.cplx else torch.float64)
        w = {"A": 0, "A-sigma": 1, "T": 2}[which]
        ncols = 1 if X.dim() == 1 else X.shape[1]
        if self.cplx:
            ncols *= 2  # real columns of the interleaved view
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
        """Current Rayleigh quotients (one per real column: each twice, for
        the complex columns of the Bloch operator) and the block V."""
        nl = 2 * self.kcols if self.cplx else self.kint
        lam = (C.c_double * nl)()
        V = torch.empty((self.n, self.kcols), dtype=torch.complex128 if self.cplx else torch.float64,
                        device="cuda")
        L.check(self.lib.plhr_get_state(self.ctx, lam, C.c_void_p(V.data_ptr())))
        return np.array(lam[:]), V


def bloch_apply(X: torch.Tensor, dims: Sequence[int], h: float = 1.0, thetas=(0.0, 0.0, 0.0),
                scale: float = 0.5, potential: Optional[torch.Tensor] = None, shift: float = 0.0,
                out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Y = (scale*(-Laplacian_theta) + diag(potential) - shift I) X on the
    Bloch-periodic nx x ny x nz box (plhr_op_apply), X a complex128 device
    block (n, ncols), enqueued on torch's current stream."""
    nx, ny, nz = (tuple(dims) + (1, 1))[:3]
    n = nx * ny * nz
    _require_cuda(X, "X", torch.complex128)
    if X.dim() != 2 or X.shape[0] != n:
        raise ValueError(f"X must be ({n}, ncols)")
    if out is None:
        out = torch.empty_like(X)
    _require_cuda(out, "out", torch.complex128)
    if out.shape != X.shape:
        raise ValueError("out must have the shape of X")
    d = L.OpDesc()
    d.kind, d.dtype, d.nx, d.ny, d.nz = L.OP_BLOCH7_3D, L.C128, nx, ny, nz
    d.h, d.scale = float(h), float(scale)
    if potential is not None:
        _require_cuda(potential, "potential")
        if potential.numel() != n:
            raise ValueError(f"potential needs {n} entries")
        d.potential = potential.data_ptr()
    d.theta[0], d.theta[1], d.theta[2] = (float(t) for t in thetas)
    lib = L.load()
    L.check(lib.plhr_op_apply(C.byref(d), float(shift), C.c_void_p(X.data_ptr()),
                              C.c_void_p(out.data_ptr()), int(X.shape[1]),
                              C.c_void_p(torch.cuda.current_stream().cuda_stream)))
    return out


def gram_c128(X: torch.Tensor, Y: Optional[torch.Tensor] = None,
              out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """G = X^H Y for complex128 device blocks (n, mx) and (n, my) on the
    matrix cores (plhr_gram_c128); Y = None means Y = X.  Enqueued on
    torch's current stream."""
    Y = X if Y is None else Y
    _require_cuda(X, "X", torch.complex128)
    _require_cuda(Y, "Y", torch.complex128)
    if X.dim() != 2 or Y.dim() != 2 or X.shape[0] != Y.shape[0]:
        raise ValueError("X and Y must be (n, mx) and (n, my)")
    n, mx, my = X.shape[0], X.shape[1], Y.shape[1]
    if out is None:
        out = torch.empty((mx, my), dtype=torch.complex128, device=X.device)
    _require_cuda(out, "out", torch.complex128)
    if tuple(out.shape) != (mx, my):
        raise ValueError(f"out must be ({mx}, {my})")
    lib = L.load()
    need = C.c_size_t()
    L.check(lib.plhr_gram_c128_workspace(n, mx, my, C.byref(need)))
    ws = torch.empty(need.value, dtype=torch.uint8, device=X.device)
    L.check(lib.plhr_gram_c128(n, C.c_void_p(X.data_ptr()), mx, C.c_void_p(Y.data_ptr()), my,
                               C.c_void_p(out.data_ptr()), C.c_void_p(ws.data_ptr()), need.value,
                               C.c_void_p(torch.cuda.current_stream().cuda_stream)))
    return out


def rowmul_c128(Z: torch.Tensor, M: torch.Tensor) -> torch.Tensor:
    """Y = Z M for complex128 device blocks Z (n, m) and M (m, k), m, k <= 64
    (plhr_rowmul_c128), on torch's current stream."""
    _require_cuda(Z, "Z", torch.complex128)
    _require_cuda(M, "M", torch.complex128)
    if Z.dim() != 2 or M.dim() != 2 or Z.shape[1] != M.shape[0]:
        raise ValueError("Z must be (n, m) and M (m, k)")
    n, m = Z.shape
    k = M.shape[1]
    Y = torch.empty((n, k), dtype=torch.complex128, device=Z.device)
    L.check(L.load().plhr_rowmul_c128(n, C.c_void_p(Z.data_ptr()), m, C.c_void_p(M.data_ptr()),
                                      k, C.c_void_p(Y.data_ptr()),
                                      C.c_void_p(torch.cuda.current_stream().cuda_stream)))
    return Y


def cholqr_c128(Z: torch.Tensor):
    """Q, R with Z = Q R, Q^H Q = I, R upper triangular with a real positive
    diagonal (plhr_cholqr_c128), for a complex128 device block (n, m),
    m <= 64.  Synchronises torch's current stream."""
    _require_cuda(Z, "Z", torch.complex128)
    if Z.dim() != 2:
        raise ValueError("Z must be (n, m)")
    n, m = Z.shape
    Q = torch.empty_like(Z)
    R = torch.empty((m, m), dtype=torch.complex128, device=Z.device)
    lib = L.load()
    need = C.c_size_t()
    L.check(lib.plhr_cholqr_c128_workspace(n, m, C.byref(need)))
    ws = torch.empty(need.value, dtype=torch.uint8, device=Z.device)
    L.check(lib.plhr_cholqr_c128(n, C.c_void_p(Z.data_ptr()), m, C.c_void_p(Q.data_ptr()),
                                 C.c_void_p(R.data_ptr()), C.c_void_p(ws.data_ptr()), need.value,
                                 C.c_void_p(torch.cuda.current_stream().cuda_stream)))
    return Q, R


def projected_solve(GL: torch.Tensor, GR: torch.Tensor, kint: int,
                    keep: Optional[torch.Tensor] = None):
    """The projected step of one iteration on given Gram matrices
    (plhr_projected_solve): G_L y = xi G_R y, the kint units of smallest
    |xi| and the real coefficient basis Y' of Algorithm 3.  GL, GR are
    float64 (m, m) device tensors, keep an optional int32 (m,) mask.
    Returns (Y (m, kint), xi (m,) complex: one entry per sorted unit, a
    pair by its Im > 0 member, zero past the last unit, kinds (kint,),
    pair (kint,), n_excluded).  Synchronises torch's current stream."""
    _require_cuda(GL, "GL")
    _require_cuda(GR, "GR")
    m = GL.shape[0]
    if GL.shape != (m, m) or GR.shape != (m, m):
        raise ValueError("GL and GR must be (m, m)")
    if keep is not None:
        _require_cuda(keep, "keep", torch.int32)
        if keep.shape != (m,):
            raise ValueError("keep must be (m,)")
    dev = GL.device
    Y = torch.empty((m, kint), dtype=torch.float64, device=dev)
    xi = torch.empty((2, m), dtype=torch.float64, device=dev)
    kinds = torch.empty(kint, dtype=torch.int32, device=dev)
    pair = torch.empty(kint, dtype=torch.int32, device=dev)
    lib = L.load()
    need = C.c_size_t()
    L.check(lib.plhr_projected_workspace(m, kint, C.byref(need)))
    ws = torch.empty(need.value, dtype=torch.uint8, device=dev)
    nex = C.c_int32()
    L.check(lib.plhr_projected_solve(m, kint, C.c_void_p(GL.data_ptr()),
                                     C.c_void_p(GR.data_ptr()), C.c_void_p(_ptr(keep)),
                                     C.c_void_p(Y.data_ptr()), C.c_void_p(xi.data_ptr()),
                                     C.c_void_p(kinds.data_ptr()), C.c_void_p(pair.data_ptr()),
                                     C.byref(nex), C.c_void_p(ws.data_ptr()), need.value,
                                     C.c_void_p(torch.cuda.current_stream().cuda_stream)))
    xic = torch.complex(xi[0], xi[1])
    return Y, xic, kinds, pair, int(nex.value)


class BlochPrecond:
    """One multigrid V-cycle for the Bloch operator scale*(-Laplacian_theta)
    on the periodic nx x ny x nz box (plhr_bloch_prec_*): apply(X) returns
    T X for a complex128 device block (n, ncols), ncols <= max_cols, on
    torch's current stream at construction.  workspace: an optional uint8
    device tensor of at least workspace_bytes(...) bytes (256-byte aligned)
    that holds every device buffer of the hierarchy."""

    @staticmethod
    def workspace_bytes(dims: Sequence[int], h: float = 1.0, thetas=(0.0, 0.0, 0.0),
                        scale: float = 0.5, levels: int = 3, nu: int = 2,
                        omega: float = 2.0 / 3.0, max_cols: int = 32) -> int:
        nx, ny, nz = (tuple(dims) + (1, 1))[:3]
        d = L.OpDesc()
        d.kind, d.dtype, d.nx, d.ny, d.nz = L.OP_BLOCH7_3D, L.C128, nx, ny, nz
        d.h, d.scale = float(h), float(scale)
        d.theta[0], d.theta[1], d.theta[2] = (float(t) for t in thetas)
        t = L.PrecDesc()
        t.kind, t.levels, t.nu_pre, t.nu_post, t.omega = (L.PREC_MG_VCYCLE, int(levels), int(nu),
                                                           int(nu), float(omega))
        sz = C.c_size_t()
        L.check(L.load().plhr_bloch_prec_workspace_size(C.byref(d), C.byref(t), int(max_cols),
                                                        C.byref(sz)))
        return int(sz.value)

    def __init__(self, dims: Sequence[int], h: float = 1.0, thetas=(0.0, 0.0, 0.0),
                 scale: float = 0.5, levels: int = 3, nu: int = 2, omega: float = 2.0 / 3.0,
                 max_cols: int = 32, workspace: Optional[torch.Tensor] = None):
        self.lib = L.load()
        self.handle = None
        nx, ny, nz = (tuple(dims) + (1, 1))[:3]
        self.n = nx * ny * nz
        self.max_cols = int(max_cols)
        d = L.OpDesc()
        d.kind, d.dtype, d.nx, d.ny, d.nz = L.OP_BLOCH7_3D, L.C128, nx, ny, nz
        d.h, d.scale = float(h), float(scale)
        d.theta[0], d.theta[1], d.theta[2] = (float(t) for t in thetas)
        t = L.PrecDesc()
        t.kind, t.levels, t.nu_pre, t.nu_post, t.omega = (L.PREC_MG_VCYCLE, int(levels), int(nu),
                                                           int(nu), float(omega))
        hdl = C.c_void_p()
        self.stream = torch.cuda.current_stream()
        ws, wsb = None, 0
        if workspace is not None:
            _require_cuda(workspace, "workspace", torch.uint8)
            ws, wsb = C.c_void_p(workspace.data_ptr()), workspace.numel()
            self._ws = workspace
        L.check(self.lib.plhr_bloch_prec_create(C.byref(d), C.byref(t), self.max_cols,
                                                C.c_void_p(self.stream.cuda_stream), ws, wsb,
                                                C.byref(hdl)))
        self.handle = hdl

    def apply(self, X: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        _require_cuda(X, "X", torch.complex128)
        if X.dim() != 2 or X.shape[0] != self.n:
            raise ValueError(f"X must be ({self.n}, ncols)")
        if out is None:
            out = torch.empty_like(X)
        _require_cuda(out, "out", torch.complex128)
        if out.shape != X.shape:
            raise ValueError("out must have the shape of X")
        L.check(self.lib.plhr_bloch_prec_apply(self.handle, C.c_void_p(X.data_ptr()),
                                               C.c_void_p(out.data_ptr()), int(X.shape[1])))
        return out

    def close(self):
        if self.handle is not None:
            self.stream.synchronize()
            self.lib.plhr_bloch_prec_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


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


class BatchResult(NamedTuple):
    eigvals: torch.Tensor     # (nbatch, k)
    V: List[torch.Tensor]     # n_b x k each
    rel_res: np.ndarray       # (nbatch, k)
    iters: np.ndarray         # (nbatch,)
    status: np.ndarray        # (nbatch,) per-problem status codes
    converged: bool


class BatchSolver:
    """Many independent 2-D problems scale*(-Laplacian) + diag(potential_b)
    (5-point Dirichlet, spacing h) solved together by plhr_batch_*; each
    problem has its own grid (dims[b]), potential and shift.  workspace: an
    optional uint8 device tensor of at least workspace_bytes() bytes
    (256-byte aligned) that holds every device buffer of the batch;
    workspace_size=True builds only the size query (no device memory)."""

    def __init__(self, dims: Sequence[Sequence[int]], h: float, sigma: Sequence[float], k: int,
                 scale: float = 1.0, potentials: Optional[Sequence[torch.Tensor]] = None,
                 precond: Optional[dict] = None, tol: float = 1e-8, max_iters: int = 10000,
                 k_extra: int = 1, lock: bool = True, check_every: int = 10,
                 drop_tol: float = 1e-10, stream: Optional[torch.cuda.Stream] = None,
                 workspace: Optional[torch.Tensor] = None, workspace_size: bool = False):
        self.lib = L.load()
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device available")
        self.nb = len(dims)
        self.dims = [tuple(int(x) for x in d) for d in dims]
        self.n = [d[0] * d[1] for d in self.dims]
        self.k = int(k)
        self.kint = int(k) + int(k_extra)
        self.potentials = None
        if potentials is not None:
            self.potentials = [p.detach().contiguous() for p in potentials]
            for p in self.potentials:
                _require_cuda(p, "potential")
        descs = (L.OpDesc * self.nb)()
        for b, d in enumerate(self.dims):
            descs[b].kind, descs[b].nx, descs[b].ny, descs[b].nz = L.OP_FD5_2D, d[0], d[1], 1
            descs[b].dtype = L.F64
            descs[b].h = float(h)
            descs[b].scale = float(scale)
            if self.potentials is not None:
                descs[b].potential = self.potentials[b].data_ptr()
        t = None
        if precond is not None:
            t = L.PrecDesc()
            kinds = {"vcycle": L.PREC_MG_VCYCLE, "av": L.PREC_AV_MG, "inv": L.PREC_INV_MG}
            t.kind = kinds[precond.get("kind", "vcycle")]
            t.levels = int(precond.get("levels", 5))
            t.nu_pre = t.nu_post = int(precond.get("nu", 2))
            t.omega = float(precond.get("omega", 2.0 / 3.0))
            t.delta = float(precond.get("delta", 0.6))
            t.degree = int(precond.get("degree", 10))
        o = L.default_options()
        o.tol, o.max_iters, o.k_extra = float(tol), int(max_iters), int(k_extra)
        o.lock, o.check_every, o.drop_tol = int(bool(lock)), int(check_every), float(drop_tol)
        sig = (C.c_double * self.nb)(*[float(x) for x in sigma])
        if workspace_size:
            sz = C.c_size_t()
            L.check(self.lib.plhr_batch_workspace_size(
                self.nb, descs, C.byref(t) if t is not None else None, sig, self.k, C.byref(o),
                C.byref(sz)))
            self.workspace_bytes = int(sz.value)
            self.ctx = None
            return
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        ctx = C.c_void_p()
        ws, wsb = None, 0
        if workspace is not None:
            _require_cuda(workspace, "workspace", torch.uint8)
            ws, wsb = C.c_void_p(workspace.data_ptr()), workspace.numel()
            self._ws = workspace
        L.check(self.lib.plhr_batch_create(self.nb, descs, C.byref(t) if t is not None else None,
                                           sig, self.k, C.byref(o),
                                           C.c_void_p(self.stream.cuda_stream), ws, wsb,
                                           C.byref(ctx)))
        self._descs, self._t = descs, t
        self.ctx = ctx

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.plhr_batch_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_graph(self, on: bool):
        L.check(self.lib.plhr_batch_set_graph(self.ctx, int(bool(on))))

    def solve(self, V0: Sequence[torch.Tensor], allow_unconverged: bool = False,
              allow_failures: bool = False) -> BatchResult:
        """allow_unconverged: return when some problems reached max_iters;
        allow_failures: return also when some problems failed (their status
        entries say how); otherwise such outcomes raise."""
        if len(V0) != self.nb:
            raise ValueError("one start block per problem")
        for b, v in enumerate(V0):
            _require_cuda(v, "V0")
            if tuple(v.shape) != (self.n[b], self.kint):
                raise ValueError(f"V0[{b}] must have shape {(self.n[b], self.kint)}")
        v0p = (C.c_void_p * self.nb)(*[v.data_ptr() for v in V0])
        ev = torch.empty((self.nb, self.k), dtype=torch.float64, device="cuda")
        V = [torch.empty((n, self.k), dtype=torch.float64, device="cuda") for n in self.n]
        vp = (C.c_void_p * self.nb)(*[v.data_ptr() for v in V])
        rr = (C.c_double * (self.nb * self.k))()
        its = (C.c_int32 * self.nb)()
        sts = (C.c_int32 * self.nb)()
        code = self.lib.plhr_batch_solve(self.ctx, v0p, C.c_void_p(ev.data_ptr()), vp, rr, its,
                                         sts)
        converged = code == L.OK
        if not (converged or (allow_unconverged and code == L.ERR_NOT_CONVERGED) or
                (allow_failures and code not in (L.ERR_ARG, L.ERR_HIP, L.ERR_STATE))):
            L.check(code)
        return BatchResult(ev, V, np.array(rr[:]).reshape(self.nb, self.k), np.array(its[:]),
                           np.array(sts[:]), converged)

    def backward(self, dL_dlam: torch.Tensor, accumulate: bool = False) -> List[torch.Tensor]:
        _require_cuda(dL_dlam, "dL_dlam")
        if tuple(dL_dlam.shape) != (self.nb, self.k):
            raise ValueError("dL_dlam must have shape (nbatch, k)")
        g = [torch.zeros(n, dtype=torch.float64, device="cuda") for n in self.n]
        gp = (C.c_void_p * self.nb)(*[x.data_ptr() for x in g])
        L.check(self.lib.plhr_batch_eigvals_backward(self.ctx,
                                                     C.c_void_p(dL_dlam.contiguous().data_ptr()),
                                                     gp, int(accumulate)))
        return g

    def apply(self, which: str, X: Sequence[torch.Tensor]) -> List[torch.Tensor]:
        w = {"A": 0, "A-sigma": 1, "T": 2}[which]
        ncols = X[0].shape[1]
        for b, x in enumerate(X):
            _require_cuda(x, "X")
            if tuple(x.shape) != (self.n[b], ncols):
                raise ValueError("X[b] must be n_b x ncols")
        Y = [torch.empty_like(x) for x in X]
        xp = (C.c_void_p * self.nb)(*[x.data_ptr() for x in X])
        yp = (C.c_void_p * self.nb)(*[y.data_ptr() for y in Y])
        L.check(self.lib.plhr_batch_apply(self.ctx, w, xp, yp, int(ncols)))
        return Y

    def tuning(self) -> dict:
        t = L.BatchTuning()
        L.check(self.lib.plhr_batch_tuning_info(self.ctx, C.byref(t)))
        return {"chunk_points": t.chunk_points, "row_threads": t.row_threads,
                "use_graph": bool(t.use_graph), "nchunks": t.nchunks,
                "tuned_ms": list(t.tuned_ms)}

    def profile_start(self, category: int = -1, max_launches: int = 200000):
        L.check(self.lib.plhr_batch_profile_start(self.ctx, int(category), int(max_launches)))

    def profile_stop(self) -> dict:
        pr = L.Profile()
        L.check(self.lib.plhr_batch_profile_stop(self.ctx, C.byref(pr)))
        out = {}
        for i, name in enumerate(L.KCAT_NAMES):
            out[name] = {"launches": pr.launches[i], "ms": pr.total_ms[i],
                         "bytes": pr.bytes[i], "flops": pr.flops[i]}
        out["truncated"] = bool(pr.truncated)
        return out


def batch_eigvals(potentials: Sequence[torch.Tensor], V0: Sequence[torch.Tensor],
                  **opts) -> torch.Tensor:
    """Differentiable (nbatch, k) eigenvalues of a batch (opts as for
    BatchSolver, without potentials); backward gives dL/dpotential_b for
    every problem from the batched Hellmann-Feynman kernel."""
    return _BatchEigvals.apply(opts, V0, *potentials)


class _BatchEigvals(torch.autograd.Function):
    @staticmethod
    def forward(ctx, opts, V0, *potentials):
        S = BatchSolver(potentials=[p.detach() for p in potentials], **opts)
        r = S.solve([v.detach().contiguous() for v in V0])
        ctx.solver = S
        return r.eigvals.clone()

    @staticmethod
    def backward(ctx, grad_lam):
        S = ctx.solver
        g = S.backward(grad_lam.detach().contiguous().to(torch.float64))
        S.close()
        return (None, None, *g)
