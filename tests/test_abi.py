"""The C-ABI library loads and exports every symbol include/plhr.h
declares; host-side argument validation (no GPU needed)."""
import ctypes as C
import os
import re

import pytest

from paper_1408_0042_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "plhr.h")).read()
    return sorted(set(re.findall(r"\b(plhr_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = L.load()
    names = _declared()
    assert "plhr_create" in names and "plhr_eigvals_backward" in names
    for name in names:
        assert hasattr(lib, name), name


def test_options_default_and_version():
    o = L.default_options()
    assert o.tol == 1e-8 and o.k_extra == 1 and o.lock == 1 and o.check_every == 1
    assert b"gfx950" in L.load().plhr_version()


def _ws(a, t=None, sigma=1.0, k=4, o=None):
    sz = C.c_size_t()
    code = L.load().plhr_workspace_size(C.byref(a), None, C.byref(t) if t else None, sigma, k,
                                        C.byref(o) if o else None, C.byref(sz))
    return code, sz.value


def _fd3(N=64):
    a = L.OpDesc()
    a.kind, a.dtype, a.nx, a.ny, a.nz, a.h, a.scale = L.OP_FD7_3D, L.F64, N, N, N, 1 / (N + 1), 1.0
    return a


def test_workspace_size_and_validation():
    a = _fd3()
    t = L.PrecDesc()
    t.kind, t.levels, t.nu_pre, t.nu_post, t.omega = L.PREC_MG_VCYCLE, 5, 2, 2, 2 / 3
    code, sz = _ws(a, t, 12667.6, 16)
    assert code == L.OK
    n, kint = 64**3, 17
    assert sz >= 3 * n * 4 * kint * 8        # Z, QZ, TQZ
    # invalid inputs are rejected on the host
    assert _ws(a, t, float("nan"), 16)[0] == L.ERR_ARG
    assert _ws(a, t, 1.0, 0)[0] == L.ERR_ARG
    bad = _fd3()
    bad.h = -1.0
    assert _ws(bad, t, 1.0, 4)[0] == L.ERR_ARG
    t2 = L.PrecDesc()
    t2.kind, t2.levels, t2.nu_pre, t2.nu_post, t2.omega = L.PREC_MG_VCYCLE, 5, 2, 1, 2 / 3
    assert _ws(a, t2, 1.0, 4)[0] == L.ERR_ARG          # asymmetric V-cycle
    t3 = L.PrecDesc()
    t3.kind, t3.levels, t3.nu_pre, t3.nu_post, t3.omega = L.PREC_MG_VCYCLE, 8, 2, 2, 2 / 3
    assert _ws(a, t3, 1.0, 4)[0] == L.ERR_ARG          # 64 not divisible by 2^7
    small = _fd3(2)
    assert _ws(small, None, 1.0, 4)[0] == L.ERR_ARG     # 4 (k + k_extra) > n
    assert _ws(a, None, 1.0, 20)[0] == 0                  # m = 84, the largest supported
    assert _ws(a, None, 1.0, 21)[0] == L.ERR_UNSUPPORTED  # m = 88: projected problem too large
    assert b"4*(k + k_extra)" in L.load().plhr_last_error()


def _ws_b(a, b, k=4, o=None):
    sz = C.c_size_t()
    code = L.load().plhr_workspace_size(C.byref(a), C.byref(b) if b is not None else None, None,
                                        1.0, k, C.byref(o) if o else None, C.byref(sz))
    return code, sz.value


def test_generalized_pencil_descriptors_are_validated_on_the_host():
    N = 16
    a = _fd3(N)
    n, kint = N ** 3, 5
    base = _ws_b(a, None)
    assert base[0] == L.OK
    d = L.OpDesc()
    d.kind, d.dtype, d.nx, d.ny, d.nz = L.OP_DIAG, L.F64, N, N, N
    d.potential = 4096                    # a device address; never read by the size query
    code, sz = _ws_b(a, d)
    assert code == L.OK and sz >= base[1] + (2 * n + 2 * n * kint) * 8
    d.potential = None
    assert _ws_b(a, d)[0] == L.ERR_ARG     # the diagonal is required
    d.potential, d.nz = 4096, N - 1
    assert _ws_b(a, d)[0] == L.ERR_ARG     # grid must match A
    q = L.OpDesc()
    q.kind, q.dtype, q.nx, q.ny, q.nz, q.h, q.scale = L.OP_Q1_3D, L.F64, N, N, N, 1 / (N + 1), 1.0
    mass = L.OpDesc()
    mass.kind, mass.dtype = L.OP_Q1_MASS, L.F64
    assert _ws_b(a, mass)[0] == L.ERR_ARG  # the consistent mass needs a Q1 A
    code, sz = _ws_b(q, mass)
    q_plain = _ws_b(q, None)
    assert code == L.OK and sz >= q_plain[1] + (n * 4 * kint + n * kint + n * 4) * 8
    d.nz = N
    assert _ws_b(q, d)[0] == L.ERR_UNSUPPORTED   # diagonal B with finite elements
    q2 = L.OpDesc()
    q2.kind, q2.dtype, q2.nx, q2.ny, q2.nz, q2.h, q2.scale = L.OP_Q1_2D, L.F64, N, N, 2, 0.1, 1.0
    assert _ws_b(q2, None)[0] == L.ERR_ARG       # 2-D needs nz = 1
    o = L.default_options()
    o.ortho_passes = 3
    assert _ws_b(a, None, o=o)[0] == L.ERR_ARG
    o.ortho_passes = 2
    assert _ws_b(a, None, o=o)[0] == L.OK


def test_csr_descriptors_are_validated_on_the_host():
    n = 4096
    a = L.OpDesc()
    a.kind, a.dtype, a.nx, a.ny, a.nz = L.OP_CSR, L.F64, n, 1, 1
    assert _ws_b(a, None)[0] == L.ERR_ARG              # arrays missing
    a.row_ptr, a.col_idx, a.values, a.nnz = 4096, 8192, 12288, 7 * n   # device addresses
    code, sz = _ws_b(a, None)
    assert code == L.OK and sz >= 3 * n * 4 * 5 * 8
    t = L.PrecDesc()
    t.kind, t.levels, t.nu_pre, t.nu_post, t.omega = L.PREC_MG_VCYCLE, 2, 2, 2, 2 / 3
    sz2 = C.c_size_t()
    code = L.load().plhr_workspace_size(C.byref(a), None, C.byref(t), 1.0, 4, None,
                                        C.byref(sz2))
    assert code == L.ERR_UNSUPPORTED                    # the V-cycle needs a grid
    b = L.OpDesc()
    b.kind, b.dtype, b.nx, b.ny, b.nz = L.OP_CSR, L.F64, n, 1, 1
    b.row_ptr, b.col_idx, b.values, b.nnz = 4096, 8192, 12288, n
    assert _ws_b(a, b)[0] == L.OK
    b.nx = n - 1
    assert _ws_b(a, b)[0] == L.ERR_ARG                  # n must match
    b.nx = n
    assert _ws_b(_fd3(16), b)[0] == L.ERR_ARG           # a CSR B needs a CSR A
    a.ny = 2
    assert _ws_b(a, None)[0] == L.ERR_ARG               # n = nx rows only


def test_bloch_op_apply_arguments_are_validated_on_the_host():
    """plhr_op_apply rejects bad descriptors before any launch; an empty
    block (ncols = 0) is a valid no-op."""
    lib = L.load()
    d = L.OpDesc()
    d.kind, d.dtype, d.nx, d.ny, d.nz, d.h, d.scale = L.OP_BLOCH7_3D, L.C128, 8, 8, 8, 1.0, 0.5
    d.theta[0], d.theta[1], d.theta[2] = 0.6, 1.2, 1.8
    X, Y = C.c_void_p(4096), C.c_void_p(4096 + 8 ** 3 * 4 * 16)   # device addresses
    assert lib.plhr_op_apply(C.byref(d), 0.0, X, Y, 0, None) == L.OK
    assert lib.plhr_op_apply(None, 0.0, X, Y, 4, None) == L.ERR_ARG
    assert lib.plhr_op_apply(C.byref(d), 0.0, None, Y, 4, None) == L.ERR_ARG
    assert lib.plhr_op_apply(C.byref(d), 0.0, X, C.c_void_p(4096 + 16), 4, None) == L.ERR_ARG
    assert lib.plhr_op_apply(C.byref(d), float("nan"), X, Y, 4, None) == L.ERR_ARG
    assert lib.plhr_op_apply(C.byref(d), 0.0, X, Y, -1, None) == L.ERR_ARG
    d.theta[1] = float("inf")
    assert lib.plhr_op_apply(C.byref(d), 0.0, X, Y, 4, None) == L.ERR_ARG
    d.theta[1] = 1.2
    d.h = 0.0
    assert lib.plhr_op_apply(C.byref(d), 0.0, X, Y, 4, None) == L.ERR_ARG
    d.h, d.nz = 1.0, 0
    assert lib.plhr_op_apply(C.byref(d), 0.0, X, Y, 4, None) == L.ERR_ARG
    d.nz, d.nx = 8, 1 << 20
    assert lib.plhr_op_apply(C.byref(d), 0.0, X, Y, 1 << 12, None) == L.ERR_ARG  # nx*ncols
    d.nx = 8
    d.dtype = L.F64
    assert lib.plhr_op_apply(C.byref(d), 0.0, X, Y, 4, None) == L.ERR_UNSUPPORTED
    d.dtype = L.C128
    f = _fd3(8)
    assert lib.plhr_op_apply(C.byref(f), 0.0, X, Y, 4, None) == L.ERR_UNSUPPORTED


def test_bloch_preconditioner_arguments_are_validated_on_the_host():
    """plhr_bloch_prec_create checks its descriptors, the coarsening and the
    positive definiteness of the coarse operator before touching the
    device: with every phase 0 the constant vector is in the null space."""
    lib = L.load()
    d = L.OpDesc()
    d.kind, d.dtype, d.nx, d.ny, d.nz, d.h, d.scale = L.OP_BLOCH7_3D, L.C128, 16, 16, 16, 1.0, 0.5
    t = L.PrecDesc()
    t.kind, t.levels, t.nu_pre, t.nu_post, t.omega = L.PREC_MG_VCYCLE, 3, 2, 2, 2 / 3
    h = C.c_void_p()

    def create(cols=8):
        return lib.plhr_bloch_prec_create(C.byref(d), C.byref(t), cols, None, None, 0,
                                          C.byref(h))
    assert create() == L.ERR_NOT_HPD                     # theta = 0: singular
    d.theta[0], d.theta[1], d.theta[2] = 0.6, 1.2, 1.8
    assert create(0) == L.ERR_ARG                        # max_cols
    t.nu_post = 1
    assert create() == L.ERR_ARG                         # T must be Hermitian
    t.nu_post, t.levels = 2, 6
    assert create() == L.ERR_ARG                         # 16 not divisible by 32
    t.levels = 40
    assert create() == L.ERR_ARG
    t.levels = 1
    assert create() == L.ERR_UNSUPPORTED                 # 4096 coarse points
    t.levels, t.omega = 3, 0.0
    assert create() == L.ERR_ARG
    t.omega, t.kind = 2 / 3, L.PREC_IDENTITY
    assert create() == L.ERR_UNSUPPORTED
    t.kind, d.dtype = L.PREC_MG_VCYCLE, L.F64
    assert create() == L.ERR_UNSUPPORTED
    assert lib.plhr_bloch_prec_apply(None, None, None, 0) == L.ERR_ARG


def test_complex_gram_arguments_are_validated_on_the_host():
    lib = L.load()
    sz = C.c_size_t()
    assert lib.plhr_gram_c128_workspace(1000, 128, 128, C.byref(sz)) == L.OK
    assert sz.value >= 128 * 128 * 8
    assert lib.plhr_gram_c128_workspace(-1, 4, 4, C.byref(sz)) == L.ERR_ARG
    assert lib.plhr_gram_c128_workspace(10, 0, 4, C.byref(sz)) == L.ERR_ARG
    assert lib.plhr_gram_c128_workspace(10, 4, 2000, C.byref(sz)) == L.ERR_ARG
    lib.plhr_gram_c128_workspace(1000, 8, 8, C.byref(sz))
    X, G, W = C.c_void_p(4096), C.c_void_p(1 << 20), C.c_void_p(1 << 24)
    assert lib.plhr_gram_c128(1000, X, 8, X, 8, G, W, sz.value - 1, None) == L.ERR_ARG
    assert lib.plhr_gram_c128(1000, X, 8, None, 8, G, W, sz.value, None) == L.ERR_ARG
    assert lib.plhr_gram_c128(1000, C.c_void_p(4104), 8, X, 8, G, W, sz.value, None) == L.ERR_ARG


def test_complex_cholqr_arguments_are_validated_on_the_host():
    lib = L.load()
    sz = C.c_size_t()
    assert lib.plhr_cholqr_c128_workspace(1000, 64, C.byref(sz)) == L.OK and sz.value > 0
    assert lib.plhr_cholqr_c128_workspace(1000, 65, C.byref(sz)) == L.ERR_ARG
    assert lib.plhr_cholqr_c128_workspace(10, 20, C.byref(sz)) == L.ERR_ARG   # n < m
    lib.plhr_cholqr_c128_workspace(1000, 8, C.byref(sz))
    Z, Q, W = C.c_void_p(4096), C.c_void_p(1 << 24), C.c_void_p(1 << 26)
    assert lib.plhr_cholqr_c128(1000, Z, 8, Q, None, W, sz.value - 1, None) == L.ERR_ARG
    assert lib.plhr_cholqr_c128(1000, Z, 8, C.c_void_p(4096 + 16), None, W, sz.value,
                                None) == L.ERR_ARG                            # overlap
    assert lib.plhr_cholqr_c128(1000, None, 8, Q, None, W, sz.value, None) == L.ERR_ARG


def test_complex_block_product_arguments_are_validated_on_the_host():
    lib = L.load()
    Z, M, Y = C.c_void_p(4096), C.c_void_p(1 << 24), C.c_void_p(1 << 26)
    assert lib.plhr_rowmul_c128(0, None, 8, None, 4, None, None) == L.OK     # no rows
    assert lib.plhr_rowmul_c128(100, Z, 65, M, 4, Y, None) == L.ERR_ARG
    assert lib.plhr_rowmul_c128(100, Z, 8, M, 0, Y, None) == L.ERR_ARG
    assert lib.plhr_rowmul_c128(100, Z, 8, None, 4, Y, None) == L.ERR_ARG
    assert lib.plhr_rowmul_c128(100, Z, 8, M, 4, C.c_void_p(4096 + 32), None) == L.ERR_ARG


def test_complex_product_and_cholqr_overlap_and_alignment_checks():
    lib = L.load()
    Z, M, Y = C.c_void_p(4096), C.c_void_p(1 << 24), C.c_void_p(1 << 26)
    # M overlapping Y, misaligned pointers
    assert lib.plhr_rowmul_c128(100, Z, 8, C.c_void_p((1 << 26) + 64), 4, Y, None) == L.ERR_ARG
    assert lib.plhr_rowmul_c128(100, C.c_void_p(4104), 8, M, 4, Y, None) == L.ERR_ARG
    assert lib.plhr_rowmul_c128(100, Z, 8, C.c_void_p((1 << 24) + 8), 4, Y, None) == L.ERR_ARG
    sz = C.c_size_t()
    lib.plhr_cholqr_c128_workspace(1000, 8, C.byref(sz))
    Q, W = C.c_void_p(1 << 24), C.c_void_p(1 << 26)
    for R in (C.c_void_p(4096 + 256), C.c_void_p((1 << 24) + 256), C.c_void_p((1 << 26) + 256)):
        assert lib.plhr_cholqr_c128(1000, Z, 8, Q, R, W, sz.value, None) == L.ERR_ARG


def test_projected_solve_arguments_are_validated_on_the_host():
    lib = L.load()
    sz = C.c_size_t()
    assert lib.plhr_projected_workspace(84, 21, C.byref(sz)) == L.OK and sz.value > 84 * 168 * 8
    assert lib.plhr_projected_workspace(85, 21, C.byref(sz)) == L.ERR_ARG
    assert lib.plhr_projected_workspace(8, 9, C.byref(sz)) == L.ERR_ARG
    assert lib.plhr_projected_workspace(8, 0, C.byref(sz)) == L.ERR_ARG
    lib.plhr_projected_workspace(16, 4, C.byref(sz))
    GL, GR = C.c_void_p(1 << 20), C.c_void_p(1 << 21)
    Y, xi, kd, pr = C.c_void_p(1 << 22), C.c_void_p(1 << 23), C.c_void_p(1 << 24), C.c_void_p(1 << 25)
    W = C.c_void_p(1 << 26)
    nex = C.c_int32()

    def call(**kw):
        a = dict(m=16, kint=4, GL=GL, GR=GR, keep=None, Y=Y, xi=xi, kinds=kd, pair=pr, W=W,
                 ws=sz.value)
        a.update(kw)
        return lib.plhr_projected_solve(a["m"], a["kint"], a["GL"], a["GR"], a["keep"], a["Y"],
                                        a["xi"], a["kinds"], a["pair"], C.byref(nex), a["W"],
                                        a["ws"], None)
    assert call(ws=sz.value - 1) == L.ERR_ARG
    assert call(W=None) == L.ERR_ARG
    assert call(W=C.c_void_p((1 << 26) + 8)) == L.ERR_ARG          # 256-byte alignment
    assert call(GR=None) == L.ERR_ARG
    assert call(GL=C.c_void_p((1 << 20) + 4)) == L.ERR_ARG         # misaligned
    assert call(Y=C.c_void_p((1 << 20) + 64)) == L.ERR_ARG         # Y overlaps G_L
    assert call(xi=C.c_void_p((1 << 22) + 8)) == L.ERR_ARG         # xi overlaps Y
    assert call(kinds=C.c_void_p((1 << 26) + 16)) == L.ERR_ARG     # kinds in the workspace
    assert call(m=100) == L.ERR_ARG


def test_single_vector_and_dense_preconditioner_options_are_validated_on_the_host():
    """PLHR_ALG_SINGLE (Algorithm 1) takes k = 1 and a basis of 8 real
    columns; PLHR_PREC_DENSE needs its matrix."""
    a = _fd3(16)
    n = 16 ** 3
    o = L.default_options()
    o.algorithm = L.ALG_SINGLE
    code, sz = _ws(a, None, 1.0, 1, o)
    assert code == L.OK and sz >= 3 * n * 8 * 8          # Z, QZ, TQZ of 8 real columns
    assert _ws(a, None, 1.0, 2, o)[0] == L.ERR_ARG         # one pair only
    assert b"k must be 1" in L.load().plhr_last_error()
    o.k_extra = 30                                         # ignored by the single iteration
    assert _ws(a, None, 1.0, 1, o)[0] == L.OK
    o.algorithm = 7
    assert _ws(a, None, 1.0, 1, o)[0] == L.ERR_ARG
    t = L.PrecDesc()
    t.kind = L.PREC_DENSE
    assert _ws(a, t, 1.0, 4)[0] == L.ERR_ARG               # no matrix
    t.matrix = 4096 + 4
    assert _ws(a, t, 1.0, 4)[0] == L.ERR_ARG               # misaligned
    t.matrix = 4096
    code_d, sz_d = _ws(a, t, 1.0, 4)
    code_i, sz_i = _ws(a, None, 1.0, 4)
    assert code_d == L.OK and sz_d == sz_i                 # no multigrid workspace
    t.kind = 9
    assert _ws(a, t, 1.0, 4)[0] == L.ERR_ARG


def test_plmr_option_is_validated_on_the_host():
    """PLHR_ALG_PLMR (Section 3.3) takes k = 1 and one real column per slot."""
    a = _fd3(16)
    n = 16 ** 3
    o = L.default_options()
    o.algorithm = L.ALG_PLMR
    code, sz = _ws(a, None, 1.0, 1, o)
    assert code == L.OK and sz >= 3 * n * 4 * 8          # Z, QZ, T(A - lam B)Z
    assert _ws(a, None, 1.0, 3, o)[0] == L.ERR_ARG
    assert b"k must be 1" in L.load().plhr_last_error()


def test_batch_and_bloch_workspace_queries_and_checks():
    """The batch and the Bloch V-cycle take caller workspaces: the size
    queries need no device, and a workspace that is too small or misaligned
    is refused before any device call."""
    lib = L.load()
    # Bloch V-cycle: levels 16^3, 8^3, 4^3 of 8 complex columns + the
    # 64 x 64 complex coarse inverse
    d = L.OpDesc()
    d.kind, d.dtype, d.nx, d.ny, d.nz, d.h, d.scale = L.OP_BLOCH7_3D, L.C128, 16, 16, 16, 1.0, 0.5
    d.theta[0], d.theta[1], d.theta[2] = 0.6, 1.2, 1.8
    t = L.PrecDesc()
    t.kind, t.levels, t.nu_pre, t.nu_post, t.omega = L.PREC_MG_VCYCLE, 3, 2, 2, 2 / 3
    sz = C.c_size_t()
    assert lib.plhr_bloch_prec_workspace_size(C.byref(d), C.byref(t), 8, C.byref(sz)) == L.OK
    lev = [16 ** 3, 8 ** 3, 4 ** 3]
    want = 2 * lev[0] * 8 * 16 + 3 * (lev[1] + lev[2]) * 8 * 16 + 64 * 64 * 16
    assert sz.value == want
    h = C.c_void_p()
    assert lib.plhr_bloch_prec_create(C.byref(d), C.byref(t), 8, None, C.c_void_p(4096),
                                      sz.value - 1, C.byref(h)) == L.ERR_ARG
    assert lib.plhr_bloch_prec_create(C.byref(d), C.byref(t), 8, None, C.c_void_p(4096 + 8),
                                      sz.value, C.byref(h)) == L.ERR_ARG
    assert lib.plhr_bloch_prec_workspace_size(C.byref(d), C.byref(t), 0, C.byref(sz)) == L.ERR_ARG
    # batch of two 2-D problems with a 3-level V-cycle
    descs = (L.OpDesc * 2)()
    for b, N in enumerate((32, 16)):
        descs[b].kind, descs[b].dtype, descs[b].nx, descs[b].ny, descs[b].nz = (
            L.OP_FD5_2D, L.F64, N, N, 1)
        descs[b].h, descs[b].scale = 1.0, 0.5
    tb = L.PrecDesc()
    tb.kind, tb.levels, tb.nu_pre, tb.nu_post, tb.omega = L.PREC_MG_VCYCLE, 3, 2, 2, 2 / 3
    sig = (C.c_double * 2)(0.1, 0.2)
    o = L.default_options()
    assert lib.plhr_batch_workspace_size(2, descs, C.byref(tb), sig, 4, C.byref(o),
                                         C.byref(sz)) == L.OK
    n, m, kint = 32 * 32 + 16 * 16, 20, 5
    assert sz.value >= 3 * n * m * 8                       # Z, QZ, TQZ at least
    hb = C.c_void_p()
    assert lib.plhr_batch_create(2, descs, C.byref(tb), sig, 4, C.byref(o), None,
                                 C.c_void_p(4096), sz.value - 8, C.byref(hb)) == L.ERR_ARG
    assert lib.plhr_batch_create(2, descs, C.byref(tb), sig, 4, C.byref(o), None,
                                 C.c_void_p(4096 + 64), sz.value, C.byref(hb)) == L.ERR_ARG
    assert lib.plhr_batch_workspace_size(2, descs, C.byref(tb), sig, 0, C.byref(o),
                                         C.byref(sz)) == L.ERR_ARG


def test_bloch_solver_options_are_validated_on_the_host():
    """The solver takes the Bloch operator (the block iteration in complex
    arithmetic): B = I, T the identity or its V-cycle, FP64, the block
    algorithm, 8 (k + k_extra) <= 84; the workspace query makes no device
    call and grows with the V-cycle's levels."""
    d = L.OpDesc()
    d.kind, d.dtype, d.nx, d.ny, d.nz, d.h, d.scale = L.OP_BLOCH7_3D, L.C128, 8, 8, 8, 1.0, 0.5
    d.theta[0], d.theta[1], d.theta[2] = 0.6, 1.2, 1.8
    code, sz0 = _ws_b(d, None, k=3)
    assert code == L.OK
    n, kint = 512, 2 * 4
    assert sz0 >= 3 * n * 4 * kint * 8 + 2 * n * 2 * kint * 8   # Z, QZ, TQZ, staging
    t = L.PrecDesc()
    t.kind, t.levels, t.nu_pre, t.nu_post, t.omega = L.PREC_MG_VCYCLE, 3, 2, 2, 2 / 3
    code, sz1 = _ws(d, t, 0.0, 3)
    assert code == L.OK and sz1 > sz0
    t.levels = 5                                   # 8 not divisible by 2^4
    assert _ws(d, t, 0.0, 3)[0] == L.ERR_ARG
    t.levels, t.kind = 3, L.PREC_AV_MG
    assert _ws(d, t, 0.0, 3)[0] == L.ERR_UNSUPPORTED
    assert b"identity or PLHR_PREC_MG_VCYCLE" in L.load().plhr_last_error()
    assert _ws_b(d, None, k=9)[0] == L.OK              # 8 * 10 = 80
    assert _ws_b(d, None, k=10)[0] == L.ERR_UNSUPPORTED   # 8 * 11 > 84
    assert b"8*(k + k_extra)" in L.load().plhr_last_error()
    o = L.default_options()
    o.precision = L.PRECISION_MIXED
    assert _ws_b(d, None, k=3, o=o)[0] == L.ERR_UNSUPPORTED
    o = L.default_options()
    o.algorithm = L.ALG_SINGLE
    assert _ws_b(d, None, k=1, o=o)[0] == L.ERR_UNSUPPORTED
    b = L.OpDesc()
    b.kind, b.dtype, b.nx, b.ny, b.nz = L.OP_DIAG, L.F64, 8, 8, 8
    b.potential = 4096
    assert _ws_b(d, b, k=3)[0] == L.ERR_UNSUPPORTED
    d.dtype = L.F64
    assert _ws_b(d, None, k=3)[0] == L.ERR_UNSUPPORTED
