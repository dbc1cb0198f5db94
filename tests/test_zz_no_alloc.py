"""The allocation-free projected step (plhr_projected_solve_noalloc):
same results as plhr_projected_solve, which takes a caller workspace, on
two calls in a row, the second with a smaller problem (the file-scope
scratch keeps the first call's contents)."""
import ctypes as C

import numpy as np
import pytest
import torch

from tests import pencils
from tests.gpu_util import dev, host

pytestmark = pytest.mark.gpu


def _noalloc(GL, GR, kint):
    from paper_1408_0042_amd import _lib as L
    lib = L.load()
    f = lib.plhr_projected_solve_noalloc
    P = C.c_void_p
    m = GL.shape[0]
    Y = torch.full((m, kint), np.nan, dtype=torch.float64, device="cuda")
    xi = torch.full((2, m), np.nan, dtype=torch.float64, device="cuda")
    kinds = torch.full((kint,), -7, dtype=torch.int32, device="cuda")
    pair = torch.full((kint,), -7, dtype=torch.int32, device="cuda")
    status = torch.full((2,), -1, dtype=torch.int32, device="cuda")
    L.check(f(m, kint, P(GL.data_ptr()), P(GR.data_ptr()), None, P(Y.data_ptr()),
              P(xi.data_ptr()), P(kinds.data_ptr()), P(pair.data_ptr()), P(status.data_ptr()),
              P(torch.cuda.current_stream().cuda_stream)))
    return host(Y), host(xi), host(kinds), host(pair), host(status)


def test_noalloc_scratch_size_is_stated():
    from paper_1408_0042_amd import _lib as L
    assert 0 < L.load().plhr_projected_noalloc_scratch_bytes() <= 400 * 1024


def test_noalloc_projected_step_matches_workspace_version():
    from paper_1408_0042_amd.plhr import projected_solve
    for m, kint, seed in ((84, 21, 5), (36, 9, 6)):
        print(f"noalloc m={m} kint={kint}", flush=True)
        units = pencils.spectrum(m, kint, seed, cut_pair=True)
        GLh, GRh, _, _ = pencils.projected_pencil(units, seed + 1, cond="ortho")
        GL, GR = dev(GLh), dev(GRh)
        Yw, xiw, kw, pw, nex = projected_solve(GL, GR, kint)
        Yn, xin, kn, pn, st = _noalloc(GL, GR, kint)
        assert st.tolist() == [0, 0]
        assert np.array_equal(host(Yw), Yn)
        assert np.array_equal(host(torch.stack([xiw.real, xiw.imag])), xin)
        assert np.array_equal(host(kw), kn) and np.array_equal(host(pw), pn)
        assert 2 in kn.tolist()          # the cut pair's ytilde column is there
