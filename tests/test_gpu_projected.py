"""GPU parity of the projected step (eq. (3.5) and the selection of
Algorithm 3) through plhr_projected_solve, on synthetic pencils with a
prescribed spectrum, against the oracle's sorted_tharmonic +
real_selection.  Cases: widths m = 8 ... 84, a conjugate pair cut by the
block size (the ytilde_R column), equal moduli, a singular G_R (tau = 0)
and dropped slots."""
import numpy as np
import pytest
import torch

from oracle import dense, plhr
from tests import pencils
from tests.gpu_util import dev, host

pytestmark = pytest.mark.gpu


def _in_span(y, S):
    c, *_ = np.linalg.lstsq(S, y, rcond=None)
    return np.linalg.norm(y - S @ c) / np.linalg.norm(y)


def _gpu(GL, GR, kint, keep=None):
    from paper_1408_0042_amd.plhr import projected_solve
    kp = None if keep is None else dev(np.asarray(keep, dtype=np.int32))
    Y, xi, kinds, pair, nex = projected_solve(dev(GL), dev(GR), kint, kp)
    return host(Y), host(xi), host(kinds), host(pair), nex


KIND = {"real": 0, "R": 1, "tilde": 2, "I": 3}


def _check(GL, GR, kint, ties, keep=None):
    m = GL.shape[0]
    sel = np.arange(m) if keep is None else np.flatnonzero(keep)
    GLk, GRk = GL[np.ix_(sel, sel)], GR[np.ix_(sel, sel)]
    xo, Yo, unit = plhr.sorted_tharmonic(GLk, GRk, real_pairs=True)
    Ypo, ko, po = plhr.real_selection(xo, Yo, unit, kint)
    Yg, xg, kg, pg, nex = _gpu(GL, GR, kint, keep)
    assert nex == 0
    nk = len(sel)
    # dropped slots carry zero rows
    if keep is not None:
        assert np.all(Yg[np.flatnonzero(np.asarray(keep) == 0)] == 0.0)
    Yg = Yg[sel]
    # the sorted xi of the selected units agree with the oracle's (the GPU
    # lists one entry per unit: a pair by its Im xi > 0 member)
    xo_u = xo[unit == np.arange(len(unit))]
    nsel = sum(1 for k in ko if k != "I")
    fin = np.isfinite(xo_u)
    assert np.all(np.isfinite(xg[:nsel]))
    scale = np.abs(xo_u[fin]).max()
    if ties:
        key = lambda z: np.lexsort((np.round(z.imag, 9), np.round(z.real, 9)))
        a, b = xg[:nsel], xo_u[:nsel]
        assert np.allclose(a[key(a)], b[key(b)], rtol=1e-10, atol=1e-12 * scale)
    else:
        assert np.allclose(xg[:nsel], xo_u[:nsel], rtol=1e-10, atol=1e-12 * scale)
    # the same column layout (kinds, partners)
    assert sorted(kg.tolist()) == sorted(KIND[k] for k in ko)
    if not ties:
        assert kg.tolist() == [KIND[k] for k in ko]
        assert pg.tolist() == po
    # span of Y' agrees with the oracle's, leaving out the ytilde_R column:
    # the real part of a complex eigenvector depends on its phase, so any
    # vector of the pair's real invariant subspace is a correct ytilde_R
    # (checked below)
    cg = [c for c in range(kint) if kg[c] != 2]
    co = [c for c in range(kint) if ko[c] != "tilde"]
    assert dense.subspace_sine(Ypo[:, co], Yg[:, cg]) < 1e-9
    # column by column: eigenvectors of their own xi; ytilde in the pair's
    # real invariant subspace
    nrm = np.linalg.norm(GLk)
    for c in range(kint):
        if kg[c] == 0:
            y = Yg[:, c]
            assert abs(np.linalg.norm(y) - 1.0) < 1e-12
            lam = np.vdot(y, GLk @ y) / np.vdot(y, GRk @ y)
            r = GLk @ y - lam * (GRk @ y)
            assert np.linalg.norm(r) <= 1e-10 * nrm
        elif kg[c] == 1:
            y = Yg[:, c] + 1j * Yg[:, pg[c]]
            assert abs(np.linalg.norm(y) - 1.0) < 1e-12
            resid = min(np.linalg.norm(GLk @ y - z * (GRk @ y)) for z in xo[:kint + 1]
                        if z.imag > 0)
            assert resid <= 1e-10 * nrm
        elif kg[c] == 2:
            # the oracle's pair vector of the cut unit: Re/Im of Yo at kint-1
            S = np.column_stack([Yo[:, kint - 1].real, Yo[:, kint - 1].imag])
            assert _in_span(Yg[:, c], S) < 1e-9


CASES = [(8, 2, True, False, 0), (36, 9, True, True, 0), (68, 17, False, True, 2),
         (80, 20, True, False, 2), (84, 21, False, False, 0), (84, 21, True, True, 3)]


@pytest.mark.parametrize("m,kint,cut,ties,singular", CASES)
def test_projected_step_matches_oracle(m, kint, cut, ties, singular):
    print(f"projected m={m} kint={kint} cut={cut} ties={ties} singular={singular}", flush=True)
    units = pencils.spectrum(m, kint, 100 + m, cut_pair=cut, ties=ties, singular=singular)
    GL, GR, mm, _ = pencils.projected_pencil(units, 200 + m, cond="ortho")
    assert mm == m
    _check(GL, GR, kint, ties)


def test_projected_step_with_dropped_slots():
    """Slots masked out by the orthonormalisation: the problem is posed on
    the kept slots alone (their rows and columns of G_L, G_R)."""
    m, kint = 40, 10
    units = pencils.spectrum(m, kint, 7, cut_pair=True)
    GL, GR, _, _ = pencils.projected_pencil(units, 8, cond="ortho")
    keep = np.ones(m, dtype=np.int32)
    keep[[3, 17, 31]] = 0
    print("projected dropped slots m=40", flush=True)
    _check(GL, GR, kint, False, keep)


def test_projected_step_rejects_bad_arguments():
    from paper_1408_0042_amd import _lib as L
    from paper_1408_0042_amd.plhr import projected_solve
    G = dev(np.eye(90))
    with pytest.raises(L.PLHRError):
        projected_solve(G, G, 10)          # m = 90 > 84
    G = dev(np.eye(8))
    with pytest.raises(L.PLHRError):
        projected_solve(G, G, 9)           # kint > m
