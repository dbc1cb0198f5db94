"""Synthetic projected pencils (G_L, G_R) with a prescribed T-harmonic
spectrum, for the selection pins of the oracle and the GPU parity of the
projected step.  Construction only: G_L = L L^T symmetric positive
definite, C = X J X^-1 with J real block diagonal (a 2 x 2 block per
conjugate pair), G_R = L C L^T, so that G_L y = xi G_R y exactly when
C u = (1/xi) u with u = L^T y."""
import numpy as np
import scipy.linalg as sla


def projected_pencil(xis, seed, cond=None):
    """xis: sequence of xi values, a complex entry standing for the pair
    (xi, conj xi), np.inf for tau = 0 (a singular G_R).  cond=None mixes
    with X = randn + 2 I; cond='ortho' with a perturbed orthogonal X
    (well conditioned at any size).  Returns (GL, GR, m, Yb): Yb[i] spans
    in y the real invariant subspace of entry i."""
    rng = np.random.default_rng(seed)
    sizes = [2 if (np.iscomplexobj(x) and np.imag(x) != 0) else 1 for x in xis]
    m = sum(sizes)
    J = np.zeros((m, m))
    pos = 0
    for x, s in zip(xis, sizes):
        tau = 0.0 if not np.isfinite(x) else 1.0 / complex(x)
        if s == 1:
            J[pos, pos] = np.real(tau)
        else:
            J[pos:pos + 2, pos:pos + 2] = [[tau.real, tau.imag], [-tau.imag, tau.real]]
        pos += s
    if cond == "ortho":
        Q, _ = np.linalg.qr(rng.standard_normal((m, m)))
        X = Q + (0.2 / np.sqrt(m)) * rng.standard_normal((m, m))
    else:
        X = rng.standard_normal((m, m)) + 2.0 * np.eye(m)
    C = X @ J @ np.linalg.inv(X)
    F = rng.standard_normal((m, m))
    GL = F @ F.T + m * np.eye(m)
    L = np.linalg.cholesky(GL)
    GR = L @ C @ L.T
    Yb, pos = [], 0
    for s in sizes:
        Yb.append(sla.solve_triangular(L.T, X[:, pos:pos + s], lower=False))
        pos += s
    return GL, GR, m, Yb


def spectrum(m, kint, seed, cut_pair=False, ties=False, singular=0, pair_frac=0.3):
    """A list of xi units filling m positions with increasing moduli.  With
    cut_pair the unit starting at position kint - 1 (0-based) is a
    conjugate pair, so the selection of kint columns cuts it (ytilde_R);
    otherwise a pair never straddles position kint.  ties adds a real
    -r / +r couple of equal modulus inside the selection.  singular puts
    that many tau = 0 units (xi = inf) at the end."""
    rng = np.random.default_rng(seed)
    units, pos, j = [], 0, 0
    while pos < m - singular:
        r = 0.05 * (1 + j + 0.5 * rng.random())      # strictly increasing
        j += 1
        left = m - singular - pos
        want_pair = rng.random() < pair_frac and left >= 2
        if pos == kint - 1:
            want_pair = cut_pair and left >= 2
        elif pos == kint - 2 and cut_pair:
            want_pair = False          # land exactly on kint - 1
        if want_pair:
            ang = rng.uniform(0.2, 1.2)
            units.append(complex(r * np.cos(ang), r * np.sin(ang)) * (1 if rng.random() < 0.5 else -1))
            pos += 2
        else:
            units.append(r * (1 if rng.random() < 0.5 else -1))
            pos += 1
    if ties and kint >= 4:
        # two consecutive real units inside the selection become -r0, +r0
        # (r0 the first one's modulus), so the order of the others is kept
        pos = 0
        for i in range(len(units) - 1):
            a, b = units[i], units[i + 1]
            if (not isinstance(a, complex) and not isinstance(b, complex)
                    and pos + 1 < kint - 2):
                r0 = abs(a)
                units[i], units[i + 1] = -r0, r0
                break
            pos += 2 if isinstance(a, complex) else 1
    units += [np.inf] * singular
    return units
