"""Closed-form spectra of the model operators, used to pin the oracle.

These follow from separation of variables and are independent of any code
under test:

* d-dim 5/7-point Dirichlet Laplacian, N_a interior points, spacing h:
      lam = sum_a (4/h^2) sin^2(i_a pi / (2 (N_a + 1))),  i_a = 1..N_a,
  eigenvectors prod_a sin(i_a pi x_a / (N_a + 1)).
* Bloch-periodic version, N_a points, phase theta_a per period:
      lam = sum_a (4/h^2) sin^2((2 pi m_a + theta_a) / (2 N_a)),  m_a = 0..N_a-1.
* Bilinear / trilinear finite elements, uniform mesh of the unit box with
  Nel elements per side, Dirichlet (interior nodes i = 1..Nel-1) or
  natural (all nodes, i = 0..Nel): the generalized pencil (K, M) has
      lam = sum_a mu_{i_a},  mu_i = (6/h^2) (1 - cos t_i) / (2 + cos t_i),
  t_i = i pi h, h = 1/Nel (tensor products of the 1-D linear-element
  pencil, whose eigenvectors are sines resp. cosines).
"""
import itertools
import math

import numpy as np


def fd_dirichlet_eigs(dims, h, scale=1.0):
    per = [np.array([(4.0 / h**2) * math.sin(i * math.pi / (2 * (N + 1))) ** 2
                     for i in range(1, N + 1)]) for N in dims]
    tot = per[0]
    for p in per[1:]:
        tot = np.add.outer(tot, p).ravel()
    return np.sort(scale * tot)


def fd_dirichlet_mode(dims, idx):
    """Eigenvector for mode indices idx (1-based), x-fastest numbering."""
    vecs = [np.sin(np.arange(1, N + 1) * i * math.pi / (N + 1)) for N, i in zip(dims, idx)]
    v = vecs[-1]
    for w in reversed(vecs[:-1]):
        v = np.kron(v, w)
    return v


def bloch_eigs(dims, h, thetas, scale=0.5):
    per = [np.array([(4.0 / h**2) * math.sin((2 * math.pi * m + t) / (2 * N)) ** 2
                     for m in range(N)]) for N, t in zip(dims, thetas)]
    tot = per[0]
    for p in per[1:]:
        tot = np.add.outer(tot, p).ravel()
    return np.sort(scale * tot)


def fe_q1_eigs(Nel, d, bc="dirichlet"):
    h = 1.0 / Nel
    idx = range(1, Nel) if bc == "dirichlet" else range(0, Nel + 1)
    mu = np.array([(6.0 / h**2) * (1 - math.cos(i * math.pi * h)) / (2 + math.cos(i * math.pi * h))
                   for i in idx])
    tot = mu
    for _ in range(d - 1):
        tot = np.add.outer(tot, mu).ravel()
    return np.sort(tot)
