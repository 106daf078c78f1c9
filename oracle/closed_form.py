"""Discrete spectrum for constant permittivity (derived from the Section-3 discretization).

For epsilon = eps0 on the whole cell, the Bloch-periodic discrete plane waves
  u_x(j1, j2) = X exp(i (q1 (j1 + 1/2) h1 + q2 j2 h2)),
  u_y(j1, j2) = Y exp(i (q1 j1 h1 + q2 (j2 + 1/2) h2)),
with q = k + 2 pi (p/a, r/b), p in [0:n), r in [0:m), diagonalise the pencil (A, M) into
2x2 blocks.  Each block has one zero eigenvalue (the discrete gradient) and

  lambda_h(q) = (1/eps0) [ (4/h1^2) s1 / (1 - 2/3 s1) + (4/h2^2) s2 / (1 - 2/3 s2) ],
  s_i = sin^2(q_i h_i / 2),

(both zero for q = 0, which only occurs at k = 0).  As h -> 0 this tends to
|k + G|^2 / eps0 with an O(h^2) error, the continuum Bloch spectrum.

Pinned by: the dense generalized eigensolve of the assembled pencil (tests); it is an
independent derivation (Fourier analysis of the stencils), not a re-statement of them.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = ["discrete_nonzero", "continuum"]


def discrete_nonzero(n: int, m: int, a: float, b: float, eps0: float, k1: float, k2: float,
                     count: int | None = None) -> np.ndarray:
    """Ascending non-zero discrete eigenvalues (with multiplicity) for constant eps0."""
    h1, h2 = a / n, b / m
    p = np.arange(n)
    r = np.arange(m)
    q1 = k1 + 2 * math.pi * p / a
    q2 = k2 + 2 * math.pi * r / b
    s1 = np.sin(q1 * h1 / 2) ** 2
    s2 = np.sin(q2 * h2 / 2) ** 2
    S1, S2 = np.meshgrid(s1, s2, indexing="xy")
    lam = (4.0 / h1 ** 2) * S1 / (1 - 2.0 / 3.0 * S1) + (4.0 / h2 ** 2) * S2 / (1 - 2.0 / 3.0 * S2)
    lam = np.sort(lam.reshape(-1)) / eps0
    # q = 0 (only at the Gamma point) gives the extra zero eigenvalue
    scale = lam.max() if lam.size else 1.0
    lam = lam[lam > 1e-12 * scale]
    return lam if count is None else lam[:count]


def continuum(a: float, b: float, eps0: float, k1: float, k2: float, count: int,
              span: int = 12) -> np.ndarray:
    """Smallest non-zero |k + G|^2 / eps0 over reciprocal vectors G = 2 pi (p/a, r/b)."""
    p = np.arange(-span, span + 1)
    P, R = np.meshgrid(p, p, indexing="xy")
    lam = ((k1 + 2 * math.pi * P / a) ** 2 + (k2 + 2 * math.pi * R / b) ** 2) / eps0
    lam = np.sort(lam.reshape(-1))
    lam = lam[lam > 1e-12]
    return lam[:count]
