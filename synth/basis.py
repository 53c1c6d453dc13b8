"""One-dimensional spectral finite-element ingredients (Sec. III.B).

Spectral hexahedral elements of degree p put their nodes on the
Gauss-Lobatto-Legendre (GLL) points: the two interval ends plus the roots of
the derivative of the Legendre polynomial P_p.  The GLL rule on those same
points integrates polynomials exactly up to degree 2(p+1)-3 and is used only
for the classical overlap block, which it makes diagonal; every other
integral uses ordinary Gauss-Legendre quadrature (exact to degree 2n-1).
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as npleg


def legendre(p: int, x: np.ndarray) -> np.ndarray:
    """Legendre polynomial P_p evaluated at x."""
    c = np.zeros(p + 1)
    c[p] = 1.0
    return npleg.legval(x, c)


def gll_rule(p: int) -> tuple[np.ndarray, np.ndarray]:
    """GLL nodes and weights for degree p on [-1, 1] (p + 1 points).

    Interior nodes are the roots of P_p'(x) (found from the Legendre-series
    derivative and polished by Newton steps); weights are
    2 / (p (p + 1) P_p(x_i)^2).
    """
    if p < 1:
        raise ValueError("GLL rule needs p >= 1")
    c = np.zeros(p + 1)
    c[p] = 1.0
    dc = npleg.legder(c)
    if p >= 2:
        interior = np.sort(npleg.legroots(dc).real)
        d2c = npleg.legder(dc)
        for _ in range(5):
            interior = interior - npleg.legval(interior, dc) / npleg.legval(interior, d2c)
        x = np.concatenate([[-1.0], interior, [1.0]])
    else:
        x = np.array([-1.0, 1.0])
    w = 2.0 / (p * (p + 1) * legendre(p, x) ** 2)
    return x, w


def gauss_rule(n: int) -> tuple[np.ndarray, np.ndarray]:
    """n-point Gauss-Legendre rule on [-1, 1]."""
    return npleg.leggauss(n)


def lagrange_eval(nodes: np.ndarray, x: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Lagrange basis through `nodes`: values and derivatives at points x.

    Returns (L, dL) of shape [len(x), len(nodes)], with L[q, i] = l_i(x_q).
    Uses the product form directly (the degrees here are small).
    """
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64).reshape(-1)
    k = nodes.size
    diff = x[:, None] - nodes[None, :]                       # [Q, k]
    L = np.empty((x.size, k))
    dL = np.empty((x.size, k))
    for i in range(k):
        others = [j for j in range(k) if j != i]
        denom = np.prod(nodes[i] - nodes[others])
        terms = diff[:, others]                                # [Q, k-1]
        L[:, i] = np.prod(terms, axis=1) / denom
        acc = np.zeros(x.size)
        for t in range(k - 1):
            rest = np.delete(terms, t, axis=1)
            acc += np.prod(rest, axis=1)
        dL[:, i] = acc / denom
    return L, dL
