"""Chebyshev filter (Sec. V), oracle side (test infrastructure).

The filter maps [a, b] onto [-1, 1] with t(x) = (2x - a - b)/(b - a) and
applies the degree-m Chebyshev polynomial of t(H~) to a block, H~ = M^-1 H.
Degree m means m applications of H~ (p_0 = identity).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def chebyshev_T(m: int, x: np.ndarray) -> np.ndarray:
    """T_m(x) in closed form: cos(m arccos x) on [-1,1], cosh(m arccosh|x|) sign(x)^m outside."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty_like(x)
    inside = np.abs(x) <= 1.0
    out[inside] = np.cos(m * np.arccos(x[inside]))
    xo = x[~inside]
    out[~inside] = np.cosh(m * np.arccosh(np.abs(xo))) * np.sign(xo) ** m
    return out


def recurrence_filter(apply_Htilde, X: np.ndarray, m: int, a: float, b: float) -> np.ndarray:
    """p_m(t(H~)) X by the three-term recurrence p_{k+1} = 2 t p_k - p_{k-1}."""
    if m < 0 or not b > a:
        raise ValueError("need m >= 0 and b > a")
    if not hasattr(X, "clone"):       # numpy input (torch CPU tensors pass through)
        X = np.asarray(X, dtype=np.float64)
    if m == 0:
        return X.clone() if hasattr(X, "clone") else X.copy()
    e = 2.0 / (b - a)             # t(H~) Y = e H~ Y - c Y
    c = (a + b) / (b - a)
    p_prev = X
    p = e * apply_Htilde(X) - c * X
    for _ in range(1, m):
        p_next = 2.0 * (e * apply_Htilde(p) - c * p) - p_prev
        p_prev, p = p, p_next
    return p


def exact_filter(Hd: np.ndarray, Md: np.ndarray, X: np.ndarray, m: int,
                 a: float, b: float) -> np.ndarray:
    """V T_m(t(Lambda)) V^T M X with H V = M V Lambda, V^T M V = I (dense)."""
    lam, V = sla.eigh(Hd, Md)
    f = chebyshev_T(m, (2.0 * lam - a - b) / (b - a))
    return V @ (f[:, None] * (V.T @ (Md @ X)))
