"""Orthonormalisation, Rayleigh-Ritz and spectrum bounds (Sec. V), oracle side.

Test infrastructure only.  Steps follow the paper's order: filter the block,
orthonormalise it (here Cholesky-QR, applied twice, after scaling columns to
unit length: a diagonal scaling that leaves the span unchanged), project the
pencil (H, M) onto it, solve the small generalized problem with a dense
direct solver and rotate back.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def cholqr(Y: np.ndarray, passes: int = 2) -> np.ndarray:
    """Q with Q^T Q = I and span(Q) = span(Y) by (repeated) Cholesky-QR."""
    Q = np.asarray(Y, dtype=np.float64)
    Q = Q / np.linalg.norm(Q, axis=0)[None, :]
    for _ in range(passes):
        G = Q.T @ Q
        R = sla.cholesky(0.5 * (G + G.T), lower=False)        # G = R^T R
        Q = sla.solve_triangular(R, Q.T, trans="T", lower=False).T   # Q R^-1
    return Q


def rayleigh_ritz(Q: np.ndarray, HQ: np.ndarray, MQ: np.ndarray):
    """Ritz values (ascending) and coefficient matrix C of the pencil (Q^T H Q, Q^T M Q)."""
    Hh = Q.T @ HQ
    Mh = Q.T @ MQ
    theta, C = sla.eigh(0.5 * (Hh + Hh.T), 0.5 * (Mh + Mh.T))
    return theta, C


def lanczos(apply_Htilde, apply_M, v0: np.ndarray, k: int):
    """k-step Lanczos on H~ = M^-1 H in the M inner product.

    H~ is self-adjoint in <x, y>_M = x^T M y, so the Arnoldi process reduces
    to Lanczos.  Returns (alpha[k], beta[k]) where beta[j] is the M-norm of
    the residual after step j (beta[k-1] = ||f_k||_M).
    """
    v = np.asarray(v0, dtype=np.float64)
    v = v / np.sqrt(v @ apply_M(v))
    v_prev = np.zeros_like(v)
    beta_prev = 0.0
    alpha = np.zeros(k)
    beta = np.zeros(k)
    for j in range(k):
        w = apply_Htilde(v) - beta_prev * v_prev
        alpha[j] = w @ apply_M(v)
        w = w - alpha[j] * v
        beta[j] = np.sqrt(max(w @ apply_M(w), 0.0))
        if beta[j] == 0.0:
            return alpha[:j + 1], beta[:j + 1]
        v_prev, v = v, w / beta[j]
        beta_prev = beta[j]
    return alpha, beta


def lanczos_bounds(alpha: np.ndarray, beta: np.ndarray) -> tuple[float, float]:
    """(smallest Ritz value, upper bound theta_max + ||f_k||_M) of the tridiagonal T_k."""
    T = np.diag(alpha)
    if alpha.size > 1:
        T += np.diag(beta[:-1], 1) + np.diag(beta[:-1], -1)
    ev = np.linalg.eigvalsh(T)
    return float(ev[0]), float(ev[-1] + beta[-1])


# ------------------------------------------------------------------ metrics
def ritz_error(theta: np.ndarray, lam_ref: np.ndarray, wanted: int) -> float:
    """max_{i < wanted} |theta_i - lambda_i| (both ascending)."""
    return float(np.max(np.abs(np.asarray(theta)[:wanted] - np.asarray(lam_ref)[:wanted])))


def energy_error(theta: np.ndarray, lam_ref: np.ndarray, wanted: int) -> float:
    """2 |sum theta_i - sum lambda_i| over the wanted set: the band-energy
    term sum_i f_i eps_i with two electrons per state (Sec. II, unit
    occupancy below the wanted edge)."""
    return float(2.0 * abs(np.sum(np.asarray(theta)[:wanted]) - np.sum(np.asarray(lam_ref)[:wanted])))


def subspace_angle(A: np.ndarray, B: np.ndarray, M) -> float:
    """Largest principal angle between span(B) and span(A) in the inner
    product <x, y>_M = x^T M y (dim span(B) <= dim span(A)).

    With Qa, Qb M-orthonormal bases, the M-orthogonal projector onto span(A)
    is Qa Qa^T M; the sine of the largest angle is the M-norm of what it
    leaves of Qb: sin = ||(I - Qa Qa^T M) Qb||_M.  Taken as the arcsine (an
    arccosine of the smallest cosine cannot resolve angles below ~1e-8)."""
    def orth(X):
        G = X.T @ (M @ X)
        Lc = sla.cholesky(0.5 * (G + G.T), lower=True)
        return sla.solve_triangular(Lc, X.T, lower=True).T
    Qa, Qb = orth(np.asarray(A, dtype=np.float64)), orth(np.asarray(B, dtype=np.float64))
    Rb = Qb - Qa @ (Qa.T @ (M @ Qb))
    G = Rb.T @ (M @ Rb)
    s2 = float(np.linalg.eigvalsh(0.5 * (G + G.T))[-1])
    return float(np.arcsin(min(1.0, np.sqrt(max(s2, 0.0)))))


def scf_step(ops, X: np.ndarray, m: int, a: float, b: float, how: str = "block"):
    """One filter -> Cholesky-QR -> Rayleigh-Ritz pass; returns (theta, Ritz vectors)."""
    from .filters import recurrence_filter
    Y = recurrence_filter(lambda Z: ops.apply_Htilde(Z, how), X, m, a, b)
    Q = cholqr(Y)
    theta, C = rayleigh_ritz(Q, ops.apply_H(Q), ops.apply_M(Q))
    return theta, Q @ C
