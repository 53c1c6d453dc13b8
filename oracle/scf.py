"""The self-consistent field quantities around the eigensolver (oracle; test
infrastructure only).

Section II and Section V of the paper.  All fields live on the quadrature
points of the cells: the plain cells' Gauss points and the adaptive grid's
points (Sec. IV.C).  w_q are the weights (Jacobian included).

* Occupations and Fermi level (Eq. FermiDirac, Eq. Mu):
  f(e, mu) = 1 / (1 + exp((e - mu) / kT)), with mu fixed by 2 sum_i f_i = N_e.
  Found by bisection.
* Electron density (Eq. Rho): rho(x) = 2 sum_i f_i psi_i(x)^2, where
  psi_i = sum_a N_a X[a, i] + sum_al N_al X[al, i].
* Exchange-correlation (Sec. II: LDA, Ceperley-Alder).  The correlation uses
  the Perdew-Zunger parametrisation of the Ceperley-Alder data, spin
  unpolarised (Phys. Rev. B 23, 5048 (1981)); exchange is the Slater form.
  eps_xc(rho) per electron, and V_xc = d(rho eps_xc) / d rho.
* Hartree potential (Eq. Hartree_possion, discretised as Eq.
  discretePoissonCFEM): (1/4 pi) int grad V_H . grad N_j = int rho N_j, with
  zero Dirichlet values on the box.  The box boundary is at finite
  distance, so the density is first neutralised by a Gaussian of the same
  charge Q = int rho at a centre c with width s:
    rho_g(x) = Q (s sqrt(pi))^-3 exp(-|x - c|^2 / s^2),
    V_g(x)   = Q erf(|x - c| / s) / |x - c|.
  The finite-element solve gets rho - rho_g, and V_g is added back at the
  points.  The electrostatic enrichment set is empty here.
* n-stage Anderson mixing of the density (Sec. V): with residuals
  F_k = rho_out,k - rho_in,k of the last m steps, the coefficients c
  minimise || sum_k c_k F_k ||_w subject to sum_k c_k = 1 (inner product
  sum_q w_q a_q b_q).  Then rho_in,next = sum_k c_k (rho_in,k + beta F_k).
* Energies (Sec. II): E_band = 2 sum f_i e_i, E_xc = int rho eps_xc, and the
  double-counting terms int rho V_xc and 1/2 int rho V_H.
"""
from __future__ import annotations

from math import erf, pi, sqrt

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


# ---------------------------------------------------------------- occupations
def fermi_dirac(eps, mu: float, kT: float) -> np.ndarray:
    """f(e, mu) of Eq. FermiDirac (written with exp of a non-positive argument)."""
    x = (np.asarray(eps, dtype=np.float64) - mu) / kT
    out = np.empty_like(x)
    pos = x > 0
    ex = np.exp(-x[pos])
    out[pos] = ex / (1.0 + ex)
    out[~pos] = 1.0 / (1.0 + np.exp(x[~pos]))
    return out


def fermi_level(eps, n_electrons: float, kT: float, iters: int = 200):
    """mu with 2 sum_i f(e_i, mu) = N_e (Eq. Mu) by bisection; returns (f, mu).
    The bracket runs from min e - 40 kT to max e + 40 kT; N_e must lie in
    (0, 2 len(e))."""
    eps = np.asarray(eps, dtype=np.float64)
    if not 0.0 < n_electrons < 2.0 * eps.size:
        raise ValueError("N_e out of range for the given states")
    lo, hi = eps.min() - 40.0 * kT, eps.max() + 40.0 * kT
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if 2.0 * fermi_dirac(eps, mid, kT).sum() < n_electrons:
            lo = mid
        else:
            hi = mid
        if hi - lo <= 4e-16 * max(1.0, abs(mid)):
            break
    mu = 0.5 * (lo + hi)
    return fermi_dirac(eps, mu, kT), mu


# ---------------------------------------------------------------- density
def density_at_points(Phi: np.ndarray, Y: np.ndarray, f: np.ndarray) -> np.ndarray:
    """rho_q = 2 sum_i f_i (sum_k Phi[q, k] Y[k, i])^2 for one cell: Phi
    [Q, K] the basis values at the cell's points, Y [K, N] the matching rows
    of the block of vectors (zero rows for Dirichlet nodes)."""
    psi = np.asarray(Phi, dtype=np.float64) @ np.asarray(Y, dtype=np.float64)
    return 2.0 * (psi * psi) @ np.asarray(f, dtype=np.float64)


# ---------------------------------------------------------------- LDA
# Perdew-Zunger (1981) fit of the Ceperley-Alder correlation energy,
# unpolarised: r_s >= 1: gamma / (1 + beta1 sqrt(r_s) + beta2 r_s);
# r_s < 1: A ln r_s + B + C r_s ln r_s + D r_s.
PZ_GAMMA, PZ_BETA1, PZ_BETA2 = -0.1423, 1.0529, 0.3334
PZ_A, PZ_B, PZ_C, PZ_D = 0.0311, -0.048, 0.0020, -0.0116


def lda_xc(rho) -> tuple[np.ndarray, np.ndarray]:
    """(eps_xc, V_xc) per point; zero where rho <= 1e-30 (no electrons)."""
    rho = np.asarray(rho, dtype=np.float64)
    eps = np.zeros_like(rho)
    vxc = np.zeros_like(rho)
    m = rho > 1e-30
    r = rho[m]
    # exchange: eps_x = -(3/4) (3/pi)^(1/3) rho^(1/3), V_x = (4/3) eps_x
    ex = -0.75 * (3.0 / pi) ** (1.0 / 3.0) * np.cbrt(r)
    vx = 4.0 / 3.0 * ex
    rs = np.cbrt(3.0 / (4.0 * pi * r))
    ec = np.empty_like(r)
    vc = np.empty_like(r)
    hi = rs >= 1.0
    s = np.sqrt(rs[hi])
    den = 1.0 + PZ_BETA1 * s + PZ_BETA2 * rs[hi]
    ec[hi] = PZ_GAMMA / den
    # V_c = eps_c - (r_s / 3) d eps_c / d r_s
    dec = -PZ_GAMMA * (0.5 * PZ_BETA1 / s + PZ_BETA2) / (den * den)
    vc[hi] = ec[hi] - rs[hi] / 3.0 * dec
    lo = ~hi
    lr = np.log(rs[lo])
    ec[lo] = PZ_A * lr + PZ_B + PZ_C * rs[lo] * lr + PZ_D * rs[lo]
    dec = PZ_A / rs[lo] + PZ_C * (lr + 1.0) + PZ_D
    vc[lo] = ec[lo] - rs[lo] / 3.0 * dec
    eps[m] = ex + ec
    vxc[m] = vx + vc
    return eps, vxc


# ---------------------------------------------------------------- Poisson
def gaussian_charge(x: np.ndarray, Q: float, c, s: float) -> tuple[np.ndarray, np.ndarray]:
    """(rho_g, V_g) of the neutralising Gaussian at points x [P, 3]."""
    d = np.sqrt(((np.asarray(x) - np.asarray(c)[None, :]) ** 2).sum(axis=1))
    rho = Q / (s * sqrt(pi)) ** 3 * np.exp(-(d / s) ** 2)
    v = np.empty_like(d)
    small = d < 1e-8 * s
    v[small] = Q * 2.0 / (sqrt(pi) * s)
    v[~small] = Q * np.array([erf(t) for t in d[~small] / s]) / d[~small]
    return rho, v


def laplace_matrix(cell_dof: np.ndarray, K: np.ndarray, n_h: int) -> sp.csr_matrix:
    """A^C_jk = (1/4 pi) int grad N_j . grad N_k over the mesh, from the kinetic
    block K = 1/2 int grad N_a . grad N_b (the same for every cell of the
    uniform mesh): each cell adds K / (2 pi) on its nodes; Dirichlet nodes
    (cell_dof < 0) are left out."""
    rows, cols, vals = [], [], []
    Kc = np.asarray(K, dtype=np.float64) / (2.0 * pi)
    npc = Kc.shape[0]
    ia, ib = np.meshgrid(np.arange(npc), np.arange(npc), indexing="ij")
    for dofs in np.asarray(cell_dof):
        da, db = dofs[ia], dofs[ib]
        m = (da >= 0) & (db >= 0)
        rows.append(da[m])
        cols.append(db[m])
        vals.append(Kc[m])
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n_h, n_h))
    return A.tocsr()


def poisson_solve(A: sp.csr_matrix, b: np.ndarray) -> np.ndarray:
    """The discrete Poisson problem A Phi = b by a sparse direct solve."""
    return spla.spsolve(A.tocsc(), b)


# ---------------------------------------------------------------- mixing
def anderson(rho_in_hist, rho_out_hist, w, beta: float) -> np.ndarray:
    """n-stage Anderson update from the last m input and output densities
    (lists, oldest first), weights w for the inner product."""
    F = [np.asarray(o) - np.asarray(i) for i, o in zip(rho_in_hist, rho_out_hist)]
    m = len(F)
    G = np.empty((m + 1, m + 1))
    for i in range(m):
        for j in range(m):
            G[i, j] = float(np.sum(w * F[i] * F[j]))
    G[m, :m] = 1.0
    G[:m, m] = 1.0
    G[m, m] = 0.0
    rhs = np.zeros(m + 1)
    rhs[m] = 1.0
    c = np.linalg.solve(G, rhs)[:m]
    return sum(c[k] * (np.asarray(rho_in_hist[k]) + beta * F[k]) for k in range(m))


# ---------------------------------------------------------------- energies
def band_energy(eps, f) -> float:
    """Eq. bandEnergy: 2 sum_i f_i e_i."""
    return float(2.0 * np.dot(np.asarray(f), np.asarray(eps)))
