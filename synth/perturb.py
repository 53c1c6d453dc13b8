"""Seeded smooth potential perturbations for self-consistent-step sequences.

A step's perturbation is dV(x) = sum_g A_g exp(-|x - c_g|^2 / (2 sigma^2)) with
8 Gaussians, sigma = 6 Bohr, amplitudes U[-0.05, 0.05] Ha and centres uniform
in the box.  It enters the classical cell matrices only, lumped at the GLL
nodes: H^cc_e[a][a] += w_a dV(x_a), with w_a the node's GLL weight in the
cell (the same quadrature as the lumped mass matrix), and only in cells that
share no DOF with a cell carrying enrichment functions.  The coupling blocks,
H^ee and the mass matrices are left unchanged, so one context can follow the
sequence through chebfilter_update_H_cc.

Why only there: a lumped diagonal term is not the projection of dV onto the
enriched basis.  Inside the enriched region M^E has near-null directions
(classical and enrichment functions that nearly cancel); a diagonal term on
their classical part does not cancel with them and gives H~ spurious
eigenvalues of order |dV| / lambda_min(M^E) (on a 4-atom cluster a 10-step
Lanczos run then reported a lower bound of -266 Ha against a lowest Ritz
value of -55 Ha, and the filtered blocks lost rank).  Away from the
enrichment supports the basis is purely classical and the lumped term is the
consistent GLL-quadrature potential term.
"""
from __future__ import annotations

import numpy as np

from .basis import gll_rule


def smooth_field(rng: np.random.Generator, lo: float, length: float, n_gauss: int = 8,
                 sigma: float = 6.0, amp: float = 0.05):
    centres = lo + length * rng.uniform(size=(n_gauss, 3))
    amps = rng.uniform(-amp, amp, size=n_gauss)

    def dV(x: np.ndarray) -> np.ndarray:
        d2 = ((x[:, None, :] - centres[None, :, :]) ** 2).sum(axis=2)
        return (amps[None, :] * np.exp(-0.5 * d2 / sigma ** 2)).sum(axis=1)
    return dV


def far_cells(prob) -> np.ndarray:
    """Mask of the cells that share no DOF with a cell carrying enrichment functions."""
    cd = np.asarray(prob.cell_dof)
    ep = np.asarray(prob.enr_ptr)
    inside = np.zeros(prob.n_h, dtype=bool)
    d = cd[np.nonzero(ep[1:] > ep[:-1])[0]].ravel()
    inside[d[d >= 0]] = True
    return np.array([not inside[r[r >= 0]].any() for r in cd])


def perturbed_H_cc(prob, dV) -> np.ndarray:
    """prob.H_cc with the GLL-lumped perturbation dV added to the diagonals of
    the far cells (see the module notes)."""
    mesh = prob.meta["mesh"]
    _, w = gll_rule(mesh.p)
    we = (0.5 * mesh.h) ** 3 * np.einsum("i,j,k->kji", w, w, w).ravel()   # x fastest
    H = np.array(prob.H_cc, dtype=np.float64, copy=True)
    cd = np.asarray(prob.cell_dof)
    vals = dV(mesh.node_xyz)                     # at the free DOFs
    ok = (cd >= 0) & far_cells(prob)[:, None]
    e_idx, a_idx = np.nonzero(ok)
    H[e_idx, a_idx, a_idx] += we[a_idx] * vals[cd[e_idx, a_idx]]
    return H


def sequence(prob, steps: int, seed: int = 0):
    """Per-step H_cc arrays of a perturbation sequence (a fresh field each step)."""
    mesh = prob.meta["mesh"]
    rng = np.random.default_rng(seed)
    for _ in range(steps):
        yield perturbed_H_cc(prob, smooth_field(rng, mesh.lo, mesh.length))


# ---------------------------------------------------------------------------
# The same field recipe evaluated on the device at the plain cells' Gauss
# points, for sequences whose operator is rebuilt on the device each step
# (the consistent quadrature term of the perturbation instead of a lumped
# diagonal; cells sharing a DOF with an enriched cell keep the unperturbed
# potential, for the reason given in the module notes).
# ---------------------------------------------------------------------------
def field_draw(rng: np.random.Generator, lo: float, length: float, n_gauss: int = 8,
               sigma: float = 6.0, amp: float = 0.05):
    """One step's field parameters, drawn in the order smooth_field draws them."""
    centres = lo + length * rng.uniform(size=(n_gauss, 3))
    amps = rng.uniform(-amp, amp, size=n_gauss)
    return centres, amps, sigma


def field_at(pts, centres, amps, sigma):
    """dV at device points pts [Q, 3] (float64 CUDA tensor) for drawn parameters."""
    import torch
    out = torch.zeros(pts.shape[0], dtype=pts.dtype, device=pts.device)
    for c, a in zip(np.asarray(centres, dtype=np.float64), np.asarray(amps, dtype=np.float64)):
        d2 = ((pts - torch.as_tensor(c, dtype=pts.dtype, device=pts.device)) ** 2).sum(dim=1)
        out += float(a) * torch.exp(d2 * (-0.5 / sigma ** 2))
    return out


def plain_cell_sets(prob):
    """(plain cells, far plain cells): cells without enrichment functions, and
    those of them that share no DOF with a cell carrying enrichment functions."""
    ep = np.asarray(prob.enr_ptr)
    plain = np.nonzero(ep[1:] == ep[:-1])[0].astype(np.int32)
    far = far_cells(prob)
    return plain, plain[far[plain]]
