"""Per-cell quadrature rules (Sec. III.B, IV.C).

* Cells met by no enrichment support use a tensor n_g^3 Gauss rule.
* Cells inside some enrichment support use the divide-and-conquer rule of
  Sec. IV.C: a box is tested against its eight children with the same n_g^3
  Gauss rule; if every trial function's integral agrees within the tolerance
  the parent's points are kept, otherwise each child is treated as a parent.
  Boxes of one cell are processed level by level.  The tolerance of each
  trial function is one fixed number for the whole mesh.
"""
from __future__ import annotations

import numpy as np

from .basis import gauss_rule

CHILD_OFFSETS = np.array([[i, j, k] for k in (0, 1) for j in (0, 1) for i in (0, 1)],
                         dtype=np.float64)


def unit_cube_rule(ng: int) -> tuple[np.ndarray, np.ndarray]:
    """ng^3 Gauss points on [0,1]^3 (x fastest) with weights summing to 1."""
    x, w = gauss_rule(ng)
    x = 0.5 * (x + 1.0)
    w = 0.5 * w
    zz, yy, xx = np.meshgrid(x, x, x, indexing="ij")
    wz, wy, wx = np.meshgrid(w, w, w, indexing="ij")
    pts = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1)
    return pts, (wx * wy * wz).ravel()


def adaptive_rule(lo: np.ndarray, size: float, trial, tau: np.ndarray, ng: int = 6,
                  max_depth: int = 10, boxes: bool = False):
    """Adaptive points/weights for the box [lo, lo+size]^3.

    `trial(points[Q,3]) -> values[Q, nt]` evaluates the trial functions and
    `tau[nt]` is the fixed tolerance of each one (Sec. IV.C): a box is
    accepted when |I_parent - sum I_children| < tau for every trial function,
    or at depth `max_depth`.  Returns (points [Q,3], weights [Q], leaf count)
    and, with boxes=True, also the accepted boxes (lower corners [L,3], sides
    [L]) in the order of their points (each box's ng^3 points consecutive,
    x fastest).
    """
    ref, wref = unit_cube_rule(ng)
    nq = ref.shape[0]
    tau = np.asarray(tau, dtype=np.float64)
    f_lo = np.asarray(lo, dtype=np.float64)[None, :]
    f_sz = np.array([float(size)])
    out_p, out_w, out_lo, out_sz = [], [], [], []
    leaves = 0
    depth = 0
    while f_lo.shape[0]:
        B = f_lo.shape[0]
        par = f_lo[:, None, :] + f_sz[:, None, None] * ref[None]             # [B,nq,3]
        half = 0.5 * f_sz
        clo = f_lo[:, None, :] + half[:, None, None] * CHILD_OFFSETS[None]   # [B,8,3]
        chi = clo[:, :, None, :] + half[:, None, None, None] * ref[None, None]  # [B,8,nq,3]
        fp = trial(par.reshape(-1, 3)).reshape(B, nq, -1)
        fc = trial(chi.reshape(-1, 3)).reshape(B, 8, nq, -1)
        Ip = np.einsum("q,bqt->bt", wref, fp) * (f_sz ** 3)[:, None]
        Ic = np.einsum("q,bcqt->bt", wref, fc) * (half ** 3)[:, None]
        ok = np.all(np.abs(Ip - Ic) < tau[None, :], axis=1)
        if depth >= max_depth:
            ok[:] = True
        if ok.any():
            out_p.append(par[ok].reshape(-1, 3))
            out_w.append((np.outer(f_sz[ok] ** 3, wref)).ravel())
            out_lo.append(f_lo[ok])
            out_sz.append(f_sz[ok])
            leaves += int(ok.sum())
        bad = ~ok
        f_lo = clo[bad].reshape(-1, 3)
        f_sz = np.repeat(half[bad], 8)
        depth += 1
    if boxes:
        return (np.concatenate(out_p), np.concatenate(out_w), leaves, np.concatenate(out_lo),
                np.concatenate(out_sz))
    return np.concatenate(out_p), np.concatenate(out_w), leaves
