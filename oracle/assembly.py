"""Element block of a cell outside every enrichment support (oracle; test
infrastructure only).

Eq. HBlocks with the cell's plain Gauss rule (Sec. III.B): the classical
block is H_cc_e[a, b] = 1/2 int grad N_a . grad N_b + int V N_a N_b.  The
first term K is a polynomial integral shared by every cell of the uniform
mesh (an input here); the second is the quadrature sum over the cell's
points x_q with weights w_q (Jacobian included):
sum_q w_q V(x_q) N_a(x_q) N_b(x_q).  Written out point by point.
"""
from __future__ import annotations

import numpy as np


def plain_cell_block(K: np.ndarray, B: np.ndarray, w: np.ndarray, V: np.ndarray) -> np.ndarray:
    """K + sum_q w_q V_q B[q]^T B[q] for one cell: B [nq, npc] shape values at
    the points, w [nq] weights, V [nq] the potential at the points."""
    K = np.asarray(K, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    H = K.copy()
    for q in range(B.shape[0]):
        H += (w[q] * V[q]) * np.outer(B[q], B[q])
    return H
