"""H^E X, M^E X and (M^E)^-1 X summed straight from the element blocks
(oracle; test infrastructure only).

The same definitions as `operators.py`, evaluated without the global
matrices, so that problems with ~10^6 DOFs and hundreds of vectors fit the
host and use all of its cores:

* H^E X (Eq. H2x2 with HBlocks): Y_c = sum_e P_e^T H^cc_e P_e X_c
  + sum_e P_e^T H^ec_e^T X_e[alpha(e)], Y_e = sum_e scatter_alpha(e)(H^ec_e P_e X_c)
  + H^ee X_e -- the elemental products of Sec. V and their assembly, cell by
  cell, each cell's contribution added to its rows (an indexed sum).
* M^E X (Eq. M2x2): the same with the GLL-lumped diagonal D for M^cc.
* (M^E)^-1 r by the block-wise inverse of Sec. IV.D, written as the 2x2
  block matrix [[D^-1 + L^T S^-1 L, -L^T S^-1], [-S^-1 L, S^-1]] with
  L = M^ec D^-1 and S = M^ee - M^ec D^-1 M^ec^T (dense Cholesky of S).

Every product is a torch CPU matmul in FP64 (the library primitive is the
step); no reordering beyond the grouping of cells into batches.  Nothing
here is shared with the GPU library.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import torch

_BATCH = 1024          # cells per batched product (bounds the gathered rows)


def _t(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype)


class CellOperators:
    """Element-block products of one problem (FP64, host, all threads)."""

    def __init__(self, prob, threads: int | None = None):
        if threads:
            torch.set_num_threads(int(threads))
        self.prob = prob
        self.n_h, self.n_e = prob.n_h, prob.n_e
        self.n = self.n_h + self.n_e
        cd = np.asarray(prob.cell_dof, dtype=np.int64)
        self.E, self.npc = cd.shape
        # Dirichlet nodes (-1) read and write a spare zero row n_h
        self.idx = _t(np.where(cd >= 0, cd, self.n_h), torch.int64)
        self.Hcc = _t(prob.H_cc).reshape(self.E, self.npc, self.npc)
        self.D = _t(prob.M_cc_diag)
        self.Dinv = 1.0 / self.D
        ep = np.asarray(prob.enr_ptr, dtype=np.int64)
        self.ecells = np.nonzero(ep[1:] > ep[:-1])[0]
        self.ep = ep
        self.ei = _t(prob.enr_idx, torch.int64)
        self.Hec = _t(prob.H_ec).reshape(-1, self.npc)
        self.Mec = _t(prob.M_ec).reshape(-1, self.npc)
        self.Hee = _t(prob.H_ee).reshape(self.n_e, self.n_e)
        self.Mee = _t(prob.M_ee).reshape(self.n_e, self.n_e)
        self._S = None

    # ---------------------------------------------------------------- pieces
    def _padded(self, Xc: torch.Tensor) -> torch.Tensor:
        return torch.cat([Xc, torch.zeros((1, Xc.shape[1]), dtype=Xc.dtype)], dim=0)

    def cell_products(self, Xc: torch.Tensor) -> torch.Tensor:
        """sum_e P_e^T H^cc_e P_e X_c (rows n_h)."""
        Xp = self._padded(Xc)
        Yp = torch.zeros_like(Xp)
        for e0 in range(0, self.E, _BATCH):
            ix = self.idx[e0:e0 + _BATCH]
            contrib = torch.bmm(self.Hcc[e0:e0 + _BATCH], Xp[ix])      # [b, npc, N]
            Yp.index_add_(0, ix.reshape(-1), contrib.reshape(-1, Xp.shape[1]))
        return Yp[:self.n_h]

    def coupling(self, blocks: torch.Tensor, Xc: torch.Tensor) -> torch.Tensor:
        """Assembled enriched-classical block times X_c: row alpha sums
        B_e[alpha] . X_c[P_e] over the cells e whose support meets alpha."""
        Xp = self._padded(Xc)
        out = torch.zeros((self.n_e, Xc.shape[1]), dtype=Xc.dtype)
        for e in self.ecells:
            r0, r1 = self.ep[e], self.ep[e + 1]
            out.index_add_(0, self.ei[r0:r1], blocks[r0:r1] @ Xp[self.idx[e]])
        return out

    def coupling_T(self, blocks: torch.Tensor, Xe: torch.Tensor) -> torch.Tensor:
        """Transpose of `coupling`: sum_e P_e^T B_e^T X_e[alpha(e)] (rows n_h)."""
        Yp = torch.zeros((self.n_h + 1, Xe.shape[1]), dtype=Xe.dtype)
        for e in self.ecells:
            r0, r1 = self.ep[e], self.ep[e + 1]
            Yp.index_add_(0, self.idx[e], blocks[r0:r1].T @ Xe[self.ei[r0:r1]])
        return Yp[:self.n_h]

    # -------------------------------------------------------------- products
    def apply_H(self, X) -> torch.Tensor:
        X = _t(X)
        Xc, Xe = X[:self.n_h], X[self.n_h:]
        Yc = self.cell_products(Xc)
        if self.n_e == 0:
            return Yc
        Yc = Yc + self.coupling_T(self.Hec, Xe)
        Ye = self.coupling(self.Hec, Xc) + self.Hee @ Xe
        return torch.cat([Yc, Ye], dim=0)

    def apply_M(self, X) -> torch.Tensor:
        X = _t(X)
        Xc, Xe = X[:self.n_h], X[self.n_h:]
        Yc = self.D[:, None] * Xc
        if self.n_e == 0:
            return Yc
        Yc = Yc + self.coupling_T(self.Mec, Xe)
        Ye = self.coupling(self.Mec, Xc) + self.Mee @ Xe
        return torch.cat([Yc, Ye], dim=0)

    def schur(self) -> np.ndarray:
        """S = M^ee - M^ec D^-1 M^ec^T (Sec. IV.D), column by column of M^ec^T."""
        if self._S is None:
            S = self.Mee.clone()
            I = torch.eye(self.n_e, dtype=torch.float64)
            for a0 in range(0, self.n_e, 256):
                cols = self.coupling_T(self.Mec, I[:, a0:a0 + 256])      # M^ec^T e_alpha
                S[:, a0:a0 + 256] -= self.coupling(self.Mec, self.Dinv[:, None] * cols)
            S = 0.5 * (S + S.T)
            self._S = (S.numpy(), sla.cho_factor(S.numpy(), lower=True))
        return self._S[0]

    def block_inverse(self, R) -> torch.Tensor:
        """[[D^-1 + L^T S^-1 L, -L^T S^-1], [-S^-1 L, S^-1]] R with L = M^ec D^-1.

        Second block row: y_e = S^-1 r_e - S^-1 L r_c.  First block row:
        D^-1 r_c + L^T S^-1 L r_c - L^T S^-1 r_e = D^-1 r_c - L^T y_e (the
        common left factor L^T taken out: one transposed coupling product)."""
        R = _t(R)
        if self.n_e == 0:
            return self.Dinv[:, None] * R
        self.schur()
        cho = self._S[1]
        Sinv = lambda B: torch.from_numpy(sla.cho_solve(cho, B.numpy()))   # noqa: E731
        L = lambda Xc: self.coupling(self.Mec, self.Dinv[:, None] * Xc)      # noqa: E731
        LT = lambda Ze: self.Dinv[:, None] * self.coupling_T(self.Mec, Ze)   # noqa: E731
        rc, re = R[:self.n_h], R[self.n_h:]
        ye = Sinv(re) - Sinv(L(rc))
        yc = self.Dinv[:, None] * rc - LT(ye)
        return torch.cat([yc, ye], dim=0)

    def apply_Htilde(self, X) -> torch.Tensor:
        return self.block_inverse(self.apply_H(X))
