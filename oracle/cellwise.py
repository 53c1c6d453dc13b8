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
step), applied to batches of cells; P_e drops the Dirichlet nodes, which is
done here by zeroing their rows and columns in a copy of the cell blocks
(their gathered values are then multiplied by zero and their sums are
zero).  Nothing here is shared with the GPU library.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import torch

_BATCH = 1024          # cells per batched classical product
_EBATCH = 128          # enriched cells per batched coupling product


def _t(a, dtype=torch.float64):
    if isinstance(a, torch.Tensor):
        return a.to(dtype)
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
        live = torch.as_tensor(cd >= 0, dtype=torch.float64)          # [E, npc]
        self.idx = torch.as_tensor(np.where(cd >= 0, cd, 0), dtype=torch.int64)
        self.Hcc = _t(prob.H_cc).reshape(self.E, self.npc, self.npc).clone()
        self.Hcc *= live[:, :, None]
        self.Hcc *= live[:, None, :]
        self.D = _t(prob.M_cc_diag)
        self.Dinv = 1.0 / self.D
        self._S = None
        if self.n_e == 0:
            return
        # enriched cells in batches of similar function counts, blocks padded
        # with zero rows whose enrichment index is the spare row n_e
        ep = np.asarray(prob.enr_ptr, dtype=np.int64)
        ei = np.asarray(prob.enr_idx, dtype=np.int64)
        cnt = ep[1:] - ep[:-1]
        ecells = np.nonzero(cnt > 0)[0]
        ecells = ecells[np.argsort(-cnt[ecells], kind="stable")]
        Hec = np.asarray(prob.H_ec).reshape(-1, self.npc)
        Mec = np.asarray(prob.M_ec).reshape(-1, self.npc)
        livec = cd >= 0
        self.ebatches = []
        for b0 in range(0, len(ecells), _EBATCH):
            cells = ecells[b0:b0 + _EBATCH]
            na = int(cnt[cells].max())
            bh = np.zeros((len(cells), na, self.npc))
            bm = np.zeros((len(cells), na, self.npc))
            al = np.full((len(cells), na), self.n_e, dtype=np.int64)
            for q, e in enumerate(cells):
                r0, r1 = ep[e], ep[e + 1]
                bh[q, :r1 - r0] = Hec[r0:r1] * livec[e][None, :]
                bm[q, :r1 - r0] = Mec[r0:r1] * livec[e][None, :]
                al[q, :r1 - r0] = ei[r0:r1]
            self.ebatches.append((self.idx[torch.as_tensor(cells)], torch.as_tensor(al),
                                  torch.as_tensor(bh), torch.as_tensor(bm)))
        self.Hee = _t(prob.H_ee).reshape(self.n_e, self.n_e)
        self.Mee = _t(prob.M_ee).reshape(self.n_e, self.n_e)

    # ---------------------------------------------------------------- pieces
    def cell_products(self, Xc: torch.Tensor, out: torch.Tensor) -> None:
        """out += sum_e P_e^T H^cc_e P_e X_c (out: n_h rows)."""
        N = Xc.shape[1]
        for e0 in range(0, self.E, _BATCH):
            ix = self.idx[e0:e0 + _BATCH]
            contrib = torch.bmm(self.Hcc[e0:e0 + _BATCH], Xc[ix])        # [b, npc, N]
            out.index_add_(0, ix.reshape(-1), contrib.reshape(-1, N))

    def coupling(self, which: int, Xc: torch.Tensor) -> torch.Tensor:
        """Assembled enriched-classical block times X_c (which: 2 = H^ec,
        3 = M^ec): row alpha sums B_e[alpha] . X_c[P_e] over the cells e
        whose support meets alpha."""
        N = Xc.shape[1]
        out = torch.zeros((self.n_e + 1, N), dtype=torch.float64)
        for bt in self.ebatches:
            ix, al, blk = bt[0], bt[1], bt[which]
            out.index_add_(0, al.reshape(-1), torch.bmm(blk, Xc[ix]).reshape(-1, N))
        return out[:self.n_e]

    def coupling_T(self, which: int, Xe: torch.Tensor, out: torch.Tensor) -> None:
        """out += transpose of `coupling` applied to X_e: sum_e P_e^T B_e^T X_e[alpha(e)]."""
        N = Xe.shape[1]
        Xp = torch.cat([Xe, torch.zeros((1, N), dtype=torch.float64)], dim=0)
        for bt in self.ebatches:
            ix, al, blk = bt[0], bt[1], bt[which]
            contrib = torch.bmm(blk.transpose(1, 2), Xp[al])              # [b, npc, N]
            out.index_add_(0, ix.reshape(-1), contrib.reshape(-1, N))

    # -------------------------------------------------------------- products
    def apply_H(self, X) -> torch.Tensor:
        X = _t(X)
        Y = torch.zeros((self.n, X.shape[1]), dtype=torch.float64)
        Xc, Xe = X[:self.n_h], X[self.n_h:]
        self.cell_products(Xc, Y[:self.n_h])
        if self.n_e:
            self.coupling_T(2, Xe, Y[:self.n_h])
            Y[self.n_h:] = self.coupling(2, Xc) + self.Hee @ Xe
        return Y

    def apply_M(self, X) -> torch.Tensor:
        X = _t(X)
        Y = torch.empty((self.n, X.shape[1]), dtype=torch.float64)
        Xc, Xe = X[:self.n_h], X[self.n_h:]
        torch.mul(self.D[:, None], Xc, out=Y[:self.n_h])
        if self.n_e:
            self.coupling_T(3, Xe, Y[:self.n_h])
            Y[self.n_h:] = self.coupling(3, Xc) + self.Mee @ Xe
        return Y

    def schur(self) -> np.ndarray:
        """S = M^ee - M^ec D^-1 M^ec^T (Sec. IV.D), column by column of M^ec^T."""
        if self._S is None:
            S = self.Mee.clone()
            I = torch.eye(self.n_e, dtype=torch.float64)
            for a0 in range(0, self.n_e, 256):
                cols = torch.zeros((self.n_h, I[:, a0:a0 + 256].shape[1]), dtype=torch.float64)
                self.coupling_T(3, I[:, a0:a0 + 256], cols)                 # M^ec^T e_alpha
                S[:, a0:a0 + 256] -= self.coupling(3, self.Dinv[:, None] * cols)
            S = 0.5 * (S + S.T)
            self._S = (S.numpy(), sla.cho_factor(S.numpy(), lower=True))
        return self._S[0]

    def block_inverse(self, R) -> torch.Tensor:
        """[[D^-1 + L^T S^-1 L, -L^T S^-1], [-S^-1 L, S^-1]] R with L = M^ec D^-1.

        Second block row: y_e = S^-1 r_e - S^-1 L r_c.  First block row:
        D^-1 r_c + L^T S^-1 L r_c - L^T S^-1 r_e = D^-1 r_c - L^T y_e (the
        common left factor L^T taken out: one transposed coupling product)."""
        R = _t(R)
        Y = torch.empty_like(R)
        rc, re = R[:self.n_h], R[self.n_h:]
        if self.n_e == 0:
            torch.mul(self.Dinv[:, None], rc, out=Y)
            return Y
        self.schur()
        cho = self._S[1]
        Sinv = lambda B: torch.from_numpy(sla.cho_solve(cho, B.numpy()))   # noqa: E731
        L_rc = self.coupling(3, self.Dinv[:, None] * rc)                    # M^ec D^-1 r_c
        ye = Sinv(re) - Sinv(L_rc)
        Y[self.n_h:] = ye
        t = torch.zeros_like(rc)
        self.coupling_T(3, ye, t)                                          # M^ec^T y_e
        torch.mul(self.Dinv[:, None], rc - t, out=Y[:self.n_h])           # D^-1 r_c - L^T y_e
        return Y

    def apply_Htilde(self, X) -> torch.Tensor:
        return self.block_inverse(self.apply_H(X))
