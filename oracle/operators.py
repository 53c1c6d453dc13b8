"""Global enriched-FE operators from element blocks (oracle; test infrastructure).

Plain definitions (Eq. H2x2, M2x2, HBlocks, MBlocks): the global matrices are
the sums of the elemental contributions; DOF order is all free classical DOFs
first, then the enrichment DOFs.  M^cc is the GLL-lumped diagonal (Sec. III.B).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def _classical_coo(cell_dof: np.ndarray, blocks: np.ndarray):
    """(rows, cols, vals) of sum_e P_e^T B_e P_e over pairs of free local nodes."""
    E, npc = cell_dof.shape
    rows = np.repeat(cell_dof, npc, axis=1).ravel()
    cols = np.tile(cell_dof, (1, npc)).ravel()
    vals = blocks.reshape(E, npc * npc).ravel()
    keep = (rows >= 0) & (cols >= 0)
    return rows[keep], cols[keep], vals[keep]


def _coupling_coo(prob, blocks: np.ndarray):
    """(alpha, j, val) of the enriched-classical block sum_e over cell rows."""
    E, npc = prob.cell_dof.shape
    cell_of = np.repeat(np.arange(E), np.diff(prob.enr_ptr))        # cell of each (e, alpha) row
    j = prob.cell_dof[cell_of]                                      # [nnz, npc]
    a = np.repeat(prob.enr_idx[:, None], npc, axis=1)
    keep = j >= 0
    return a[keep], j[keep], blocks[keep]


def assemble_global(prob, which: str) -> sp.csr_matrix:
    """Global H^E ("H") or M^E ("M") as a sparse matrix of order n_h + n_e."""
    n_h, n_e = prob.n_h, prob.n_e
    n = n_h + n_e
    if which == "H":
        r, c, v = _classical_coo(prob.cell_dof, prob.H_cc)
        a, j, w = _coupling_coo(prob, prob.H_ec)
        ee = prob.H_ee
    elif which == "M":
        r = np.arange(n_h)
        c = np.arange(n_h)
        v = prob.M_cc_diag
        a, j, w = _coupling_coo(prob, prob.M_ec)
        ee = prob.M_ee
    else:
        raise ValueError(which)
    ea, eb = np.meshgrid(np.arange(n_e), np.arange(n_e), indexing="ij")
    rows = np.concatenate([r, n_h + a, j, n_h + ea.ravel()])
    cols = np.concatenate([c, j, n_h + a, n_h + eb.ravel()])
    vals = np.concatenate([v, w, w, ee.ravel()])
    return sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()


class Operators:
    """H^E, M^E of one problem with the two ways of applying (M^E)^-1."""

    def __init__(self, prob, which=("H", "M"), M=None):
        """which: the global matrices to assemble (("M",) skips H^E, whose
        element entries are the bulk of the memory on large problems); M: an
        already assembled global M^E."""
        self.prob = prob
        self.n_h, self.n_e = prob.n_h, prob.n_e
        self.n = self.n_h + self.n_e
        self.H = assemble_global(prob, "H") if "H" in which else None
        self.M = M if M is not None else assemble_global(prob, "M")
        self._lu = None
        self._blk = None

    # -- plain products
    def apply_H(self, X: np.ndarray) -> np.ndarray:
        return np.asarray(self.H @ X)

    def apply_M(self, X: np.ndarray) -> np.ndarray:
        return np.asarray(self.M @ X)

    # -- (M^E)^-1 by a sparse direct solve (definition)
    def solve_M(self, R: np.ndarray) -> np.ndarray:
        if self._lu is None:
            self._lu = spla.splu(self.M.tocsc())
        return self._lu.solve(np.asarray(R, dtype=np.float64))

    # -- (M^E)^-1 by the block-wise (Banachiewicz) inverse of Sec. IV.D
    def _block_setup(self):
        n_h = self.n_h
        Mcc = self.M[:n_h, :n_h].diagonal()
        Mec = self.M[n_h:, :n_h].tocsr()                    # n_e x n_h
        Minv_cc = sp.diags(1.0 / Mcc)
        L = (Mec @ Minv_cc).tocsr()                         # L = M^ec (M^cc)^-1
        S = self.M[n_h:, n_h:].toarray() - (L @ Mec.T).toarray()   # Schur complement
        S = 0.5 * (S + S.T)
        self._blk = (Minv_cc, L, sla.cho_factor(S, lower=True), S)

    def schur(self) -> np.ndarray:
        if self._blk is None:
            self._block_setup()
        return self._blk[3]

    def block_inverse(self, R: np.ndarray) -> np.ndarray:
        """[[Mcc^-1 + L^T S^-1 L, -L^T S^-1], [-S^-1 L, S^-1]] applied to R."""
        if self._blk is None:
            self._block_setup()
        Minv_cc, L, cho, _ = self._blk
        R = np.asarray(R, dtype=np.float64)
        vec = R.ndim == 1
        if vec:
            R = R[:, None]
        rc, re = R[:self.n_h], R[self.n_h:]
        Sinv = lambda B: sla.cho_solve(cho, B)              # noqa: E731
        SinvL_rc = Sinv(L @ rc)
        Sinv_re = Sinv(re)
        yc = Minv_cc @ rc + L.T @ SinvL_rc - L.T @ Sinv_re
        ye = -SinvL_rc + Sinv_re
        Y = np.vstack([yc, ye])
        return Y[:, 0] if vec else Y

    # -- H~ = (M^E)^-1 H^E
    def apply_Htilde(self, X: np.ndarray, how: str = "block") -> np.ndarray:
        HX = self.apply_H(X)
        return self.block_inverse(HX) if how == "block" else self.solve_M(HX)

    def dense(self) -> tuple[np.ndarray, np.ndarray]:
        return self.H.toarray(), self.M.toarray()


def sampled_rows(prob, rows: np.ndarray, X: np.ndarray, which: str, H_cc=None) -> np.ndarray:
    """Rows `rows` of H^E X (which="H") or M^E X (which="M") summed straight
    from the element blocks (Eq. H2x2 / M2x2, HBlocks / MBlocks), without the
    global matrices: for a classical DOF i, the cells' rows of H^cc_e (or the
    lumped D_i) at i's local positions, plus H^ec_e^T (M^ec_e^T) X_e of the
    enriched cells that contain i; for an enrichment DOF alpha, every cell
    row of H^ec (M^ec) that belongs to alpha, plus row alpha of H^ee (M^ee).
    H_cc overrides the problem's classical blocks for the cells it lists
    ({cell: block}); used where the global operator is too large to form."""
    cd = np.asarray(prob.cell_dof)
    ep, ei = np.asarray(prob.enr_ptr), np.asarray(prob.enr_idx)
    n_h = cd.max() + 1 if prob.n_e == 0 else prob.n_h
    Xe = X[n_h:]
    cpl = np.asarray(prob.H_ec if which == "H" else prob.M_ec)
    ee = np.asarray(prob.H_ee if which == "H" else prob.M_ee)
    out = np.zeros((len(rows), X.shape[1]))
    for k, i in enumerate(rows):
        if i < n_h:
            if which == "M":
                out[k] = prob.M_cc_diag[i] * X[i]
            for e, a in zip(*np.nonzero(cd == i)):
                d = cd[e]
                ok = d >= 0
                if which == "H":
                    blk = H_cc[e] if (H_cc is not None and e in H_cc) else prob.H_cc[e]
                    out[k] += blk[a, ok] @ X[d[ok]]
                r0, r1 = ep[e], ep[e + 1]
                if r1 > r0:
                    out[k] += cpl[r0:r1, a] @ Xe[ei[r0:r1]]
        else:
            al = i - n_h
            for r in np.nonzero(ei == al)[0]:
                e = np.searchsorted(ep, r, side="right") - 1
                d = cd[e]
                ok = d >= 0
                out[k] += cpl[r, ok] @ X[d[ok]]
            out[k] += ee[al] @ Xe
    return out
