"""Container for one discrete enriched-FE problem (the element blocks).

Field names and layouts follow the library's `cf_problem` input:

* cell_dof  int64 [E, npc]        free classical DOF of each local node, -1 = Dirichlet
* H_cc      float64 [E, npc, npc] elemental classical Hamiltonian blocks (Eq. Hcc)
* M_cc_diag float64 [n_h]         assembled GLL-lumped classical overlap (Sec. III.B)
* enr_ptr   int64 [E + 1]         CSR over cells of the enrichment functions meeting the cell
* enr_idx   int64 [nnz]           enrichment index alpha in [0, n_e)
* H_ec, M_ec float64 [nnz, npc]   per-cell enriched-classical blocks, row alpha (Eq. Hec, Mec)
* H_ee, M_ee float64 [n_e, n_e]   assembled enriched-enriched blocks (Eq. Hee, Mee)
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Problem:
    p: int
    cell_dof: np.ndarray
    H_cc: np.ndarray
    M_cc_diag: np.ndarray
    enr_ptr: np.ndarray
    enr_idx: np.ndarray
    H_ec: np.ndarray
    M_ec: np.ndarray
    H_ee: np.ndarray
    M_ee: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def npc(self) -> int:
        return (self.p + 1) ** 3

    @property
    def n_cells(self) -> int:
        return int(self.cell_dof.shape[0])

    @property
    def n_h(self) -> int:
        return int(self.M_cc_diag.shape[0])

    @property
    def n_e(self) -> int:
        return int(self.H_ee.shape[0])

    @property
    def n(self) -> int:
        return self.n_h + self.n_e

    def enriched_cells(self) -> np.ndarray:
        return np.nonzero(np.diff(self.enr_ptr) > 0)[0]

    def save(self, path: str) -> None:
        np.savez(path, p=self.p, cell_dof=self.cell_dof, H_cc=self.H_cc,
                 M_cc_diag=self.M_cc_diag, enr_ptr=self.enr_ptr, enr_idx=self.enr_idx,
                 H_ec=self.H_ec, M_ec=self.M_ec, H_ee=self.H_ee, M_ee=self.M_ee)

    @staticmethod
    def load(path: str) -> "Problem":
        z = np.load(path, allow_pickle=False)
        return Problem(p=int(z["p"]), cell_dof=z["cell_dof"], H_cc=z["H_cc"],
                       M_cc_diag=z["M_cc_diag"], enr_ptr=z["enr_ptr"], enr_idx=z["enr_idx"],
                       H_ec=z["H_ec"], M_ec=z["M_ec"], H_ee=z["H_ee"], M_ee=z["M_ee"])
