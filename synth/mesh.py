"""Uniform hexahedral mesh of degree-p spectral elements on a cube (Sec. III).

Global nodes form a (p*nc+1)^3 lattice, x fastest.  Nodes on the cube faces
carry the homogeneous Dirichlet condition and are removed; the remaining
"free" classical DOFs are numbered in the same x-fastest order.  Each cell
lists its (p+1)^3 local nodes (x fastest) as free-DOF indices, -1 marking a
Dirichlet node.  Cells are numbered x fastest as well.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .basis import gll_rule


@dataclass
class Mesh:
    p: int
    nc: int               # cells per axis
    lo: float             # cube is [lo, lo + length]^3
    length: float
    cell_dof: np.ndarray  # int64 [E, (p+1)^3], -1 = Dirichlet
    n_h: int              # number of free classical DOFs
    node_xyz: np.ndarray  # float64 [n_h, 3] coordinates of free DOFs

    @property
    def h(self) -> float:
        return self.length / self.nc

    @property
    def n_cells(self) -> int:
        return self.nc ** 3

    @property
    def npc(self) -> int:
        return (self.p + 1) ** 3

    def cell_lo(self) -> np.ndarray:
        """Lower corner of every cell, [E, 3]."""
        i = np.arange(self.nc)
        cz, cy, cx = np.meshgrid(i, i, i, indexing="ij")
        ijk = np.stack([cx.ravel(), cy.ravel(), cz.ravel()], axis=1)
        return self.lo + ijk * self.h

    def cell_ijk(self) -> np.ndarray:
        i = np.arange(self.nc)
        cz, cy, cx = np.meshgrid(i, i, i, indexing="ij")
        return np.stack([cx.ravel(), cy.ravel(), cz.ravel()], axis=1)


def build_mesh(p: int, nc: int, lo: float, length: float) -> Mesh:
    npd = p * nc + 1                      # global nodes per axis
    g = np.arange(npd)
    interior = (g > 0) & (g < npd - 1)
    # free-DOF index of each global lattice node (x fastest), -1 on the boundary
    free_1d = np.where(interior, np.cumsum(interior) - 1, -1)
    nfree_1d = int(interior.sum())
    fx = free_1d[None, None, :]
    fy = free_1d[None, :, None]
    fz = free_1d[:, None, None]
    free = np.where((fx >= 0) & (fy >= 0) & (fz >= 0),
                    fx + nfree_1d * (fy + nfree_1d * fz), -1)   # [z, y, x]

    # local node offsets (x fastest)
    a = np.arange(p + 1)
    az, ay, ax = np.meshgrid(a, a, a, indexing="ij")
    ax, ay, az = ax.ravel(), ay.ravel(), az.ravel()
    c = np.arange(nc)
    cz, cy, cx = np.meshgrid(c, c, c, indexing="ij")
    cx, cy, cz = cx.ravel(), cy.ravel(), cz.ravel()
    gx = cx[:, None] * p + ax[None, :]
    gy = cy[:, None] * p + ay[None, :]
    gz = cz[:, None] * p + az[None, :]
    cell_dof = free[gz, gy, gx].astype(np.int64)

    # coordinates of free DOFs
    xi, _ = gll_rule(p)
    h = length / nc
    coord_1d = np.empty(npd)
    for ci in range(nc):
        coord_1d[ci * p:(ci + 1) * p + 1] = lo + ci * h + (xi + 1.0) * 0.5 * h
    ci_free = coord_1d[interior]
    zz, yy, xx = np.meshgrid(ci_free, ci_free, ci_free, indexing="ij")
    node_xyz = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1)
    return Mesh(p=p, nc=nc, lo=lo, length=length, cell_dof=cell_dof,
                n_h=nfree_1d ** 3, node_xyz=node_xyz)
