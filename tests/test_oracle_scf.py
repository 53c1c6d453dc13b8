"""Pins of the oracle's self-consistent field pieces (oracle/scf.py).

* Fermi level: the electron count is met.  Two levels holding one pair of
  electrons put mu exactly at their midpoint (f_1 + f_2 = 1 forces
  symmetry).  A small kT gives aufbau filling.
* LDA: V_xc equals d(rho eps_xc)/d rho by central differences on both
  branches of the correlation fit.  Exchange has the closed form -0.458165/r_s.
* Density: for one basis function, rho = 2 f phi^2.  The weighted sum of the
  density of enrichment unit vectors reproduces the generator's M^ee
  diagonal (an independent quadrature of the same integrals).
* Poisson: the Laplace matrix is symmetric and annihilates a linear field
  on the rows whose cells miss the boundary.  A Gaussian charge distribution
  solved on a mesh, with a different neutralising Gaussian, gives the
  analytic potential Q erf(r/s)/r to the mesh's accuracy.
* Anderson: one stage is simple mixing.  On a linear fixed-point map in
  dimension n, n + 1 stages with affinely independent inputs give the fixed
  point exactly.
"""
from math import erf, pi, sqrt

import numpy as np
import pytest

from oracle.scf import (anderson, density_at_points, fermi_dirac, fermi_level, gaussian_charge,
                        laplace_matrix, lda_xc, poisson_solve)


def test_fermi_level_counts_electrons_and_symmetry():
    rng = np.random.default_rng(0)
    eps = np.sort(rng.uniform(-5.0, 1.0, 40))
    for ne, kT in ((10.0, 0.01), (31.0, 0.1), (7.5, 0.003)):
        f, mu = fermi_level(eps, ne, kT)
        assert 2.0 * f.sum() == pytest.approx(ne, rel=1e-12)
        assert np.all(np.diff(f) <= 0.0)
    f, mu = fermi_level(np.array([-1.3, 0.7]), 2.0, 0.2)
    assert mu == pytest.approx(-0.3, abs=1e-13)
    assert f[0] + f[1] == pytest.approx(1.0, abs=1e-13)
    eps = np.array([-3.0, -2.0, -1.0, 1.0, 2.0])
    f, mu = fermi_level(eps, 6.0, 1e-3)
    assert np.allclose(f, [1, 1, 1, 0, 0], atol=1e-12)
    assert fermi_dirac(np.array([mu]), mu, 0.5)[0] == 0.5


def test_lda_derivative_and_exchange():
    rho = np.logspace(-6, 3, 61)                  # r_s from ~62 down to ~0.06
    eps, v = lda_xc(rho)
    h = 1e-6 * rho
    ep, _ = lda_xc(rho + h)
    em, _ = lda_xc(rho - h)
    fd = ((rho + h) * ep - (rho - h) * em) / (2 * h)
    assert np.allclose(v, fd, rtol=1e-7, atol=1e-12)
    rs = np.cbrt(3.0 / (4.0 * pi * rho))
    ex = -0.75 * (3.0 / pi) ** (1.0 / 3.0) * np.cbrt(rho)
    assert np.allclose(ex * rs, -0.45816529328314287, rtol=1e-14)
    assert np.all(eps < 0) and np.all(v < 0)
    e0, v0 = lda_xc(np.array([0.0, -1.0]))
    assert np.array_equal(e0, [0.0, 0.0]) and np.array_equal(v0, [0.0, 0.0])


def test_density_single_function_and_mass_consistency(tiny_enriched):
    Phi = np.random.default_rng(1).standard_normal((30, 7))
    Y = np.zeros((7, 3))
    Y[2, 1] = 1.0
    f = np.array([0.9, 0.25, 0.1])
    assert np.allclose(density_at_points(Phi, Y, f), 2 * 0.25 * Phi[:, 2] ** 2, rtol=1e-15)
    # enrichment unit vectors: sum over cells and points of w rho = 2 f M^ee[al, al]
    from oracle.enriched import atom_functions, box_points, cell_basis
    from synth.basis import gll_rule
    prob = tiny_enriched
    mesh, qb, enr = prob.meta["mesh"], prob.meta["quad_boxes"], prob.meta["enr"]
    x, w = np.polynomial.legendre.leggauss(qb["ng"])
    gx, gw = 0.5 * (x + 1), 0.5 * w
    ep, idx = np.asarray(prob.enr_ptr), np.asarray(prob.enr_idx)
    bp = np.asarray(qb["box_ptr"])
    tot = np.zeros(prob.n_e)
    for e in range(mesh.n_cells):
        if ep[e + 1] == ep[e]:
            continue
        pts, wq, _ = box_points(qb["box_lo"][bp[e]:bp[e + 1]], qb["box_size"][bp[e]:bp[e + 1]],
                                gx, gw)
        N, _ = cell_basis(0.5 * (gll_rule(mesh.p)[0] + 1), mesh.cell_lo()[e], mesh.h, pts)
        E, _ = atom_functions(enr.centers[0], enr.shell_terms(), enr.r0, enr.t, pts)
        Phi = np.concatenate([N, E], axis=1)
        for al in idx[ep[e]:ep[e + 1]]:
            Y = np.zeros((Phi.shape[1], 1))
            Y[N.shape[1] + al, 0] = 1.0
            tot[al] += wq @ density_at_points(Phi, Y, np.array([0.5]))
    assert np.allclose(tot, np.diag(prob.M_ee), rtol=1e-12)


def test_laplace_matrix_symmetry_and_linear_fields(hydrogen_small):
    from synth.assemble import reference_kinetic
    prob = hydrogen_small
    mesh = prob.meta["mesh"]
    K = reference_kinetic(mesh.p, mesh.h)
    A = laplace_matrix(prob.cell_dof, K, prob.n_h)
    assert abs(A - A.T).max() < 1e-14 * abs(A).max()
    # node coordinates of every classical DOF
    from synth.basis import gll_rule
    xi = 0.5 * (gll_rule(mesh.p)[0] + 1)
    k = mesh.p + 1
    nz, ny, nx = np.meshgrid(xi, xi, xi, indexing="ij")
    loc = np.stack([nx.ravel(), ny.ravel(), nz.ravel()], axis=1)
    X = np.zeros((prob.n_h, 3))
    inner = np.ones(prob.n_h, dtype=bool)
    for e, dofs in enumerate(np.asarray(prob.cell_dof)):
        pts = mesh.cell_lo()[e] + mesh.h * loc
        m = dofs >= 0
        X[dofs[m]] = pts[m]
        if np.any(~m):
            inner[dofs[m]] = False
    u = 2.0 * X[:, 0] - 0.5 * X[:, 1] + X[:, 2]
    r = A @ u
    assert inner.sum() > 0
    assert np.abs(r[inner]).max() < 1e-12 * abs(A).max() * np.abs(u).max()
    assert k ** 3 == prob.cell_dof.shape[1]


def poisson_gaussian_error(nc, length, Q, c, s1, s2):
    """max |V_H - Q erf(r/s1)/r| over the Gauss points of nc^3 degree-4
    cells, V_H from the oracle's Poisson solve of the Gaussian rho(s1) with
    the neutralising Gaussian rho(s2) at the same centre (their difference
    is spherical with no net charge: its potential vanishes outside both,
    so the zero Dirichlet values hold); also max |Q erf(r/s1)/r|."""
    from synth.assemble import reference_kinetic, shape_at
    from synth.mesh import build_mesh
    from synth.quad import unit_cube_rule
    mesh = build_mesh(4, nc, -0.5 * length, length)
    A = laplace_matrix(mesh.cell_dof, reference_kinetic(mesh.p, mesh.h), mesh.n_h)
    ref, wref = unit_cube_rule(6)
    B, _ = shape_at(mesh.p, 2.0, -np.ones(3), 2.0 * ref - 1.0, need_grad=False)
    lo_all = mesh.cell_lo()
    b = np.zeros(mesh.n_h)
    for e in range(mesh.n_cells):
        pts = lo_all[e] + mesh.h * ref
        r1, _ = gaussian_charge(pts, Q, c, s1)
        r2, _ = gaussian_charge(pts, Q, c, s2)
        d = mesh.cell_dof[e]
        m = d >= 0
        np.add.at(b, d[m], (B.T @ (wref * mesh.h ** 3 * (r1 - r2)))[m])
    phi = poisson_solve(A, b)
    err = vmax = 0.0
    for e in range(mesh.n_cells):
        pts = lo_all[e] + mesh.h * ref
        ph = np.zeros(B.shape[1])
        d = mesh.cell_dof[e]
        ph[d >= 0] = phi[d[d >= 0]]
        _, vg = gaussian_charge(pts, Q, c, s2)
        _, v1 = gaussian_charge(pts, Q, c, s1)
        err = max(err, np.abs(B @ ph + vg - v1).max())
        vmax = max(vmax, np.abs(v1).max())
    return err, vmax


@pytest.mark.slow
def test_poisson_gaussian_against_erf_potential():
    """A Gaussian charge (Q = 2, width 2) off the box centre, with the
    neutralising Gaussian of width 2.5: V_H at the Gauss points matches
    Q erf(r/s)/r to 4e-3 of its maximum on 6^3 degree-4 cells of a 24-Bohr
    box, and the error falls by more than half on 8^3 cells (the mesh's
    discretisation error; a wrong scale such as a lost 4 pi would leave
    an O(1) error on both)."""
    c = np.array([0.4, -0.3, 0.2])
    e6, vmax = poisson_gaussian_error(6, 24.0, 2.0, c, 2.0, 2.5)
    e8, _ = poisson_gaussian_error(8, 24.0, 2.0, c, 2.0, 2.5)
    assert e6 < 4e-3 * vmax
    assert e8 < 0.5 * e6


def test_anderson_simple_mixing_and_linear_fixed_point():
    rng = np.random.default_rng(2)
    w = rng.uniform(0.5, 2.0, 6)
    ri, ro = rng.standard_normal(6), rng.standard_normal(6)
    assert np.allclose(anderson([ri], [ro], w, 0.3), ri + 0.3 * (ro - ri), rtol=1e-15)
    n = 3
    M = rng.standard_normal((n, n)) * 0.4
    c = rng.standard_normal(n)
    xs = [rng.standard_normal(n) for _ in range(n + 1)]
    gs = [M @ x + c for x in xs]
    x_star = np.linalg.solve(np.eye(n) - M, c)
    out = anderson(xs, gs, np.ones(n), 0.7)
    assert np.allclose(out, x_star, rtol=1e-10, atol=1e-12)
    # the weighted inner product enters: same fixed point with other weights
    out2 = anderson(xs, gs, np.array([3.0, 0.2, 1.0]), 0.7)
    assert np.allclose(out2, x_star, rtol=1e-10, atol=1e-12)
    assert erf(0.0) == 0.0 and sqrt(4.0) == 2.0
