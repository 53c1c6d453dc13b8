"""Pins of oracle/assembly.py (the plain-cell element block, Eq. HBlocks with
the cell's Gauss rule) against closed forms computed another way.

With V constant or linear in one coordinate, the potential term of the block
is a product of one-dimensional polynomial integrals of the Lagrange basis on
the GLL nodes (x fastest in the local numbering), which numpy's exact
polynomial arithmetic gives without any quadrature.  A dropped weight, a wrong
Jacobian, a transposed table or a wrong axis order fails one of them.
"""
import numpy as np
import pytest
from numpy.polynomial import Polynomial

from oracle.assembly import plain_cell_block
from synth.assemble import plain_points, plain_tables
from synth.basis import gll_rule


def lagrange_polys(nodes):
    out = []
    for i, xi in enumerate(nodes):
        P = Polynomial([1.0])
        for m, xm in enumerate(nodes):
            if m != i:
                P = P * Polynomial([-xm, 1.0]) / (xi - xm)
        out.append(P)
    return out


def moment_matrix(p, h, power):
    """M[i, j] = int_0^h x^power l_i(x) l_j(x) dx, exactly: on the reference
    interval t in [-1, 1] (x = h (t + 1) / 2, well-conditioned monomials)."""
    xi, _ = gll_rule(p)
    L = lagrange_polys(xi)
    xp = (0.5 * h * Polynomial([1.0, 1.0])) ** power
    M = np.empty((p + 1, p + 1))
    for i in range(p + 1):
        for j in range(p + 1):
            F = (xp * L[i] * L[j]).integ()
            M[i, j] = 0.5 * h * (F(1.0) - F(-1.0))
    return M


def kron3(mx, my, mz):
    """Operator on x-fastest local indices: mx on x, my on y, mz on z."""
    return np.kron(mz, np.kron(my, mx))


@pytest.fixture(scope="module")
def tables(hydrogen_small):
    B, w, K, ref = plain_tables(hydrogen_small)
    return hydrogen_small, B, w, K, ref


def test_constant_potential_gives_mass_matrix(tables):
    prob, B, w, K, ref = tables
    mesh = prob.meta["mesh"]
    M1 = moment_matrix(mesh.p, mesh.h, 0)
    H = plain_cell_block(K, B, w, np.full(len(w), 2.5))
    ref_M = kron3(M1, M1, M1)
    assert np.abs(H - K - 2.5 * ref_M).max() < 1e-13 * np.abs(ref_M).max()


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_linear_potential_gives_moment_matrix(tables, axis):
    prob, B, w, K, ref = tables
    mesh = prob.meta["mesh"]
    M0, M1 = moment_matrix(mesh.p, mesh.h, 0), moment_matrix(mesh.p, mesh.h, 1)
    V = mesh.h * ref[:, axis]                 # the coordinate measured from the cell's corner
    H = plain_cell_block(K, B, w, V)
    facs = [M0, M0, M0]
    facs[axis] = M1
    want = kron3(*facs)
    assert np.abs(H - K - want).max() < 1e-13 * np.abs(want).max()


def test_kinetic_block_and_generator_cells(tables):
    """K annihilates constants (partition of unity); on cells without
    enrichment the generator's blocks are this quadrature sum."""
    prob, B, w, K, ref = tables
    assert np.abs(K @ np.ones(K.shape[0])).max() < 1e-12 * np.abs(K).max()
    ep = np.asarray(prob.enr_ptr)
    plain = np.nonzero(ep[1:] == ep[:-1])[0][:5]
    V = prob.meta["potential"](plain_points(prob, plain).reshape(-1, 3)).reshape(len(plain), -1)
    for k, e in enumerate(plain):
        H = plain_cell_block(K, B, w, V[k])
        H = 0.5 * (H + H.T)
        assert np.abs(H - prob.H_cc[e]).max() < 1e-12 * np.abs(H).max()
