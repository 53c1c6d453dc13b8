"""Pins of the oracle's enriched element blocks (oracle/enriched.py) against
what the mathematics fixes.

* The 1D Lagrange basis: the interpolation property, reproduction of x^p
  and of its derivative, and the partition of unity.
* The smooth cutoff (Eq. Moll1): 1 below r0, 0 beyond r0 + r0/t, exactly 1/2
  at the middle of the transition (r~ = 1/2), and the derivative against
  central differences.
* The enrichment functions: gradients against central differences.  On the
  y axis only the first p component is nonzero (the (y, z, x) order).  The
  addition theorem fixes the sum over m of a p shell's squares.  The
  radials are normalised (1D library quadrature).
* The blocks on an adaptive grid around one atom.  A hydrogen 1s function
  with a far cutoff gives the closed forms: norm 1, kinetic energy 1/2,
  potential energy -1 for V = -1/r.  A 1s and a 2p function with a near
  cutoff are checked against 1D radial integrals of the same cutoff radial
  (scipy.integrate.quad): the norms, the integrals of N_al times the
  constant and the linear global fields (coefficients 1 and the nodes'
  x-coordinates), and the kinetic cross terms against those fields, which
  vanish for a compactly supported function.
* H^cc on the union of boxes equals the plain-rule block when V is a
  polynomial that both rules integrate exactly.
"""
from math import pi, sqrt

import numpy as np
import pytest
from scipy.integrate import quad

from oracle.assembly import plain_cell_block
from oracle.enriched import (Y00, Y1, atom_functions, box_points, cell_basis,
                             enriched_cell_blocks, lagrange_1d, radial_terms, smooth_cutoff)

GLL5 = np.array([0.0, 0.5 - sqrt(21.0) / 14.0, 0.5, 0.5 + sqrt(21.0) / 14.0, 1.0])


def gauss01(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def test_lagrange_interpolates_and_reproduces_polynomials():
    L, dL = lagrange_1d(GLL5, GLL5)
    assert np.allclose(L, np.eye(5), atol=1e-14)
    x = np.linspace(-0.3, 1.2, 37)
    L, dL = lagrange_1d(GLL5, x)
    assert np.allclose(L.sum(axis=1), 1.0, atol=1e-13)
    assert np.allclose(dL.sum(axis=1), 0.0, atol=1e-11)
    for k in range(5):
        assert np.allclose(L @ GLL5 ** k, x ** k, atol=1e-12)
        assert np.allclose(dL @ GLL5 ** k, k * x ** max(k - 1, 0) if k else 0.0, atol=1e-10)


def test_cell_basis_reproduces_trilinear_field_and_gradient():
    lo, h = np.array([1.0, -2.0, 0.5]), 3.0
    rng = np.random.default_rng(0)
    pts = lo + h * rng.random((50, 3))
    N, G = cell_basis(GLL5, lo, h, pts)
    k = len(GLL5)
    nz, ny, nx = np.meshgrid(GLL5, GLL5, GLL5, indexing="ij")
    X = lo[0] + h * nx.ravel()
    Y = lo[1] + h * ny.ravel()
    Z = lo[2] + h * nz.ravel()
    f = X * Y ** 2 - 3 * Z * X + Y ** 4                     # degree <= 4 per axis
    fx = pts[:, 0] * pts[:, 1] ** 2 - 3 * pts[:, 2] * pts[:, 0] + pts[:, 1] ** 4
    assert np.allclose(N @ f, fx, rtol=1e-12, atol=1e-10)
    gx = pts[:, 1] ** 2 - 3 * pts[:, 2]
    gy = 2 * pts[:, 0] * pts[:, 1] + 4 * pts[:, 1] ** 3
    gz = -3 * pts[:, 0]
    assert np.allclose(G[0] @ f, gx, atol=1e-9)
    assert np.allclose(G[1] @ f, gy, atol=1e-9)
    assert np.allclose(G[2] @ f, gz, atol=1e-9)
    assert N.shape == (50, k ** 3)


@pytest.mark.parametrize("r0,t", [(3.0, 1.0), (2.0, 0.5)])
def test_smooth_cutoff_closed_values(r0, t):
    r = np.array([0.0, 0.5 * r0, r0 * 0.999, r0 + r0 / t * 1.001, 5 * r0])
    hv, _ = smooth_cutoff(r, r0, t)
    assert np.array_equal(hv, [1.0, 1.0, 1.0, 0.0, 0.0])
    hm, _ = smooth_cutoff(np.array([r0 + 0.5 * r0 / t]), r0, t)
    assert hm[0] == pytest.approx(0.5, abs=1e-15)
    rr = np.linspace(r0 * 1.01, r0 + r0 / t * 0.99, 41)
    _, dh = smooth_cutoff(rr, r0, t)
    eps = 1e-6
    fd = (smooth_cutoff(rr + eps, r0, t)[0] - smooth_cutoff(rr - eps, r0, t)[0]) / (2 * eps)
    assert np.allclose(dh, fd, rtol=1e-6, atol=1e-8)
    assert np.all(dh <= 0.0)


SI_LIKE = [(0, [(2.0, 0, 1.0)]),                                   # hydrogen-type 1s
           (0, [(1.0 / sqrt(2.0), 0, 0.5), (-0.5 / sqrt(2.0), 1, 0.5)]),   # 2s-type
           (1, [(sqrt(2.0 ** 5 / 24.0), 1, 1.0)])]                 # 2p Slater, zeta 1


def test_radials_are_normalised():
    for _, terms in SI_LIKE:
        v = quad(lambda r: radial_terms(terms, np.array([r]))[0][0] ** 2 * r * r, 0, 80,
                 limit=200)[0]
        assert v == pytest.approx(1.0, abs=1e-10)


def test_enrichment_gradients_and_harmonics():
    c = np.array([0.3, -0.2, 0.1])
    rng = np.random.default_rng(1)
    pts = c + rng.uniform(-4.0, 4.0, size=(60, 3))
    val, grad = atom_functions(c, SI_LIKE, 3.0, 1.0, pts)
    eps = 1e-6
    for d in range(3):
        e = np.zeros(3)
        e[d] = eps
        vp, _ = atom_functions(c, SI_LIKE, 3.0, 1.0, pts + e)
        vm, _ = atom_functions(c, SI_LIKE, 3.0, 1.0, pts - e)
        assert np.allclose(grad[:, :, d], (vp - vm) / (2 * eps), rtol=1e-6, atol=1e-9)
    # the p shell's components in the order (y, z, x)
    on_y = c + np.array([[0.0, 1.3, 0.0]])
    v, _ = atom_functions(c, SI_LIKE, 3.0, 1.0, on_y)
    assert v[0, 2] != 0.0 and v[0, 3] == 0.0 and v[0, 4] == 0.0
    on_x = c + np.array([[1.3, 0.0, 0.0]])
    v, _ = atom_functions(c, SI_LIKE, 3.0, 1.0, on_x)
    assert v[0, 4] != 0.0 and v[0, 2] == 0.0 and v[0, 3] == 0.0
    # addition theorem: sum_m (Y_1m q r)^2 = 3/(4 pi) (h R)^2
    r = np.sqrt(((pts - c) ** 2).sum(axis=1))
    hc, _ = smooth_cutoff(r, 3.0, 1.0)
    R, _ = radial_terms(SI_LIKE[2][1], r)
    assert np.allclose((val[:, 2:5] ** 2).sum(axis=1), 3.0 / (4 * pi) * (hc * R) ** 2,
                       rtol=1e-12, atol=1e-300)
    R0, _ = radial_terms(SI_LIKE[0][1], r)
    assert np.allclose(val[:, 0], Y00 * hc * R0, rtol=1e-14)


def adaptive_grid(center, shells, r0, t, h, nc, V, tau, depth):
    """The generator's adaptive rule (Sec. IV.C) on nc^3 cells of side h
    around `center` (at the middle vertex), trial functions sum N^2,
    sum |grad N|^2 and |V| sum N^2.  Returns per cell (lo, box_lo, box_size)."""
    from synth.quad import adaptive_rule

    def trial(x):
        v, g = atom_functions(center, shells, r0, t, x)
        s = (v * v).sum(axis=1)
        return np.stack([s, (g * g).sum(axis=(1, 2)), np.abs(V(x)) * s], axis=1)

    out = []
    base = center - 0.5 * nc * h
    for k in range(nc):
        for j in range(nc):
            for i in range(nc):
                lo = base + h * np.array([i, j, k], dtype=np.float64)
                _, _, _, blo, bsz = adaptive_rule(lo, h, trial, tau, ng=6, max_depth=depth,
                                                  boxes=True)
                out.append((lo, blo, bsz))
    return out


def sum_blocks(grid, center, shells, r0, t, h, V):
    gx, gw = gauss01(6)
    K = np.zeros((125, 125))
    tot = None
    for lo, blo, bsz in grid:
        pts, w, _ = box_points(blo, bsz, gx, gw)
        b = enriched_cell_blocks(K, GLL5, lo, h, pts, w, V(pts), [0], center[None], shells, r0, t)
        nz, ny, nx = np.meshgrid(GLL5, GLL5, GLL5, indexing="ij")
        xnode = lo[0] + h * nx.ravel()
        one = np.ones(125)
        part = {"Mee": b[4], "Hee": b[3],
                "M1": b[2] @ one, "Mx": b[2] @ xnode,
                "K1": b[1] @ one, "Kx": b[1] @ xnode}
        tot = part if tot is None else {k: tot[k] + part[k] for k in tot}
    return tot


def test_hydrogen_1s_closed_forms():
    """1s = 2 e^{-r} Y00 with the cutoff at r0 = 10 (tail beyond 10 below
    3e-7 of the norm): M = 1, kinetic 1/2, potential -1 (V = -1/r)."""
    c = np.zeros(3)
    shells = [(0, [(2.0, 0, 1.0)])]
    r0, t = 10.0, 1.0
    V = lambda x: -1.0 / np.sqrt((x * x).sum(axis=1))          # noqa: E731
    zero = lambda x: np.zeros(x.shape[0])                        # noqa: E731
    grid = adaptive_grid(c, shells, r0, t, 20.0, 2, V, np.array([1e-10, 1e-10, 1e-9]), 16)
    s_v = sum_blocks(grid, c, shells, r0, t, 20.0, V)
    s_0 = sum_blocks(grid, c, shells, r0, t, 20.0, zero)
    # the cutoff's own effect, from 1D integrals of the same radial
    g = lambda r: smooth_cutoff(np.array([r]), r0, t)[0][0] * 2.0 * np.exp(-r)   # noqa: E731
    norm = quad(lambda r: g(r) ** 2 * r * r, 0, 2 * r0, points=[r0], limit=200)[0]
    assert norm == pytest.approx(1.0, abs=1e-6)
    assert s_0["Mee"][0, 0] == pytest.approx(norm, abs=1e-9)
    assert s_0["Hee"][0, 0] == pytest.approx(0.5, abs=1e-6)
    assert s_v["Hee"][0, 0] - s_0["Hee"][0, 0] == pytest.approx(-1.0, abs=1e-5)


def test_cross_terms_against_radial_integrals():
    """A 1s and a 2p (y, z, x) function with the cutoff at r0 = 2, t = 1
    (support radius 4) on 2^3 cells of side 4 around the atom.  The p_x row
    against the linear field x gives Y1 (4 pi / 3) int q r^4 dr (q = h R / r).
    The s row against the constant field gives sqrt(4 pi) int h R r^2 dr.
    The kinetic rows against both fields give 1/2 int d/dx N_al = 0."""
    c = np.array([0.0, 0.0, 0.0])
    shells = [(0, [(2.0, 0, 1.0)]), (1, [(sqrt(2.0 ** 5 / 24.0), 1, 1.0)])]
    r0, t = 2.0, 1.0
    zero = lambda x: np.zeros(x.shape[0])                        # noqa: E731
    grid = adaptive_grid(c, shells, r0, t, 4.0, 2, zero, np.array([1e-13, 1e-12, 1.0]), 16)
    s = sum_blocks(grid, c, shells, r0, t, 4.0, zero)
    hcut = lambda r: smooth_cutoff(np.array([r]), r0, t)[0][0]                          # noqa: E731
    R_s = lambda r: radial_terms(shells[0][1], np.array([r]))[0][0]                     # noqa: E731
    q_p = lambda r: radial_terms(shells[1][1], np.array([r]), shift=1)[0][0]            # noqa: E731
    int_s = sqrt(4 * pi) * quad(lambda r: hcut(r) * R_s(r) * r * r, 0, 2 * r0, points=[r0])[0]
    int_px = Y1 * 4 * pi / 3 * quad(lambda r: hcut(r) * q_p(r) * r ** 4, 0, 2 * r0, points=[r0])[0]
    assert s["M1"][0] == pytest.approx(int_s, rel=1e-9)
    assert s["Mx"][3] == pytest.approx(int_px, rel=1e-9)        # index 3 = p_x
    assert abs(s["Mx"][1]) < 1e-10 and abs(s["Mx"][2]) < 1e-10   # p_y, p_z against x
    assert np.all(np.abs(s["K1"]) < 1e-9)
    # p_x against x: the kink of x^2 q'(r) / r at the nucleus limits the
    # grid's accuracy to ~1e-9 here (6e-8 with ten times looser tolerances)
    assert np.all(np.abs(s["Kx"]) < 5e-9)
    # norms of the cut functions, and the s-p overlap vanishing by parity
    ns = quad(lambda r: (hcut(r) * R_s(r)) ** 2 * r * r, 0, 2 * r0, points=[r0])[0]
    npn = quad(lambda r: (hcut(r) * q_p(r) * r) ** 2 * r * r, 0, 2 * r0, points=[r0])[0]
    assert s["Mee"][0, 0] == pytest.approx(ns, rel=1e-9)
    assert np.allclose(np.diag(s["Mee"])[1:], npn, rtol=1e-9)
    assert np.all(np.abs(s["Mee"][0, 1:]) < 1e-11)


def test_box_union_matches_plain_rule_for_polynomial_potential():
    """On a union of sub-boxes the tensor Gauss rule of each box is exact for
    the degree-11 integrands of a cubic V times two basis functions, like the
    plain rule on the whole cell: the two H^cc agree."""
    gx, gw = gauss01(6)
    lo, h = np.array([-1.0, 2.0, 0.0]), 2.5
    blo = np.array([lo, lo + [h / 2, 0, 0], lo + [0, h / 2, 0], lo + [h / 2, h / 2, 0],
                    lo + [0, 0, h / 2], lo + [h / 2, 0, h / 2], lo + [0, h / 2, h / 2]])
    bsz = np.full(7, h / 2)
    # the last octant split once more
    oct_lo = lo + [h / 2, h / 2, h / 2]
    sub = np.array([[i, j, k] for k in (0, 1) for j in (0, 1) for i in (0, 1)]) * (h / 4)
    blo = np.concatenate([blo, oct_lo + sub])
    bsz = np.concatenate([bsz, np.full(8, h / 4)])
    pts, w, _ = box_points(blo, bsz, gx, gw)
    assert w.sum() == pytest.approx(h ** 3, rel=1e-14)
    V = lambda x: 1.0 + x[:, 0] * x[:, 1] - 0.5 * x[:, 2] ** 3     # noqa: E731
    K = np.random.default_rng(2).standard_normal((125, 125))
    Hb = enriched_cell_blocks(K, GLL5, lo, h, pts, w, V(pts), [], None, None, 1.0, 1.0)[0]
    ppts, pw, _ = box_points(lo[None], np.array([h]), gx, gw)
    B, _ = cell_basis(GLL5, lo, h, ppts)
    Hp = plain_cell_block(K, B, pw, V(ppts))
    assert np.allclose(Hb, Hp, rtol=1e-11, atol=1e-11)
