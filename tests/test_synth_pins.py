"""Pins of the synthetic-problem generator (basis, quadrature, enrichment, element blocks).

Each check compares against a closed form, a textbook property or an
independent 1D integral, never against the generator's own formula.
"""
import os
from math import factorial, pi, sqrt

import numpy as np
import pytest
from scipy import integrate

from synth import configs
from synth.assemble import reference_kinetic, shape_at
from synth.basis import gauss_rule, gll_rule, lagrange_eval
from synth.enrich import EnrichmentSet, Radial, cutoff
from synth.mesh import build_mesh
from synth.quad import adaptive_rule

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_gll_p4_closed_form():
    ref = np.loadtxt(os.path.join(GOLD, "gll_p4.txt"))
    x, w = gll_rule(4)
    assert np.allclose(x, ref[:, 0], atol=1e-15, rtol=0)
    assert np.allclose(w, ref[:, 1], atol=1e-15, rtol=0)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
def test_gll_exactness_degree(p):
    """n = p+1 GLL points integrate x^k exactly for k <= 2n-3 and not for k = 2n-2 (Sec. III.B)."""
    x, w = gll_rule(p)
    n = p + 1
    for k in range(0, 2 * n - 2):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(w @ x ** k - exact) < 1e-13
    k = 2 * n - 2
    assert abs(w @ x ** k - 2.0 / (k + 1)) > 1e-6


@pytest.mark.parametrize("n", [2, 4, 6])
def test_gauss_exactness(n):
    x, w = gauss_rule(n)
    for k in range(0, 2 * n):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(w @ x ** k - exact) < 1e-13


def test_lagrange_partition_and_cardinal():
    xi, _ = gll_rule(4)
    pts = np.linspace(-1, 1, 37)
    L, dL = lagrange_eval(xi, pts)
    assert np.allclose(L.sum(axis=1), 1.0, atol=1e-13)
    assert np.allclose(dL.sum(axis=1), 0.0, atol=1e-11)
    Ln, _ = lagrange_eval(xi, xi)
    assert np.allclose(Ln, np.eye(5), atol=1e-14)
    # derivative against a centred finite difference
    e = 1e-6
    Lp, _ = lagrange_eval(xi, pts + e)
    Lm, _ = lagrange_eval(xi, pts - e)
    assert np.allclose((Lp - Lm) / (2 * e), dL, atol=1e-7)


def test_element_kinetic_nullspace_and_symmetry():
    K = reference_kinetic(4, 2.5)
    assert np.allclose(K, K.T, atol=1e-14)
    assert np.abs(K @ np.ones(125)).max() < 1e-12
    ev = np.linalg.eigvalsh(K)
    assert ev[0] > -1e-12 and np.sum(ev < 1e-10) == 1
    # 1/2 int |grad f|^2 for f = x on [0,h]^3 is h^3/2: nodal values of x are exact
    h = 2.5
    xi, _ = gll_rule(4)
    xs = np.tile((xi + 1) * 0.5 * h, 25)
    assert abs(xs @ K @ xs - 0.5 * h ** 3) < 1e-12


def test_lumped_mass_total_volume():
    mesh = build_mesh(4, 3, -1.5, 3.0)
    _, w = gll_rule(4)
    we = (0.5 * mesh.h) ** 3 * np.einsum("i,j,k->kji", w, w, w).ravel()
    assert abs(we.sum() * mesh.n_cells - 27.0) < 1e-12
    prob = configs.box(nc=3, length=3.0, p=4)
    assert prob.M_cc_diag.min() > 0 and prob.M_cc_diag.sum() < 27.0


def test_shape_functions_gradient_fd():
    lo = np.array([0.3, -1.0, 2.0])
    h = 1.7
    pts = lo + h * np.random.default_rng(1).random((5, 3))
    N, G = shape_at(4, h, lo, pts, need_grad=True)
    assert np.allclose(N.sum(axis=1), 1.0, atol=1e-13)
    e = 1e-6
    for d in range(3):
        dp = np.zeros(3)
        dp[d] = e
        Np, _ = shape_at(4, h, lo, pts + dp, need_grad=False)
        Nm, _ = shape_at(4, h, lo, pts - dp, need_grad=False)
        assert np.allclose((Np - Nm) / (2 * e), G[d], atol=1e-6)


@pytest.mark.parametrize("rad", [Radial("h1s"), Radial("h2s"), Radial("slater", 1, 2.7),
                                 Radial("slater", 2, 1.3), Radial("slater", 3, 0.8, 1)])
def test_radial_normalised(rad):
    val, _ = integrate.quad(lambda r: rad.eval(np.array([r]))[0][0] ** 2 * r * r, 0, 80,
                            limit=400)
    assert abs(val - 1.0) < 1e-10


def test_slater_normalisation_constant():
    z, n = 1.9, 3
    r = np.array([0.7])
    R, _ = Radial("slater", n, z).eval(r)
    assert abs(R[0] - sqrt((2 * z) ** (2 * n + 1) / factorial(2 * n)) * 0.7 ** 2 * np.exp(-z * 0.7)) < 1e-14


def test_cutoff_properties():
    r0, t = 3.0, 1.0
    r = np.linspace(0, 8, 801)
    h, dh = cutoff(r, r0, t)
    assert np.all(h[r < r0] == 1.0)
    assert np.all(h[r > r0 + r0 / t] == 0.0)
    assert np.all(np.diff(h) <= 1e-15)
    mid = (r > r0 + 0.01) & (r < 2 * r0 - 0.01)
    e = 1e-6
    hp, _ = cutoff(r[mid] + e, r0, t)
    hm, _ = cutoff(r[mid] - e, r0, t)
    assert np.allclose((hp - hm) / (2 * e), dh[mid], atol=1e-6)


def _enr():
    shells = [Radial("slater", 1, 1.1), Radial("slater", 2, 0.9, 1), Radial("slater", 3, 0.7)]
    return EnrichmentSet(centers=np.array([[0.1, -0.2, 0.3]]), shells=shells, r_c=6.0)


def test_enrichment_gradients_fd_and_addition_theorem():
    enr = _enr()
    pts = np.random.default_rng(2).uniform(-3, 3, (40, 3))
    v, g = enr.eval_atom(0, pts)
    e = 1e-6
    for d in range(3):
        dp = np.zeros(3)
        dp[d] = e
        vp, _ = enr.eval_atom(0, pts + dp, need_grad=False)
        vm, _ = enr.eval_atom(0, pts - dp, need_grad=False)
        assert np.allclose((vp - vm) / (2 * e), g[:, :, d], atol=1e-7)
    f3, f4 = enr.trial_sums(0, pts)
    assert np.allclose(f3, (v ** 2).sum(axis=1), rtol=1e-12)
    assert np.allclose(f4, (g ** 2).sum(axis=(1, 2)), rtol=1e-10)


def test_real_harmonics_orthonormal():
    """Angular parts of one shell are orthonormal on the unit sphere."""
    enr = EnrichmentSet(centers=np.zeros((1, 3)), shells=[Radial("slater", 2, 1.0, 0),
                                                          Radial("slater", 2, 1.0, 1)], r_c=50.0)
    xg, wg = gauss_rule(24)
    th = np.arccos(xg)
    ph = (np.arange(48) + 0.5) * 2 * pi / 48
    T, P = np.meshgrid(th, ph, indexing="ij")
    W = np.repeat(wg, 48) * (2 * pi / 48)
    pts = np.stack([np.sin(T) * np.cos(P), np.sin(T) * np.sin(P), np.cos(T)], axis=-1).reshape(-1, 3)
    v, _ = enr.eval_atom(0, pts, need_grad=False)
    R, _ = Radial("slater", 2, 1.0).eval(np.array([1.0]))
    Y = v / R[0]
    assert np.allclose((Y * W[:, None]).T @ Y, np.eye(4), atol=1e-12)


def test_adaptive_quadrature_closed_form():
    """sum over cells of the adaptive rule of exp(-2r) on a cube of side 20 -> pi."""
    mesh = build_mesh(4, 4, -10.0, 20.0)
    f = lambda x: np.exp(-2.0 * np.sqrt((x ** 2).sum(axis=1)))[:, None]   # noqa: E731
    total = 0.0
    for lo in mesh.cell_lo():
        p, w, _ = adaptive_rule(lo, mesh.h, f, np.array([1e-12]))
        total += w @ f(p)[:, 0]
    # tail outside the cube is below 4 pi int_10^inf r^2 e^{-2r} dr ~ 1e-6
    tail = 4 * pi * integrate.quad(lambda r: r * r * np.exp(-2 * r), 10, np.inf)[0]
    assert abs(total - (pi - tail)) < 2e-6


def _radial_1d(g, V=None, r_c=6.0):
    """int over the support of (g^2, g'^2 + V g^2 terms) for an l = 0 function g(r) / sqrt(4 pi)."""
    def gv(r):
        a, b = g(np.array([r]))
        return a[0], b[0]
    m = integrate.quad(lambda r: gv(r)[0] ** 2 * r * r, 0, r_c, limit=400, points=[r_c / 2])[0]
    k = integrate.quad(lambda r: 0.5 * gv(r)[1] ** 2 * r * r, 0, r_c, limit=400, points=[r_c / 2])[0]
    pot = 0.0
    if V is not None:
        pot = integrate.quad(lambda r: V(r) * gv(r)[0] ** 2 * r * r, 0, r_c, limit=400,
                             points=[r_c / 2])[0]
    return m, k + pot


def test_enriched_blocks_vs_radial_integrals(hydrogen_small):
    """Same-atom M^ee and H^ee entries equal 1D radial integrals (1s, 2s of hydrogen)."""
    P = hydrogen_small
    enr = P.meta["enr"]
    for a in range(2):
        g = lambda r, a=a: enr.radial_g(a, r)                       # noqa: E731
        m, hval = _radial_1d(g, V=lambda r: -1.0 / r, r_c=enr.r_c)
        assert abs(P.M_ee[a, a] - m) < 1e-8
        assert abs(P.H_ee[a, a] - hval) < 1e-6
    g0 = lambda r: enr.radial_g(0, r)                               # noqa: E731
    g1 = lambda r: enr.radial_g(1, r)                               # noqa: E731
    m01 = integrate.quad(lambda r: g0(np.array([r]))[0][0] * g1(np.array([r]))[0][0] * r * r, 0,
                         enr.r_c, limit=400)[0]
    assert abs(P.M_ee[0, 1] - m01) < 1e-8


def test_coupling_row_sums(hydrogen_small):
    """sum_a M^ec_e[al,a] = int_cell N_al and sum_a H^ec_e[al,a] = int_cell V N_al (partition of unity).

    Summed over every cell this is int N_al and int V N_al, which are 1D radial integrals.
    The support stays clear of boundary cells, so no Dirichlet node is involved.
    """
    P = hydrogen_small
    enr = P.meta["enr"]
    for a in range(2):
        rows = np.nonzero(P.enr_idx == a)[0]
        g = lambda r, a=a: enr.radial_g(a, np.array([r]))[0][0]     # noqa: E731
        intN = integrate.quad(lambda r: g(r) * r * r, 0, enr.r_c, limit=400)[0] * sqrt(4 * pi)
        intVN = integrate.quad(lambda r: -g(r) * r, 0, enr.r_c, limit=400)[0] * sqrt(4 * pi)
        # relative 1e-6: the adaptive rule controls sum N^2 and |grad N|^2 to ~1e-10 of
        # their totals, the signed integral of the 2s function (with cancellation) less tightly
        assert abs(P.M_ec[rows].sum() - intN) < 1e-6 * abs(intN)
        assert abs(P.H_ec[rows].sum() - intVN) < 1e-6 * abs(intVN)


def test_diamond_sites_shells():
    s = configs.diamond_sites(30)
    d = np.sqrt((s ** 2).sum(axis=1))
    assert np.allclose(s[0], 0.0)
    assert abs(d[1] - sqrt(3) / 4 * configs.SI_LATTICE) < 1e-9      # nearest neighbours
    assert np.all(np.diff(np.round(d, 9)) >= 0)
    # nearest-neighbour distance in the cluster is the diamond bond length
    from scipy.spatial.distance import pdist
    assert abs(pdist(s).min() - sqrt(3) / 4 * configs.SI_LATTICE) < 1e-9


def test_generation_is_deterministic_in_worker_count():
    a = configs.si_cluster(n_atoms=2, length=24.0, nc=4, p=2, r_c=6.0, seed=5, workers=1)
    b = configs.si_cluster(n_atoms=2, length=24.0, nc=4, p=2, r_c=6.0, seed=5, workers=3, chunk=2)
    c = configs.si_cluster(n_atoms=2, length=24.0, nc=4, p=2, r_c=6.0, seed=5, workers=1, chunk=2)
    for f in ("H_cc", "H_ec", "M_ec", "H_ee", "M_ee"):
        assert np.array_equal(getattr(b, f), getattr(c, f))
        assert np.allclose(getattr(a, f), getattr(b, f), rtol=1e-12, atol=1e-14)


def test_device_field_recipe_matches_host_field():
    """The perturbation field evaluated as tensors (used where the operator is
    rebuilt on the device each step) is the host recipe: same draws in the
    same order, the same values to rounding."""
    import torch
    from synth import perturb
    rng_a, rng_b = np.random.default_rng(5), np.random.default_rng(5)
    f = perturb.smooth_field(rng_a, -24.0, 48.0)
    c, a, sg = perturb.field_draw(rng_b, -24.0, 48.0)
    pts = np.random.default_rng(6).uniform(-24.0, 24.0, (500, 3))
    ref = f(pts)
    got = perturb.field_at(torch.tensor(pts), c, a, sg).numpy()
    assert np.abs(got - ref).max() <= 1e-15 * max(1.0, np.abs(ref).max())
    # the next draws continue in step
    f2 = perturb.smooth_field(rng_a, -24.0, 48.0)
    c2, a2, sg2 = perturb.field_draw(rng_b, -24.0, 48.0)
    assert np.abs(perturb.field_at(torch.tensor(pts), c2, a2, sg2).numpy() - f2(pts)).max() < 1e-15
