"""Pins of the FP64 oracle against closed forms, textbook limits, library
routines and brute force (none re-types the oracle's own formulas)."""
import os
from math import pi, sqrt

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla
from numpy.polynomial import chebyshev as npcheb
from scipy import integrate

from oracle.filters import chebyshev_T, exact_filter, recurrence_filter
from oracle.operators import Operators
from oracle.subspace import (cholqr, lanczos, lanczos_bounds, rayleigh_ritz, scf_step,
                             subspace_angle)
from synth import configs

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _ops(prob):
    return Operators(prob)


# ------------------------------------------------------------------ assembly
def test_particle_in_a_box():
    """V = 0, no enrichment: lambda -> pi^2 (n1^2+n2^2+n3^2) / (2 L^2) (P3)."""
    L = 3.0
    ops = _ops(configs.box(nc=3, length=L, p=4))
    H, M = ops.dense()
    lam = sla.eigh(H, M, eigvals_only=True)[:7]
    ex = pi ** 2 / (2 * L ** 2) * np.array([3, 6, 6, 6, 9, 9, 9])
    assert np.max(np.abs(lam - ex) / ex) < 2e-4
    # degeneracy structure of the cube
    assert np.ptp(lam[1:4]) < 1e-9 and np.ptp(lam[4:7]) < 1e-9


def test_box_spectral_convergence_in_p():
    L = 2.0
    errs = []
    for p in (2, 3, 4):
        ops = _ops(configs.box(nc=2, length=L, p=p))
        H, M = ops.dense()
        lam = sla.eigh(H, M, eigvals_only=True)[0]
        errs.append(abs(lam - 3 * pi ** 2 / (2 * L ** 2)))
    assert errs[0] > 5 * errs[1] > 25 * errs[2]


@pytest.mark.slow
def test_hydrogen_ground_state(hydrogen_cfg1):
    """Enriched basis on the 8^3 mesh: lambda_1 within 1e-4 of -1/2 Ha (P9).

    The classical-only basis on the same mesh misses it by more (3.7e-4 below,
    the GLL-lumped overlap lowers eigenvalues), so the coupling blocks matter.
    """
    E = dict(np.loadtxt(os.path.join(GOLD, "hydrogen_levels.txt")))
    ops = _ops(hydrogen_cfg1)
    lam = np.sort(spla.eigsh(ops.H, k=5, M=ops.M, sigma=-1.0, which="LM")[0])
    assert abs(lam[0] - E[1.0]) < 1e-4
    # n = 2 levels, shifted up by the 20 Bohr box (2p: three-fold)
    assert np.ptp(lam[1:4]) < 1e-8 and 0 < lam[1] - E[2.0] < 5e-3 and 0 < lam[4] - E[2.0] < 1e-2


def test_global_coupling_row_sums(hydrogen_cfg1):
    """The assembled M^E and H^E rows of an enrichment DOF, summed over the classical
    columns, equal int N_al and int V N_al (1D radial integrals; partition of unity).
    On this mesh the supports (r < 6) stay clear of the boundary cells (|x| > 7.5)."""
    P = hydrogen_cfg1
    ops = _ops(P)
    enr = P.meta["enr"]
    for a in range(2):
        g = lambda r, a=a: enr.radial_g(a, np.array([r]))[0][0]     # noqa: E731
        intN = integrate.quad(lambda r: g(r) * r * r, 0, enr.r_c, limit=400)[0] * sqrt(4 * pi)
        intVN = integrate.quad(lambda r: -g(r) * r, 0, enr.r_c, limit=400)[0] * sqrt(4 * pi)
        row = ops.n_h + a
        assert abs(ops.M[row, :ops.n_h].sum() - intN) < 1e-6 * abs(intN)
        assert abs(ops.H[row, :ops.n_h].sum() - intVN) < 1e-6 * abs(intVN)
        # symmetric placement of the coupling block
        assert abs(ops.M[:ops.n_h, row].sum() - ops.M[row, :ops.n_h].sum()) < 1e-12
    assert abs(ops.M - ops.M.T).max() < 1e-15 and abs(ops.H - ops.H.T).max() < 1e-14


def test_enrichment_basis_invariance(tiny_enriched):
    """Rescaling or permuting enrichment functions leaves the spectrum unchanged (P12)."""
    P = tiny_enriched
    H, M = _ops(P).dense()
    lam = sla.eigh(H, M, eigvals_only=True)
    s = np.array([3.0, -0.25])
    import copy
    Q = copy.deepcopy(P)
    Q.H_ec = P.H_ec * s[P.enr_idx][:, None]
    Q.M_ec = P.M_ec * s[P.enr_idx][:, None]
    Q.H_ee = P.H_ee * np.outer(s, s)
    Q.M_ee = P.M_ee * np.outer(s, s)
    H2, M2 = _ops(Q).dense()
    assert np.allclose(sla.eigh(H2, M2, eigvals_only=True), lam, rtol=1e-9, atol=1e-11)
    perm = np.array([1, 0])
    Q2 = copy.deepcopy(P)
    Q2.enr_idx = perm[P.enr_idx]
    Q2.H_ee = P.H_ee[np.ix_(np.argsort(perm), np.argsort(perm))]
    Q2.M_ee = P.M_ee[np.ix_(np.argsort(perm), np.argsort(perm))]
    H3, M3 = _ops(Q2).dense()
    assert np.allclose(sla.eigh(H3, M3, eigvals_only=True), lam, rtol=1e-10, atol=1e-12)


# ------------------------------------------------------------------ overlap inverse
@pytest.mark.parametrize("fix", ["tiny_enriched", "si_small"])
def test_block_inverse_equals_direct_solve(fix, request):
    """Banachiewicz block inverse == sparse direct solve; M (M^-1 r) = r (P5)."""
    P = request.getfixturevalue(fix)
    ops = _ops(P)
    R = np.random.default_rng(0).standard_normal((ops.n, 5))
    Y1 = ops.block_inverse(R)
    Y2 = ops.solve_M(R)
    assert np.abs(Y1 - Y2).max() <= 1e-9 * np.abs(Y2).max()
    assert np.abs(ops.apply_M(Y1) - R).max() <= 1e-10 * np.abs(R).max()
    S = ops.schur()
    assert np.linalg.eigvalsh(S).min() > 0


def test_block_inverse_dense(tiny_enriched):
    ops = _ops(tiny_enriched)
    H, M = ops.dense()
    R = np.random.default_rng(1).standard_normal((ops.n, 3))
    assert np.allclose(ops.block_inverse(R), np.linalg.solve(M, R), rtol=1e-11, atol=1e-12)


# ------------------------------------------------------------------ Chebyshev
def test_chebyshev_closed_form_matches_series():
    x = np.linspace(-2.5, 2.5, 101)
    for m in (0, 1, 2, 7, 20):
        c = np.zeros(m + 1)
        c[m] = 1.0
        assert np.allclose(chebyshev_T(m, x), npcheb.chebval(x, c), rtol=1e-11, atol=1e-12)
        assert chebyshev_T(m, np.array([1.0]))[0] == 1.0
        assert chebyshev_T(m, np.array([-1.0]))[0] == (-1.0) ** m


@pytest.mark.parametrize("m", [0, 1, 2, 5, 12])
def test_recurrence_equals_exact_filter(tiny_enriched, m):
    """Three-term recurrence (both M^-1 routes) == V T_m(t(Lambda)) V^T M X (P6)."""
    ops = _ops(tiny_enriched)
    H, M = ops.dense()
    lam = sla.eigh(H, M, eigvals_only=True)
    a, b = lam[4], lam[-1] * 1.01
    X = np.random.default_rng(2).standard_normal((ops.n, 6))
    Y = exact_filter(H, M, X, m, a, b)
    for how in ("block", "solve"):
        Yr = recurrence_filter(lambda Z: ops.apply_Htilde(Z, how), X, m, a, b)
        assert np.abs(Yr - Y).max() <= 1e-10 * max(1.0, np.abs(Y).max())


def test_filter_on_eigenvector(tiny_enriched):
    ops = _ops(tiny_enriched)
    H, M = ops.dense()
    lam, V = sla.eigh(H, M)
    a, b = lam[3], lam[-1]
    m = 9
    for i in (0, 3, len(lam) - 1):
        y = recurrence_filter(lambda Z: ops.apply_Htilde(Z), V[:, [i]], m, a, b)
        f = chebyshev_T(m, np.array([(2 * lam[i] - a - b) / (b - a)]))[0]
        assert np.allclose(y[:, 0], f * V[:, i], rtol=1e-8, atol=1e-10 * abs(f))


def test_filter_rejects_bad_bounds(tiny_enriched):
    ops = _ops(tiny_enriched)
    X = np.ones((ops.n, 1))
    with pytest.raises(ValueError):
        recurrence_filter(ops.apply_Htilde, X, 3, 1.0, 1.0)
    with pytest.raises(ValueError):
        recurrence_filter(ops.apply_Htilde, X, -1, 0.0, 1.0)


# ------------------------------------------------------------------ CholQR / RR / Lanczos
def test_cholqr_orthonormal_and_span():
    Y = np.random.default_rng(3).standard_normal((500, 20)) @ np.diag(np.logspace(0, 6, 20))
    Q = cholqr(Y)
    assert np.abs(Q.T @ Q - np.eye(20)).max() < 1e-13
    # same span: Y is reproduced by projecting onto Q
    assert np.abs(Q @ (Q.T @ Y) - Y).max() < 1e-12 * np.abs(Y).max()
    # agrees with LAPACK QR up to column signs
    Qr, _ = np.linalg.qr(Y)
    assert np.allclose(np.abs(Q.T @ Qr), np.eye(20), atol=1e-10)


def test_rayleigh_ritz_bounds_and_exactness(tiny_enriched):
    """theta_i >= lambda_i (Courant-Fischer); exact eigenvectors give theta = lambda (P8)."""
    ops = _ops(tiny_enriched)
    H, M = ops.dense()
    lam, V = sla.eigh(H, M)
    X = np.random.default_rng(4).standard_normal((ops.n, 8))
    Q = cholqr(X)
    th, C = rayleigh_ritz(Q, ops.apply_H(Q), ops.apply_M(Q))
    assert np.all(th >= lam[:8] - 1e-12)
    Q = cholqr(V[:, :5])
    th, C = rayleigh_ritz(Q, ops.apply_H(Q), ops.apply_M(Q))
    assert np.allclose(th, lam[:5], atol=1e-11)
    # invariance under X -> X G
    G = np.random.default_rng(5).standard_normal((8, 8))
    th1, _ = rayleigh_ritz(cholqr(X), ops.apply_H(cholqr(X)), ops.apply_M(cholqr(X)))
    XG = X @ G
    th2, _ = rayleigh_ritz(cholqr(XG), ops.apply_H(cholqr(XG)), ops.apply_M(cholqr(XG)))
    assert np.allclose(th1, th2, atol=1e-10)
    # Ritz vectors are M-orthonormal
    Qx = cholqr(X)
    th, C = rayleigh_ritz(Qx, ops.apply_H(Qx), ops.apply_M(Qx))
    Z = Qx @ C
    assert np.abs(Z.T @ M @ Z - np.eye(8)).max() < 1e-11


def test_lanczos_brackets_spectrum(tiny_enriched):
    ops = _ops(tiny_enriched)
    H, M = ops.dense()
    lam = sla.eigh(H, M, eigvals_only=True)
    v0 = np.random.default_rng(6).standard_normal(ops.n)
    al, be = lanczos(ops.apply_Htilde, ops.apply_M, v0, 10)
    lo, hi = lanczos_bounds(al, be)
    assert hi >= lam[-1] - 1e-9 and lo >= lam[0] - 1e-9
    # a full run (k = n) reproduces the extreme eigenvalues
    al, be = lanczos(ops.apply_Htilde, ops.apply_M, v0, ops.n)
    T = np.diag(al) + np.diag(be[:-1], 1) + np.diag(be[:-1], -1)
    ev = np.linalg.eigvalsh(T)
    assert abs(ev[0] - lam[0]) < 1e-8 * abs(lam).max() and abs(ev[-1] - lam[-1]) < 1e-8 * abs(lam).max()


def test_chefsi_converges_to_dense_spectrum(tiny_enriched):
    """Brute force (P10): filter -> CholQR -> RR iterations reach the dense spectrum."""
    ops = _ops(tiny_enriched)
    H, M = ops.dense()
    lam = sla.eigh(H, M, eigvals_only=True)
    N, wanted = 6, 4
    X = np.random.default_rng(7).standard_normal((ops.n, N))
    Q = cholqr(X)
    th, C = rayleigh_ritz(Q, ops.apply_H(Q), ops.apply_M(Q))
    X = Q @ C
    al, be = lanczos(ops.apply_Htilde, ops.apply_M, np.ones(ops.n), 10)
    b = lanczos_bounds(al, be)[1]
    for _ in range(30):
        th, X = scf_step(ops, X, 8, th[-1], b)
    assert np.max(np.abs(th[:wanted] - lam[:wanted])) < 1e-10
    _, V = sla.eigh(H, M)
    assert subspace_angle(X[:, :wanted], V[:, :wanted], M) < 1e-6


def test_sampled_rows_match_global_operators(si_small):
    """The per-row element sums (used where the global operator is too large)
    against the assembled global H^E and M^E, on classical rows inside,
    touching and outside the enriched region, and on enrichment rows."""
    from oracle.operators import Operators, sampled_rows
    prob = si_small
    ops = Operators(prob)
    rng = np.random.default_rng(31)
    X = rng.standard_normal((ops.n, 3))
    rows = np.concatenate([rng.choice(prob.n_h, 40, replace=False),
                           prob.n_h + rng.choice(prob.n_e, 10, replace=False)])
    for which, A in (("H", ops.H), ("M", ops.M)):
        Yo = np.asarray(A[rows] @ X)
        Ys = sampled_rows(prob, rows, X, which)
        assert np.abs(Ys - Yo).max() < 1e-12 * np.abs(Yo).max(), which


def test_sampled_rows_constant_potential_row_sums(si_small):
    """With the plain cells' blocks rebuilt for V = c (oracle assembly), a
    classical row of H applied to the constant vector, for a DOF whose cells
    are all plain and away from the boundary, is c times the lumped GLL
    weight of the DOF (the kinetic part annihilates constants; the row sum of
    the consistent mass is the integral of the shape function, which the GLL
    rule integrates exactly)."""
    from oracle.assembly import plain_cell_block
    from oracle.operators import sampled_rows
    from synth.assemble import plain_tables
    prob = si_small
    B, w, K, _ = plain_tables(prob)
    cd = np.asarray(prob.cell_dof)
    ep = np.asarray(prob.enr_ptr)
    plain = ep[1:] == ep[:-1]
    c = -0.7
    blocks = {e: plain_cell_block(K, B, w, np.full(len(w), c)) for e in np.nonzero(plain)[0]}
    good = [i for i in range(prob.n_h)
            if all(plain[e] and (cd[e] >= 0).all() for e in np.nonzero((cd == i).any(1))[0])]
    assert len(good) > 5
    rows = np.array(good[:: max(1, len(good) // 12)])
    X = np.zeros((prob.n, 1))
    X[:prob.n_h] = 1.0
    Y = sampled_rows(prob, rows, X, "H", H_cc=blocks)[:, 0]
    D = np.asarray(prob.M_cc_diag)[rows]
    assert np.abs(Y - c * D).max() < 1e-12 * abs(c) * D.max()


# ------------------------------------------------------------- error metrics
def _angle_pair(t, n=9, seed=11):
    """Euclidean spans with principal angles t (closed form): A = [e_1..e_k],
    B = [cos t_i e_i + sin t_i e_{k+i}], rotated by a random orthogonal Q."""
    k = len(t)
    A = np.zeros((n, k))
    B = np.zeros((n, k))
    for i, ti in enumerate(t):
        A[i, i] = 1.0
        B[i, i] = np.cos(ti)
        B[k + i, i] = np.sin(ti)
    Q, _ = np.linalg.qr(np.random.default_rng(seed).standard_normal((n, n)))
    G = np.random.default_rng(seed + 1).standard_normal((k, k)) + 3 * np.eye(k)   # any basis
    return Q @ A @ G, Q @ B


@pytest.mark.parametrize("t", [(0.3, 1e-9, 0.05), (1.2, 0.7, 0.2), (3e-11, 1e-12, 2e-12)])
def test_subspace_angle_closed_form_euclidean(t):
    """Largest principal angle = max t_i exactly, also below arccos's resolution
    (a min/max mix-up returns the smallest t_i; arccos of the smallest
    cosine returns 0 or ~1e-8 for the tiny angles; an arcsin/arccos swap
    returns pi/2 - t)."""
    A, B = _angle_pair(t)
    got = subspace_angle(A, B, np.eye(A.shape[0]))
    assert abs(got - max(t)) <= 1e-14 + 1e-9 * max(t)


def test_subspace_angle_closed_form_M_weighted():
    """In the M inner product, M = G^T G: angles between span(G^-1 A) and
    span(G^-1 B) equal the Euclidean angles between span(A) and span(B)."""
    t = (0.4, 0.02, 1e-7)
    A, B = _angle_pair(t, n=10, seed=5)
    G = np.random.default_rng(2).standard_normal((10, 10)) + 4 * np.eye(10)
    Gi = np.linalg.inv(G)
    M = G.T @ G
    got = subspace_angle(Gi @ A, Gi @ B, M)
    assert abs(got - 0.4) <= 1e-12
    # the Euclidean angle of the same pair differs (the weight matters)
    assert abs(subspace_angle(Gi @ A, Gi @ B, np.eye(10)) - 0.4) > 1e-3


def test_ritz_and_energy_error_hand_computed():
    """Hand-computed: theta = (-1, -0.5, 3), lambda = (-1.02, -0.45, 0),
    two wanted: Ritz error max(0.02, 0.05) = 0.05; energy error
    2 |(-1.5) - (-1.47)| = 0.06; the unwanted third pair is ignored."""
    from oracle.subspace import energy_error, ritz_error
    th = np.array([-1.0, -0.5, 3.0])
    lam = np.array([-1.02, -0.45, 0.0])
    assert abs(ritz_error(th, lam, 2) - 0.05) < 1e-15
    assert abs(energy_error(th, lam, 2) - 0.06) < 1e-15
    assert abs(ritz_error(th, lam, 3) - 3.0) < 1e-15


# ------------------------------------------------------- cell-wise operators
@pytest.mark.parametrize("fix", ["tiny_enriched", "si_small", "hydrogen_classical"])
def test_cellwise_operators_equal_assembled(fix, request):
    """The cell-by-cell products (used on problems whose global matrices do
    not fit) against the assembled global H^E, M^E, the sparse direct solve
    of M^E and the assembled Schur complement."""
    from oracle.cellwise import CellOperators
    prob = request.getfixturevalue(fix)
    ops = _ops(prob)
    co = CellOperators(prob)
    X = np.random.default_rng(4).standard_normal((ops.n, 5))
    for a, b in ((ops.apply_H(X), co.apply_H(X).numpy()), (ops.apply_M(X), co.apply_M(X).numpy())):
        assert np.abs(a - b).max() <= 1e-13 * np.abs(a).max()
    y = ops.solve_M(X)
    assert np.abs(co.block_inverse(X).numpy() - y).max() <= 1e-10 * np.abs(y).max()
    if prob.n_e:
        assert np.abs(co.schur() - ops.schur()).max() <= 1e-13 * np.abs(ops.schur()).max()
