"""GPU-vs-oracle parity through the C ABI (element by element, FP64).

Tolerances (relative to the largest magnitude of the oracle result):
* H X, M X: 1e-12.  Both sides sum the same elemental products in a
  different order; rows collect at most 8 cells x 125 terms plus the
  enrichment terms, so the rounding difference is a few hundred ulps of the
  largest partial sum.
* (M^E)^-1 X: 10 u kappa(M^E), the forward-error scale of a backward-stable
  solve (u = 2^-53; kappa from the extreme eigenvalues of M^E); the device
  applies S^-1 explicitly, the oracle factors M^E by sparse LU.
* filter: 10 u kappa(M^E) per Chebyshev step (m applications of H~).
* Ritz values: 1e-8 Ha absolute (the target accuracy of the method).
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle.filters import recurrence_filter
from oracle.operators import Operators
from oracle.subspace import cholqr, lanczos, lanczos_bounds, rayleigh_ritz

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def relerr(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


_CTX = {}
_KAPPA = {}
U = 2.0 ** -53


def kappa_M(name, ops):
    """Condition number of M^E from its extreme eigenvalues."""
    import scipy.sparse.linalg as spla
    if name not in _KAPPA:
        lmax = spla.eigsh(ops.M, k=1, which="LA", return_eigenvectors=False)[0]
        lmin = spla.eigsh(ops.M, k=1, sigma=0, which="LM", return_eigenvectors=False)[0]
        _KAPPA[name] = lmax / lmin
    return _KAPPA[name]


def context(name, prob, max_cols=96):
    from paper_1610_02121_amd import Context
    key = (name, max_cols)
    if key not in _CTX:
        _CTX[key] = (Context(prob, max_cols=max_cols), Operators(prob))
    return _CTX[key]


FIXTURES = ["tiny_enriched", "hydrogen_small", "si_small"]
WIDTHS = [1, 5, 16, 37, 70]


@pytest.mark.parametrize("fix", FIXTURES)
@pytest.mark.parametrize("N", WIDTHS)
def test_apply_H_M(fix, N, request):
    print(f"[apply_H/M] {fix} N={N}", flush=True)
    ctx, ops = context(fix, request.getfixturevalue(fix))
    X = np.random.default_rng(N).standard_normal((ops.n, N))
    Xd = dev(X)
    assert relerr(host(ctx.apply_H(Xd)), ops.apply_H(X)) < 1e-12
    assert relerr(host(ctx.apply_M(Xd)), ops.apply_M(X)) < 1e-12


@pytest.mark.parametrize("fix", FIXTURES)
@pytest.mark.parametrize("N", [1, 16, 37])
def test_apply_Sinv(fix, N, request):
    print(f"[apply_Sinv] {fix} N={N}", flush=True)
    ctx, ops = context(fix, request.getfixturevalue(fix))
    X = np.random.default_rng(10 + N).standard_normal((ops.n, N))
    Y = host(ctx.apply_Sinv(dev(X)))
    Yo = ops.solve_M(X)
    tol = 10 * U * kappa_M(fix, ops)
    assert relerr(Y, Yo) < tol
    # residual of M (M^-1 X) = X
    assert relerr(ops.apply_M(Y), X) < tol


def test_strided_blocks(si_small):
    """Leading dimensions larger than N (column views of a wider block)."""
    print("[strided] si_small", flush=True)
    ctx, ops = context("si_small", si_small)
    W = np.random.default_rng(3).standard_normal((ops.n, 40))
    Wd = dev(W)
    Xv = Wd[:, 3:24]
    Out = torch.zeros((ops.n, 50), dtype=torch.float64, device="cuda")
    ctx.apply_H(Xv, Out[:, 7:28])
    o = host(Out)
    assert relerr(o[:, 7:28], ops.apply_H(W[:, 3:24])) < 1e-12
    assert np.all(o[:, :7] == 0) and np.all(o[:, 28:] == 0)


@pytest.mark.parametrize("fix,m", [("tiny_enriched", 7), ("hydrogen_small", 12), ("si_small", 10)])
def test_filter(fix, m, request):
    print(f"[filter] {fix} m={m}", flush=True)
    ctx, ops = context(fix, request.getfixturevalue(fix))
    H, M = None, None
    v0 = np.random.default_rng(5).standard_normal(ops.n)
    al, be = lanczos(ops.apply_Htilde, ops.apply_M, v0, 10)
    lo, hi = lanczos_bounds(al, be)
    a = lo + 0.05 * (hi - lo)
    X = np.random.default_rng(6).standard_normal((ops.n, 21))
    Y = host(ctx.filter(dev(X), m, a, hi))
    Yo = recurrence_filter(lambda Z: ops.apply_Htilde(Z), X, m, a, hi)
    assert relerr(Y, Yo) < 10 * U * kappa_M(fix, ops) * m


@pytest.mark.parametrize("fix", FIXTURES)
def test_filter_single_column_strided(fix, request):
    """One column (the single-column cell kernel, with the recurrence fused
    into it) taken from a wider block (leading dimension > 1)."""
    print(f"[filter N=1 strided] {fix}", flush=True)
    ctx, ops = context(fix, request.getfixturevalue(fix))
    W = np.random.default_rng(15).standard_normal((ops.n, 6))
    Wd = dev(W)
    Out = torch.zeros((ops.n, 4), dtype=torch.float64, device="cuda")
    m, a, b = 6, -1.0, 40.0
    ctx.filter(Wd[:, 2:3], m, a, b, Out[:, 1:2])
    o = host(Out)
    Yo = recurrence_filter(lambda Z: ops.apply_Htilde(Z), W[:, 2:3], m, a, b)
    assert relerr(o[:, 1:2], Yo) < 10 * U * kappa_M(fix, ops) * m
    assert np.all(o[:, 0] == 0) and np.all(o[:, 2:] == 0)
    Y1 = host(ctx.apply_H(Wd[:, 4:5]))
    assert relerr(Y1, ops.apply_H(W[:, 4:5])) < 1e-12


@pytest.mark.parametrize("fix", FIXTURES)
def test_single_column_kernels_match_block_kernels(fix, request):
    """The single-column kernels (cell products, coupling partials, transposed
    coupling) against the block kernels on the same column: H x, M x, M^-1 x
    and a filter step agree to a few units of rounding (the sums run in
    different orders)."""
    print(f"[N=1 vs block] {fix}", flush=True)
    ctx, ops = context(fix, request.getfixturevalue(fix))
    W = dev(np.random.default_rng(16).standard_normal((ops.n, 17)))
    col = W[:, 5:6].contiguous()
    for name, f in (("H", ctx.apply_H), ("M", ctx.apply_M), ("Sinv", ctx.apply_Sinv),
                    ("filter", lambda Z: ctx.filter(Z, 3, -1.0, 40.0))):
        one = host(f(col))[:, 0]
        blk = host(f(W))[:, 5]
        tol = 1e-12 if name in ("H", "M") else 10 * U * kappa_M(fix, ops) * 3
        assert np.abs(one - blk).max() <= tol * np.abs(blk).max(), name


def test_filter_degree_zero_and_one(si_small):
    ctx, ops = context("si_small", si_small)
    X = np.random.default_rng(8).standard_normal((ops.n, 9))
    assert np.array_equal(host(ctx.filter(dev(X), 0, -1.0, 5.0)), X)
    Y1 = host(ctx.filter(dev(X), 1, -1.0, 5.0))
    e, c = 2.0 / 6.0, 4.0 / 6.0
    Yo = e * ops.apply_Htilde(X, "solve") - c * X
    assert relerr(Y1, Yo) < 10 * U * kappa_M("si_small", ops)


def test_cholqr(si_small):
    print("[cholqr] si_small", flush=True)
    ctx, ops = context("si_small", si_small)
    X = np.random.default_rng(9).standard_normal((ops.n, 40)) @ np.diag(np.logspace(0, 5, 40))
    Q = host(ctx.cholqr(dev(X)))
    assert np.abs(Q.T @ Q - np.eye(40)).max() < 1e-13
    Qo = cholqr(X)
    # same span: projectors agree
    assert np.abs(Q @ (Q.T @ Qo) - Qo).max() < 1e-11
    # same columns (no sign freedom: both take R with positive diagonal)
    assert relerr(Q, Qo) < 1e-10


@pytest.mark.parametrize("fix,N", [("hydrogen_small", 16), ("si_small", 50), ("tiny_enriched", 7)])
def test_rayleigh_ritz(fix, N, request):
    print(f"[rayleigh_ritz] {fix} N={N}", flush=True)
    ctx, ops = context(fix, request.getfixturevalue(fix))
    v0 = np.random.default_rng(11).standard_normal(ops.n)
    al, be = lanczos(ops.apply_Htilde, ops.apply_M, v0, 10)
    lo, hi = lanczos_bounds(al, be)
    X = np.random.default_rng(12).standard_normal((ops.n, N))
    # a filtered block, as in the method (moderate degree keeps it well conditioned)
    Xf = recurrence_filter(lambda Z: ops.apply_Htilde(Z), X, 6, lo + 0.2 * (hi - lo), hi)
    Yd = dev(Xf)
    theta = ctx.rayleigh_ritz(Yd)
    Q = cholqr(Xf)
    th_o, C = rayleigh_ritz(Q, ops.apply_H(Q), ops.apply_M(Q))
    assert np.abs(theta - th_o).max() < 1e-8
    Z = host(Yd)
    MZ = ops.apply_M(Z)
    assert np.abs(Z.T @ MZ - np.eye(N)).max() < 1e-10
    # Ritz pairs: Z^T H Z = diag(theta)
    assert np.abs(Z.T @ ops.apply_H(Z) - np.diag(theta)).max() < 1e-8 * max(1.0, np.abs(theta).max())


@pytest.mark.parametrize("fix", FIXTURES)
def test_lanczos_bounds(fix, request):
    print(f"[lanczos] {fix}", flush=True)
    ctx, ops = context(fix, request.getfixturevalue(fix))
    v0 = np.random.default_rng(13).standard_normal(ops.n)
    lo, hi = ctx.lanczos_bounds(dev(v0).reshape(-1), 10)
    al, be = lanczos(ops.apply_Htilde, ops.apply_M, v0, 10)
    lo_o, hi_o = lanczos_bounds(al, be)
    assert abs(lo - lo_o) < 1e-9 * abs(hi_o) and abs(hi - hi_o) < 1e-9 * abs(hi_o)


def test_determinism(si_small):
    ctx, ops = context("si_small", si_small)
    X = dev(np.random.default_rng(14).standard_normal((ops.n, 33)))
    a = host(ctx.filter(X, 4, -2.0, 50.0))
    b = host(ctx.filter(X, 4, -2.0, 50.0))
    assert np.array_equal(a, b)


def test_scf_steps_match_oracle(hydrogen_cfg1):
    """Two subspace-iteration steps (filter m = 20, Rayleigh-Ritz) from the same
    start: GPU and oracle Ritz values agree to 1e-8 Ha at every step."""
    print("[scf] hydrogen 8^3", flush=True)
    ctx, ops = context("hydrogen_cfg1", hydrogen_cfg1, max_cols=16)
    N, m = 16, 20
    X = np.random.default_rng(0).standard_normal((ops.n, N))
    v0 = np.random.default_rng(1).standard_normal(ops.n)
    lo, b = ctx.lanczos_bounds(dev(v0).reshape(-1), 10)
    Xd = dev(X)
    th = ctx.rayleigh_ritz(Xd)
    Q = cholqr(X)
    th_o, C = rayleigh_ritz(Q, ops.apply_H(Q), ops.apply_M(Q))
    Xo = Q @ C
    assert np.abs(th - th_o).max() < 1e-8
    for step in range(2):
        a = th[-1]
        Yd = ctx.filter(Xd, m, a, b)
        th = ctx.rayleigh_ritz(Yd)
        Yo = recurrence_filter(lambda Z: ops.apply_Htilde(Z), Xo, m, th_o[-1], b)
        Q = cholqr(Yo)
        th_o, C = rayleigh_ritz(Q, ops.apply_H(Q), ops.apply_M(Q))
        Xo = Q @ C
        Xd = Yd
        assert np.abs(th - th_o).max() < 1e-8, step


# ---------------------------------------------------------------- error paths
def test_invalid_arguments(si_small):
    from paper_1610_02121_amd import ChebFilterError
    ctx, ops = context("si_small", si_small)
    X = dev(np.ones((ops.n, 4)))
    with pytest.raises(ChebFilterError, match="CF_EINVAL"):
        ctx.filter(X, 3, 1.0, 1.0)
    with pytest.raises(ChebFilterError, match="CF_EINVAL"):
        ctx.filter(X, -1, 0.0, 1.0)
    with pytest.raises(ChebFilterError, match="CF_EINVAL"):
        ctx.filter(X, 2, 0.0, float("nan"))
    # in place is allowed only with one leading dimension
    W = dev(np.ones((ops.n, 8)))
    with pytest.raises(ChebFilterError, match="CF_EINVAL"):
        ctx.filter(W[:, :4], 2, 0.0, 1.0, Y=torch.as_strided(W, (ops.n, 4), (4, 1)))
    with pytest.raises(ChebFilterError, match="CF_EINVAL"):
        ctx.filter(X, 2, 0.0, 1.0, prec=7)
    big = dev(np.ones((ops.n, ctx.max_cols + 1)))
    with pytest.raises(ChebFilterError, match="CF_ENOMEM"):
        ctx.apply_H(big)
    with pytest.raises(ChebFilterError, match="CF_ENOTSPD"):
        ctx.cholqr(dev(np.zeros((ops.n, 3))))
    empty = dev(np.ones((ops.n, 0)))
    assert ctx.apply_H(empty).shape == (ops.n, 0)


def test_init_rejects_bad_problems(tiny_enriched):
    import copy
    from paper_1610_02121_amd import ChebFilterError, Context
    P = copy.deepcopy(tiny_enriched)
    P.M_ee = np.zeros_like(P.M_ee)                # Schur complement negative definite
    with pytest.raises(ChebFilterError, match="CF_ENOTSPD"):
        Context(P, max_cols=4)
    Q = copy.deepcopy(tiny_enriched)
    Q.H_cc = Q.H_cc.copy()
    Q.H_cc[0, 0, 1] += 1.0                        # not symmetric
    with pytest.raises(ChebFilterError, match="CF_EINVAL"):
        Context(Q, max_cols=4)
    R = copy.deepcopy(tiny_enriched)
    R.cell_dof = R.cell_dof.copy()
    R.cell_dof[0, 0] = R.n_h + 5                  # out of range
    with pytest.raises(ChebFilterError, match="CF_EINVAL"):
        Context(R, max_cols=4)
    S = copy.deepcopy(tiny_enriched)
    S.enr_idx = S.enr_idx.copy()
    S.enr_idx[0] = 7                              # alpha >= n_e
    with pytest.raises(ChebFilterError, match="CF_EINVAL"):
        Context(S, max_cols=4)


# ------------------------------------------- widths the benchmark runs, chunks
def report(name, theta, th_ref, wanted, Z=None, Z_ref=None, M=None):
    """Print the Ritz error, band-energy error and (when both vector sets are
    given) the largest principal angle between the wanted Ritz spaces."""
    from oracle.subspace import energy_error, ritz_error, subspace_angle
    msg = (f"[metrics] {name}: ritz_err={ritz_error(theta, th_ref, wanted):.3e} Ha "
           f"energy_err={energy_error(theta, th_ref, wanted):.3e} Ha")
    if Z is not None:
        msg += f" angle={subspace_angle(Z_ref[:, :wanted], Z[:, :wanted], M):.3e} rad"
    print(msg, flush=True)


@pytest.mark.parametrize("N,chunk", [(65, 0), (128, 0), (200, 0), (200, 64), (130, 48)])
def test_cholqr_multi_tile(si_small, N, chunk):
    """Cholesky-QR past one 64 x 64 Gram tile (upper-tile mapping, skipped
    blocks below the diagonal), and in place by row blocks when N exceeds the
    column chunk: orthonormal to 1e-13 and the oracle's Q to 1e-10."""
    print(f"[cholqr] si_small N={N} chunk={chunk}", flush=True)
    ctx, ops = context("si_small", si_small, max_cols=200) if chunk == 0 else \
        chunked_context("si_small", si_small, 200, chunk)
    X = np.random.default_rng(31).standard_normal((ops.n, N)) @ np.diag(np.logspace(0, 4, N))
    Q = host(ctx.cholqr(dev(X)))
    assert np.abs(Q.T @ Q - np.eye(N)).max() < 1e-13
    assert relerr(Q, cholqr(X)) < 1e-10


def chunked_context(name, prob, max_cols, chunk):
    from paper_1610_02121_amd import Context
    key = (name, max_cols, "chunk", chunk)
    if key not in _CTX:
        _CTX[key] = (Context(prob, max_cols=max_cols, col_chunk=chunk), Operators(prob))
    return _CTX[key]


@pytest.mark.parametrize("N,chunk", [(65, 0), (128, 0), (200, 0), (200, 64), (130, 48)])
def test_rayleigh_ritz_multi_tile(si_small, N, chunk):
    """Rayleigh-Ritz of a filtered block at widths past one Gram tile, whole
    and by column slabs: Ritz values within 1e-8 Ha of the oracle's, Z^T M Z = I,
    Z^T H Z = diag(theta); the wanted Ritz space's angle to the oracle's."""
    print(f"[rayleigh_ritz] si_small N={N} chunk={chunk}", flush=True)
    ctx, ops = context("si_small", si_small, max_cols=200) if chunk == 0 else \
        chunked_context("si_small", si_small, 200, chunk)
    v0 = np.random.default_rng(11).standard_normal(ops.n)
    al, be = lanczos(ops.apply_Htilde, ops.apply_M, v0, 10)
    lo, hi = lanczos_bounds(al, be)
    X = np.random.default_rng(32).standard_normal((ops.n, N))
    Xf = recurrence_filter(lambda Z: ops.apply_Htilde(Z), X, 6, lo + 0.2 * (hi - lo), hi)
    Yd = dev(Xf)
    theta = ctx.rayleigh_ritz(Yd)
    Q = cholqr(Xf)
    th_o, C = rayleigh_ritz(Q, ops.apply_H(Q), ops.apply_M(Q))
    Z = host(Yd)
    wanted = N - N // 5
    report(f"rayleigh_ritz si_small N={N} chunk={chunk}", theta, th_o, wanted, Z, Q @ C, ops.M)
    assert np.abs(theta - th_o).max() < 1e-8
    assert np.abs(Z.T @ ops.apply_M(Z) - np.eye(N)).max() < 1e-10
    assert np.abs(Z.T @ ops.apply_H(Z) - np.diag(theta)).max() < 1e-8 * max(1.0, np.abs(theta).max())


def test_column_chunks_equal_whole_blocks(si_small):
    """A context with 64-column work blocks gives, on N = 200 (chunks 64, 64,
    64, 8), bit for bit the whole-block results of H X, M X, (M^E)^-1 X and
    the FP64 / FP32 filters (columns are independent), and the filter in
    place equals the filter into a separate block."""
    print("[chunks] si_small N=200 chunk=64", flush=True)
    whole, ops = context("si_small", si_small, max_cols=200)
    ch, _ = chunked_context("si_small", si_small, 200, 64)
    X = dev(np.random.default_rng(33).standard_normal((ops.n, 200)))
    for f in ("apply_H", "apply_M", "apply_Sinv"):
        assert torch.equal(getattr(whole, f)(X), getattr(ch, f)(X)), f
    for prec in ("fp64", "fp32"):
        a = whole.filter(X, 5, -2.0, 60.0, prec=prec)
        b = ch.filter(X, 5, -2.0, 60.0, prec=prec)
        assert torch.equal(a, b), prec
        Xi = X.clone()
        ch.filter(Xi, 5, -2.0, 60.0, Y=Xi, prec=prec)
        assert torch.equal(Xi, b), prec
    th = np.linspace(-1.0, 3.0, 200)
    assert np.array_equal(whole.residual_norms(X, th), ch.residual_norms(X, th))



def test_epilogue_paths_agree(si_small):
    """The epilogue's two-columns-per-lane path (aligned blocks, even leading
    dimensions) and its element path (here forced by an odd leading
    dimension) compute each element the same way: filters, H X, M X and
    (M^E)^-1 X agree bit for bit."""
    ctx, ops = context("si_small", si_small, max_cols=96)
    X = np.random.default_rng(35).standard_normal((ops.n, 40))
    Xe = dev(X)
    W = torch.zeros((ops.n, 41), dtype=torch.float64, device="cuda")
    W[:, :40] = Xe
    Xo = W[:, :40]
    assert Xo.stride(0) == 41
    for name, f in (("H", ctx.apply_H), ("M", ctx.apply_M), ("Sinv", ctx.apply_Sinv),
                    ("filter", lambda Z, Y=None: ctx.filter(Z, 5, -2.0, 60.0, Y=Y))):
        a = f(Xe)
        Yo = torch.zeros((ops.n, 41), dtype=torch.float64, device="cuda")[:, :40]
        b = f(Xo, Y=Yo)
        assert torch.equal(a, b), name
