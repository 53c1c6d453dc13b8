"""Reduced-precision filter forms (CF_FP32, CF_BF16) against the oracle.

What the reduced forms compute: FP32 recurrence blocks; elemental and coupling
products on FP32 MFMA (CF_BF16: cell matrices and gathered vector tiles
rounded to BF16, products accumulated in FP32); enrichment-row sums, the
Schur-complement solve and its output in FP64.

Tolerances (u32 = 2^-24, ub = 2^-8 unit roundoffs):
* Degree 1, rows outside the enriched region.  There the step is
  y_i = e d_i^-1 (H^cc x)_i - c x_i, with no coupling and no Schur solve, so
  the error has an elementwise bound free of conditioning:
    |y_i - y_model,i| <= e d_i^-1 (K + 2) u32 (|H^cc| |x|)_i + 4 u32 (e d_i^-1 |(H^cc x)_i| + |c x_i|),
  K = 136 the longest chain of FP32 roundings behind an output: 128 padded
  products summed within a cell (the MFMA chain) and up to 8 cell partials
  added in turn (+2 for the FP32 copies of H^cc and of d^-1).  The inputs x are exactly representable
  in BF16, and for CF_BF16 the model H^cc is the device's BF16 rounding of the
  cell matrices (to nearest, ties to even, from FP64), so the bound holds for both
  forms with the FP32 constant: it pins the BF16 operand layout and rounding,
  not just the magnitude of the error.  (The BF16 form takes BF16 products
  only in cells with no DOF in the enriched region; the model does the same.)
* All rows, each Chebyshev step k = 1..m: the device's Y_k against the model
  step applied to the device's own Y_{k-1}, Y_{k-2} (outputs of the filters
  of degree k-1 and k-2, which are the same FP32 iterates widened exactly):
  10 u32 kappa(M^E), the FP64 parity bound of one step with FP32's unit
  roundoff.  For CF_BF16 the model step rounds H^cc and the classical rows of
  Y_{k-1} to BF16 as the device does, so the check stays at FP32 level.
* All rows, whole filter (CF_FP32): 10 u32 kappa(M^E) per step against the
  FP64 oracle (the FP32 copy of the operator is within that).
* Wide damping interval, m = 60 (iterates far beyond FP32's range unscaled):
  the last step against the model, and for CF_FP32 the whole filter against
  the oracle, with the bounds above.
* Mixed subspace iteration: reduced-precision filter passes, then FP64
  passes (the cleanup); Ritz values of the wanted set within 1e-6 Ha of the
  eigenvalues of the discrete pencil.
"""
import copy

import numpy as np
import pytest

from oracle.filters import recurrence_filter
from oracle.operators import Operators
from oracle.subspace import lanczos, lanczos_bounds

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

U32 = 2.0 ** -24
UB = 2.0 ** -8


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def bf16_round(x):
    """Round FP64 values to the nearest BF16 (ties to even) in one rounding, as
    the device converts the cell matrices (and FP32 vector values, for which
    this is the same as rounding from FP32), returned as FP64."""
    b = np.ascontiguousarray(x, dtype=np.float64).view(np.uint64)
    b = (b + np.uint64((1 << 44) - 1) + ((b >> np.uint64(45)) & np.uint64(1))) \
        & ~np.uint64((1 << 45) - 1)
    return b.view(np.float64)


def bf16_block(shape, seed):
    return bf16_round(np.random.default_rng(seed).standard_normal(shape))


_CTX = {}


def context(name, prob, max_cols=48):
    from paper_1610_02121_amd import Context
    if name not in _CTX:
        _CTX[name] = (Context(prob, max_cols=max_cols), Operators(prob))
    return _CTX[name]


def kappa_M(ops):
    import scipy.sparse.linalg as spla
    lmax = spla.eigsh(ops.M, k=1, which="LA", return_eigenvectors=False)[0]
    lmin = spla.eigsh(ops.M, k=1, sigma=0, which="LM", return_eigenvectors=False)[0]
    return lmax / lmin


def region_dofs(prob):
    """Mask of the classical DOFs that belong to an enriched cell."""
    cd = np.asarray(prob.cell_dof)
    ep = np.asarray(prob.enr_ptr)
    enriched = np.nonzero(ep[1:] > ep[:-1])[0]
    inside = np.zeros(prob.n_h, dtype=bool)
    d = cd[enriched].ravel()
    inside[d[d >= 0]] = True
    return inside


def far_cells(prob):
    """Cells with no DOF in the enriched region: the only cells whose products
    the BF16 form takes in BF16 (the others stay FP32)."""
    inside = region_dofs(prob)
    cd = np.asarray(prob.cell_dof)
    return np.array([not inside[r[r >= 0]].any() for r in cd])


def outside_rows(prob):
    """Classical DOFs that belong to no enriched cell."""
    return np.nonzero(~region_dofs(prob))[0]


_MODEL = {}


class Model:
    """The FP64 operator the reduced form approximates to FP32 rounding.  For
    CF_BF16 the far cells' matrices are the device's BF16 values, and the
    classical rows of the vector enter those cells' products rounded to BF16."""

    def __init__(self, prob, prec):
        self.prec = prec
        self.prob = prob
        self.far = None
        if prec == "bf16":
            far = far_cells(prob)
            H = np.asarray(prob.H_cc, dtype=np.float64)
            Hs = 0.5 * (H + H.transpose(0, 2, 1))
            Hm = np.where(far[:, None, None], bf16_round(Hs), Hs)
            P = copy.deepcopy(prob)
            P.H_cc = Hm
            self.prob = P
            if far.any():
                F = copy.deepcopy(prob)
                F.H_cc = np.where(far[:, None, None], Hm, 0.0)
                self.far = Operators(F).H[:prob.n_h, :prob.n_h].tocsr()
        self.ops = Operators(self.prob)

    def htilde(self, X):
        HX = np.asarray(self.ops.H @ X)
        if self.far is not None:
            n_h = self.ops.n_h
            HX[:n_h] += np.asarray(self.far @ (bf16_round(X[:n_h]) - X[:n_h]))
        return self.ops.block_inverse(HX)


def model(name, prob, prec):
    if (name, prec) not in _MODEL:
        _MODEL[(name, prec)] = Model(prob, prec)
    return _MODEL[(name, prec)]


def abs_classical_product(prob, X):
    """(|H^cc| |X|) over the classical rows, |H^cc| assembled from |H_e|."""
    P = copy.deepcopy(prob)
    P.H_cc = np.abs(np.asarray(prob.H_cc, dtype=np.float64))
    A = Operators(P)
    return np.asarray(A.H[:prob.n_h, :prob.n_h] @ np.abs(X[:prob.n_h]))


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("fix", ["hydrogen_cfg1", "si_small"])
def test_degree_one_outside_rows(fix, prec, request):
    print(f"[lowp m=1] {fix} {prec}", flush=True)
    prob = request.getfixturevalue(fix)
    ctx, ops = context(fix, prob)
    N = 37
    X = bf16_block((ops.n, N), 31)
    a, b = -1.0, 80.0
    e, c = 2.0 / (b - a), (a + b) / (b - a)
    Y = host(ctx.filter(dev(X), 1, a, b, prec=prec))
    mod = model(fix, prob, prec)
    HX = np.asarray(mod.ops.H[:prob.n_h] @ X)
    dinv = 1.0 / np.asarray(prob.M_cc_diag)
    rows = outside_rows(prob)
    assert rows.size > 0
    y_model = e * dinv[rows, None] * HX[rows] - c * X[rows]
    absHX = abs_classical_product(mod.prob, X)[rows]
    K = 128 + 8
    bound = (e * dinv[rows, None] * (K + 2) * U32 * absHX
             + 4 * U32 * (e * dinv[rows, None] * np.abs(HX[rows]) + np.abs(c * X[rows])))
    err = np.abs(Y[rows] - y_model)
    print(f"  max err/bound {float((err / bound).max()):.3e}", flush=True)
    assert np.all(err <= bound)
    if prec == "bf16":
        # the far cells' BF16 matrices are visible: the unrounded operator is further away
        assert far_cells(prob).any()
        y64 = e * dinv[rows, None] * np.asarray(ops.H[:prob.n_h] @ X)[rows] - c * X[rows]
        assert np.abs(Y[rows] - y64).max() > 10 * err.max()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("fix,m", [("tiny_enriched", 5), ("hydrogen_small", 8), ("si_small", 6),
                                   ("si_dense", 4)])
def test_filter_steps(fix, m, prec, request):
    """Every step of the reduced recurrence against the model applied to the
    device's own previous iterates (filters of degree 1..m; the FP32 state is
    exact in the FP64 output), to 10 u32 kappa(M^E) of one step.  For CF_FP32
    also the whole filter against the FP64 oracle, to 10 u32 kappa(M^E) per step."""
    print(f"[lowp filter] {fix} m={m} {prec}", flush=True)
    prob = request.getfixturevalue(fix)
    if fix == "si_dense":
        # cells with more than 64 functions: the coupling kernels' second row group
        assert np.diff(prob.enr_ptr).max() > 64
    ctx, ops = context(fix, prob)
    mod = model(fix, prob, prec)
    v0 = np.random.default_rng(5).standard_normal(ops.n)
    al, be = lanczos(ops.apply_Htilde, ops.apply_M, v0, 10)
    lo, hi = lanczos_bounds(al, be)
    a = lo + 0.05 * (hi - lo)
    e, c = 2.0 / (hi - a), (a + hi) / (hi - a)
    X = bf16_block((ops.n, 21), 32)
    Xd = dev(X)
    Ys = [X] + [host(ctx.filter(Xd, k, a, hi, prec=prec)) for k in range(1, m + 1)]
    kap = kappa_M(ops)
    for k in range(1, m + 1):
        if k == 1:
            rhs = e * mod.htilde(X) - c * X
        else:
            rhs = 2.0 * (e * mod.htilde(Ys[k - 1]) - c * Ys[k - 1]) - Ys[k - 2]
        rel = float(np.abs(Ys[k] - rhs).max() / np.abs(rhs).max())
        print(f"  step {k}: rel err {rel:.3e} tol {10 * U32 * kap:.3e}", flush=True)
        assert rel < 10 * U32 * kap, k
    if prec == "fp32":
        Yo = recurrence_filter(lambda Z: ops.apply_Htilde(Z), X, m, a, hi)
        rel = float(np.abs(Ys[m] - Yo).max() / np.abs(Yo).max())
        print(f"  whole filter: rel err {rel:.3e}", flush=True)
        assert rel < 10 * U32 * kap * m


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("fix", ["hydrogen_small", "hydrogen_cfg1"])
def test_wide_interval_high_degree(fix, prec, request):
    """Damping interval [a, b] at the top of the spectrum and m = 60: the
    unscaled iterates reach T_60(t(lambda_min)) ~ 1e130, far outside FP32's
    range.  The reduced forms keep their iterates scaled by powers of two and
    return the unscaled result: the last step against the model (as in
    test_filter_steps) and, for CF_FP32, the whole filter against the FP64
    oracle."""
    print(f"[lowp wide] {fix} {prec}", flush=True)
    prob = request.getfixturevalue(fix)
    ctx, ops = context(fix, prob)
    mod = model(fix, prob, prec)
    v0 = np.random.default_rng(5).standard_normal(ops.n)
    al, be = lanczos(ops.apply_Htilde, ops.apply_M, v0, 10)
    lo, hi = lanczos_bounds(al, be)
    a = hi - 0.02 * (hi - lo)
    e, c = 2.0 / (hi - a), (a + hi) / (hi - a)
    m = 60
    X = bf16_block((ops.n, 12), 35)
    Xd = dev(X)
    Ym2, Ym1, Ym = (host(ctx.filter(Xd, k, a, hi, prec=prec)) for k in (m - 2, m - 1, m))
    assert np.isfinite(Ym).all()
    assert np.abs(Ym).max() > 1e60
    kap = kappa_M(ops)
    rhs = 2.0 * (e * mod.htilde(Ym1) - c * Ym1) - Ym2
    rel = float(np.abs(Ym - rhs).max() / np.abs(rhs).max())
    print(f"  max |Y| {np.abs(Ym).max():.3e}; last step rel err {rel:.3e}", flush=True)
    assert rel < 10 * U32 * kap
    if prec == "fp32":
        Yo = recurrence_filter(lambda Z: ops.apply_Htilde(Z), X, m, a, hi)
        rel = float(np.abs(Ym - Yo).max() / np.abs(Yo).max())
        print(f"  whole filter rel err {rel:.3e}", flush=True)
        assert rel < 10 * U32 * kap * m


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_mixed_subspace_iteration(hydrogen_cfg1, prec):
    """Six reduced-precision passes, then three FP64 cleanup passes, from the
    atomic-orbital start (hydrogen, 8^3 cells, N = 24, m = 40, 14 wanted):
    the wanted Ritz values end within 1e-6 Ha of the discrete eigenvalues, and
    the reduced passes alone get within 1e-2 Ha."""
    import scipy.sparse.linalg as spla
    from synth import configs
    print(f"[mixed scf] hydrogen 8^3 {prec}", flush=True)
    ctx, ops = context("hydrogen_cfg1", hydrogen_cfg1, max_cols=24)
    N, m, wanted = 24, 40, 14
    lam = np.sort(spla.eigsh(ops.H, k=wanted, M=ops.M, sigma=-1.0, which="LM",
                             return_eigenvectors=False))
    v0 = np.random.default_rng(1).standard_normal(ops.n)
    _, b = ctx.lanczos_bounds(dev(v0).reshape(-1), 10)
    Xd = dev(configs.initial_block(hydrogen_cfg1, N))
    th = ctx.rayleigh_ritz(Xd)
    errs = []
    for step, p in enumerate([prec] * 6 + ["fp64"] * 3):
        Yd = ctx.filter(Xd, m, float(th[-1]), b, prec=p)
        th = ctx.rayleigh_ritz(Yd)
        Xd = Yd
        errs.append(float(np.abs(th[:wanted] - lam).max()))
        print(f"  pass {step} ({p}): ritz err {errs[-1]:.3e}", flush=True)
    assert errs[5] < 1e-2
    assert errs[-1] < 1e-6


def test_reduced_forms_deterministic(si_small):
    ctx, ops = context("si_small", si_small)
    X = dev(bf16_block((ops.n, 19), 33))
    for prec in ("fp32", "bf16"):
        a = host(ctx.filter(X, 3, -2.0, 50.0, prec=prec))
        b = host(ctx.filter(X, 3, -2.0, 50.0, prec=prec))
        assert np.array_equal(a, b)


def test_reduced_degree_zero_copies(si_small):
    ctx, ops = context("si_small", si_small)
    X = np.random.default_rng(34).standard_normal((ops.n, 5))
    for prec in ("fp32", "bf16"):
        assert np.array_equal(host(ctx.filter(dev(X), 0, -1.0, 5.0, prec=prec)), X)


def test_cell_tile_shapes_agree_and_autotune(si_small):
    """The reduced cell product's tile shape (one or two 16-column MFMA blocks
    per column tile) is a launch parameter: both shapes give bit-identical
    filters (37 columns: a ragged second block), and the autotuner returns one
    of them; with the coupling map it also tunes put back to the default, the
    results are the same bits."""
    from paper_1610_02121_amd import ChebFilterError, Context
    print("[cell tile shapes]", flush=True)
    prob = si_small
    ctx = Context(prob, max_cols=40)
    v0 = dev(np.random.default_rng(61).standard_normal(prob.n)).reshape(-1)
    lo, hi = ctx.lanczos_bounds(v0, 10)
    a, b = lo + 0.1 * (hi - lo), hi
    X = dev(np.random.default_rng(62).standard_normal((prob.n, 37)))
    for prec in ("fp32", "bf16"):
        outs = []
        for nsb in (1, 2):
            ctx.set_cell_tile(prec, nsb)
            outs.append(host(ctx.filter(X, 6, a, b, prec=prec)))
        assert np.array_equal(outs[0], outs[1]), prec
        default_map = ctx.tuning()["coupling_map"]
        ch = ctx.autotune(X, 6, a, b, prec=prec, reps=2)
        print(f"  {prec}: autotuner chose {ch} block(s) per tile, coupling map "
              f"{ctx.tuning()['coupling_map']:08b}", flush=True)
        assert ch in (1, 2)
        ctx.tuning(default_map)
        assert np.array_equal(host(ctx.filter(X, 6, a, b, prec=prec)), outs[0]), prec
    with pytest.raises(ChebFilterError, match="CF_EINVAL"):
        ctx.set_cell_tile("fp64", 1)
    with pytest.raises(ChebFilterError, match="CF_EINVAL"):
        ctx.set_cell_tile("fp32", 3)
    ctx.close()


def test_coupling_map_choices_agree_and_autotune(si_dense):
    """The FP32 coupling partials' wave split per row-block bucket (1 x 8,
    2 x 4 or 4 x 2 row blocks x k parts) changes only the order of FP32 sums:
    every map gives the filter within 10 u32 kappa(M^E) per step of the
    default map's (which test_filter_steps pins to the oracle); the autotuner
    keeps a valid map and the tuning state reports it."""
    from paper_1610_02121_amd import ChebFilterError, Context
    print("[coupling map]", flush=True)
    prob = si_dense
    ctx = Context(prob, max_cols=24)
    ops = Operators(prob)
    kap = kappa_M(ops)
    v0 = dev(np.random.default_rng(63).standard_normal(prob.n)).reshape(-1)
    lo, hi = ctx.lanczos_bounds(v0, 10)
    a, b = lo + 0.1 * (hi - lo), hi
    X = dev(bf16_block((prob.n, 21), 64))
    m = 4
    default = ctx.tuning()["coupling_map"]
    ref = host(ctx.filter(X, m, a, b, prec="fp32"))
    for cmap in (0, 0b01010101, 0b10101010, 0b00100100):
        ctx.tuning(cmap)
        Y = host(ctx.filter(X, m, a, b, prec="fp32"))
        rel = float(np.abs(Y - ref).max() / np.abs(ref).max())
        print(f"  map {cmap:08b}: rel diff {rel:.2e}", flush=True)
        assert rel < 10 * U32 * kap * m
    ctx.tuning(default)
    assert np.array_equal(host(ctx.filter(X, m, a, b, prec="fp32")), ref)
    ctx.autotune(X, m, a, b, prec="fp32", reps=1)
    cmap = ctx.tuning()["coupling_map"]
    print(f"  autotuned map {cmap:08b}", flush=True)
    assert all(((cmap >> (2 * q)) & 3) < 3 for q in range(4))
    with pytest.raises(ChebFilterError, match="CF_EINVAL"):
        ctx.tuning(0b11)
    ctx.close()
