"""Batches of independent problems (chebfilter_*_batch) against the
single-problem entry points and the oracle.

The batched reduced-precision filter runs every entry through the same device
bodies as the single-problem kernels, in merged launches; its result must be
bit for bit the single-problem result of the same precision (which
test_gpu_lowp pins to the oracle).  One entry is also checked against the FP64
oracle directly, with the FP32 bound of test_gpu_lowp (10 u32 kappa(M^E) per
step).  The batch mixes problems, repeats problems (shared operator, separate
blocks), column counts and intervals.
"""
import numpy as np
import pytest

from oracle.filters import recurrence_filter
from oracle.operators import Operators

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

U32 = 2.0 ** -24
MAXC = 40


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


_STATE = {}


def state(tiny_enriched, hydrogen_small, si_small):
    """(batch, entry problems, single contexts by problem id, N, intervals)."""
    if "b" not in _STATE:
        from paper_1610_02121_amd import Batch, Context
        probs = [tiny_enriched, hydrogen_small, si_small, hydrogen_small, tiny_enriched, si_small,
                 hydrogen_small]
        Ns = [5, 16, 37, 1, 7, 40, 23]
        singles = {}
        for p in probs:
            if id(p) not in singles:
                singles[id(p)] = Context(p, max_cols=MAXC)
        batch = Batch(probs, max_cols=MAXC)
        # per-entry damping interval from the entry's Lanczos bound
        v0 = [dev(np.random.default_rng(40 + i).standard_normal(p.n)).reshape(-1)
              for i, p in enumerate(probs)]
        lo, hi = batch.lanczos_bounds(v0, 10)
        ab = [(l + (0.05 + 0.05 * i) * (h - l), h) for i, (l, h) in enumerate(zip(lo, hi))]
        _STATE.update(b=batch, probs=probs, singles=singles, Ns=Ns, ab=ab, v0=v0)
    s = _STATE
    return s["b"], s["probs"], s["singles"], s["Ns"], s["ab"]


def blocks(probs, Ns, seed):
    return [np.random.default_rng(seed + i).standard_normal((p.n, N))
            for i, (p, N) in enumerate(zip(probs, Ns))]


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_filter_equals_single(prec, use_graph, tiny_enriched, hydrogen_small, si_small):
    print(f"[batch filter] {prec} graph={use_graph}", flush=True)
    batch, probs, singles, Ns, ab = state(tiny_enriched, hydrogen_small, si_small)
    m = 9
    Xs = blocks(probs, Ns, 50)
    Xd = [dev(x) for x in Xs]
    Yb = batch.filter(Xd, m, [a for a, _ in ab], [b for _, b in ab], prec=prec, use_graph=use_graph)
    Yb = [host(y) for y in Yb]
    for i, p in enumerate(probs):
        a, b = ab[i]
        Ys = host(singles[id(p)].filter(Xd[i], m, a, b, prec=prec))
        assert np.isfinite(Yb[i]).all()
        assert np.array_equal(Yb[i], Ys), i


def test_batch_graph_replays(tiny_enriched, hydrogen_small, si_small):
    """One captured graph replayed with new blocks and intervals, eager work
    and synchronisations between the replays; every replay checked."""
    print("[batch graph replays]", flush=True)
    batch, probs, singles, Ns, ab = state(tiny_enriched, hydrogen_small, si_small)
    m = 12
    for r in range(3):
        Xs = blocks(probs, Ns, 60 + 10 * r)
        Xd = [dev(x) for x in Xs]
        shift = 0.03 * r
        a = [lo + shift * (hi - lo) for lo, hi in ab]
        b = [hi for _, hi in ab]
        Yb = batch.filter(Xd, m, a, b, prec="fp32", use_graph=True)
        junk = torch.randn(1000, 100, device="cuda", dtype=torch.float64).sum()   # eager work
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        for i, p in enumerate(probs):
            Ys = host(singles[id(p)].filter(Xd[i], m, a[i], b[i], prec="fp32"))
            assert np.array_equal(host(Yb[i]), Ys), (r, i)


def test_batch_entry_against_oracle(tiny_enriched, hydrogen_small, si_small):
    print("[batch vs oracle]", flush=True)
    import scipy.sparse.linalg as spla
    batch, probs, singles, Ns, ab = state(tiny_enriched, hydrogen_small, si_small)
    m = 6
    Xs = blocks(probs, Ns, 70)
    Yb = batch.filter([dev(x) for x in Xs], m, [a for a, _ in ab], [b for _, b in ab], prec="fp32")
    i = 2                                   # si_small entry, N = 37
    ops = Operators(probs[i])
    a, b = ab[i]
    Yo = recurrence_filter(lambda Z: ops.apply_Htilde(Z), Xs[i], m, a, b)
    lmax = spla.eigsh(ops.M, k=1, which="LA", return_eigenvectors=False)[0]
    lmin = spla.eigsh(ops.M, k=1, sigma=0, which="LM", return_eigenvectors=False)[0]
    rel = float(np.abs(host(Yb[i]) - Yo).max() / np.abs(Yo).max())
    print(f"  rel err {rel:.3e}", flush=True)
    assert rel < 10 * U32 * (lmax / lmin) * m


def same_subspace_result(Yb, Ys, th_b, th_s):
    """Ritz values within 1e-12 relative and Ritz vectors equal column by
    column up to sign (the batched eigensolver may order its rounding
    differently from the single one)."""
    assert np.abs(th_b - th_s).max() <= 1e-12 * max(1.0, np.abs(th_s).max())
    sgn = np.sign(np.einsum("ij,ij->j", Yb, Ys))
    err = np.abs(Yb * sgn[None, :] - Ys).max() / np.abs(Ys).max()
    return float(err)


def test_batch_fp64_and_rayleigh_ritz(tiny_enriched, hydrogen_small, si_small):
    """The FP64 batch filter of every entry equals the single-problem entry
    point bit for bit; the batched projection (no host waits, one eigensolve
    per block width) and the grouped Lanczos runs match the single-problem
    ones to rounding."""
    print("[batch fp64 + rr]", flush=True)
    batch, probs, singles, Ns, ab = state(tiny_enriched, hydrogen_small, si_small)
    m = 5
    Xs = blocks(probs, Ns, 80)
    Xd = [dev(x) for x in Xs]
    Yb = batch.filter(Xd, m, [a for a, _ in ab], [b for _, b in ab], prec="fp64")
    Ycopy = [y.clone() for y in Yb]
    th_b = batch.rayleigh_ritz(Yb)
    for i, p in enumerate(probs):
        a, b = ab[i]
        Ys = singles[id(p)].filter(Xd[i], m, a, b, prec="fp64")
        assert np.array_equal(host(Ycopy[i]), host(Ys)), i
        th_s = singles[id(p)].rayleigh_ritz(Ys)
        err = same_subspace_result(host(Yb[i]), host(Ys), th_b[i], th_s)
        print(f"  entry {i}: N={Ns[i]} vectors rel diff {err:.2e} "
              f"bitwise={np.array_equal(host(Yb[i]), host(Ys))}", flush=True)
        assert err < 1e-10, i
    # Lanczos runs of entries sharing a problem go as the columns of one block
    # (column-wise dot products in another summation order): the bounds agree
    # with the single-vector runs to rounding, amplified at most mildly by 10 steps
    lo_b, hi_b = batch.lanczos_bounds(_STATE["v0"], 10)
    for i, p in enumerate(probs):
        lo_s, hi_s = singles[id(p)].lanczos_bounds(_STATE["v0"][i], 10)
        scale = max(abs(lo_s), abs(hi_s))
        print(f"  lanczos entry {i}: {abs(lo_b[i] - lo_s) / scale:.1e} {abs(hi_b[i] - hi_s) / scale:.1e}")
        assert abs(lo_b[i] - lo_s) <= 1e-10 * scale and abs(hi_b[i] - hi_s) <= 1e-10 * scale, i


def test_batch_rayleigh_ritz_redo_and_failure(tiny_enriched, hydrogen_small, si_small):
    """An entry whose block is nearly rank deficient (one column a 1e-12
    perturbation of another) takes the shifted path of the single-problem
    projection and gives its result; an entry with a zero column fails with
    CF_ENOTSPD naming the entry and leaves that block as it was."""
    from paper_1610_02121_amd import ChebFilterError
    print("[batch rr redo]", flush=True)
    batch, probs, singles, Ns, ab = state(tiny_enriched, hydrogen_small, si_small)
    Xs = blocks(probs, Ns, 90)
    k = 2                                   # si_small, 37 columns
    Xs[k][:, 5] = Xs[k][:, 4] * (1.0 + 1e-12 * np.random.default_rng(5).standard_normal(probs[k].n))
    Yb = [dev(x) for x in Xs]
    th_b = batch.rayleigh_ritz(Yb)
    for i, p in enumerate(probs):
        Ys = dev(Xs[i])
        th_s = singles[id(p)].rayleigh_ritz(Ys)
        err = same_subspace_result(host(Yb[i]), host(Ys), th_b[i], th_s)
        assert err < 1e-10, i
    Xs[4][:, 2] = 0.0                       # tiny_enriched, 7 columns
    Yb = [dev(x) for x in Xs]
    with pytest.raises(ChebFilterError, match="CF_ENOTSPD.*entry 4"):
        batch.rayleigh_ritz(Yb)
    assert np.array_equal(host(Yb[4]), Xs[4])


def test_batch_autotune_keeps_results(tiny_enriched, hydrogen_small, si_small):
    """The batched autotuner (tile shape of the batched reduced cell product,
    graph rebuilt on a change) returns one of the two shapes, and the batched
    BF16 filter after it (with the coupling map it also tunes put back)
    equals the one before it bit for bit."""
    print("[batch autotune]", flush=True)
    batch, probs, singles, Ns, ab = state(tiny_enriched, hydrogen_small, si_small)
    m = 4
    Xd = [dev(x) for x in blocks(probs, Ns, 95)]
    a, b = [x for x, _ in ab], [y for _, y in ab]
    before = [host(y) for y in batch.filter(Xd, m, a, b, prec="bf16")]
    default_map = batch.tuning()["coupling_map"]
    ch = batch.autotune(Xd, m, a, b, prec="bf16", reps=1)
    print(f"  autotuner chose {ch} block(s) per tile, coupling map "
          f"{batch.tuning()['coupling_map']:08b}", flush=True)
    assert ch in (1, 2)
    batch.tuning(default_map)
    after = [host(y) for y in batch.filter(Xd, m, a, b, prec="bf16")]
    for i in range(len(probs)):
        assert np.array_equal(before[i], after[i]), i


def test_batch_errors(tiny_enriched, hydrogen_small, si_small):
    from paper_1610_02121_amd import ChebFilterError
    batch, probs, singles, Ns, ab = state(tiny_enriched, hydrogen_small, si_small)
    Xd = [dev(np.ones((p.n, 3))) for p in probs]
    a = [x for x, _ in ab]
    b = [y for _, y in ab]
    with pytest.raises(ChebFilterError, match="CF_EINVAL"):
        batch.filter(Xd, 3, b, a, prec="fp32")                     # a > b
    with pytest.raises(ChebFilterError, match="CF_EINVAL"):
        batch.filter(Xd, -1, a, b, prec="fp32")
    with pytest.raises(ChebFilterError, match="CF_EINVAL"):
        batch.filter(Xd, 3, a, b, prec=9)
    big = [dev(np.ones((p.n, MAXC + 1))) for p in probs]
    with pytest.raises(ChebFilterError, match="CF_ENOMEM"):
        batch.filter(big, 3, a, b, prec="fp32")
    with pytest.raises(ValueError):
        batch.filter(Xd[:-1], 3, a, b, prec="fp32")


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_batch_dense_cells_equal_single(prec, si_dense, si_small):
    """Cells with up to 90 enrichment functions (two 64-row groups of the
    batched coupling bodies): batched filter = single-problem filter, bit for
    bit (the single path is pinned to the oracle on the same problem)."""
    from paper_1610_02121_amd import Batch, Context
    print(f"[batch dense] {prec}", flush=True)
    assert np.diff(si_dense.enr_ptr).max() > 64
    probs = [si_dense, si_small, si_dense]
    Ns = [24, 9, 17]
    batch = Batch(probs, max_cols=24)
    singles = {id(p): Context(p, max_cols=24) for p in probs}
    ab = [(-40.0, 400.0), (-35.0, 300.0), (-20.0, 420.0)]
    Xd = [dev(x) for x in blocks(probs, Ns, 70)]
    Yb = batch.filter(Xd, 5, [a for a, _ in ab], [b for _, b in ab], prec=prec)
    for i, p in enumerate(probs):
        Ys = host(singles[id(p)].filter(Xd[i], 5, ab[i][0], ab[i][1], prec=prec))
        assert np.array_equal(host(Yb[i]), Ys), i


def test_batch_coupling_map_equals_single(si_dense, si_small):
    """With the same coupling map set on the batch and on the single
    contexts, the batched FP32 filter equals the single-problem one bit for
    bit; the batch autotuner keeps a valid map."""
    from paper_1610_02121_amd import Batch, Context
    print("[batch coupling map]", flush=True)
    probs = [si_dense, si_small]
    Ns = [20, 12]
    batch = Batch(probs, max_cols=20)
    singles = [Context(p, max_cols=20) for p in probs]
    ab = [(-40.0, 400.0), (-35.0, 300.0)]
    Xd = [dev(x) for x in blocks(probs, Ns, 90)]
    cmap = 0b01010101                    # 2 row blocks x 4 k parts in every bucket
    batch.tuning(cmap)
    for c in singles:
        c.tuning(cmap)
    Yb = batch.filter(Xd, 5, [a for a, _ in ab], [b for _, b in ab], prec="fp32")
    for i, c in enumerate(singles):
        assert np.array_equal(host(Yb[i]), host(c.filter(Xd[i], 5, ab[i][0], ab[i][1], prec="fp32")))
    batch.autotune(Xd, 5, [a for a, _ in ab], [b for _, b in ab], prec="fp32", reps=1)
    got = batch.tuning()["coupling_map"]
    assert all(((got >> (2 * q)) & 3) < 3 for q in range(4))
