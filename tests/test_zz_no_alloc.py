"""The Lanczos bound on the library's fixed device scratch
(chebfilter_lanczos_bounds_noalloc) against the entry point that uses the
context's work blocks: the same kernels in the same order, so the bounds
agree bit for bit; two calls in a row, the second on a smaller problem (the
scratch keeps the first call's contents), then the first problem again, and
a problem too large for the scratch is refused with CF_ENOMEM."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def test_noalloc_lanczos_equals_context_lanczos(si_small, hydrogen_small):
    from paper_1610_02121_amd import Context
    print("[noalloc] si_small k=10, hydrogen_small k=6, si_small k=10", flush=True)
    big = Context(si_small, max_cols=8)
    small = Context(hydrogen_small, max_cols=8)
    assert small.n < big.n
    vb = dev(np.random.default_rng(71).standard_normal(big.n))
    vs = dev(np.random.default_rng(72).standard_normal(small.n))
    for ctx, v, k in ((big, vb, 10), (small, vs, 6), (big, vb, 10)):
        ref = ctx.lanczos_bounds(v, k)
        got = ctx.lanczos_bounds_noalloc(v, k)
        print(f"  n={ctx.n} k={k}: context {ref} fixed scratch {got}", flush=True)
        assert got == ref
    big.close()
    small.close()


def test_noalloc_refuses_problems_beyond_the_scratch():
    """A classical box with 1.7 M free DOFs needs 5 n doubles > 64 MiB."""
    from paper_1610_02121_amd import ChebFilterError, Context
    from synth import configs
    print("[noalloc] too large", flush=True)
    prob = configs.box(nc=120, length=2.0, p=1)
    assert 5 * prob.n * 8 > 64 * 2 ** 20
    ctx = Context(prob, max_cols=1)
    v = dev(np.ones(prob.n))
    with pytest.raises(ChebFilterError, match="CF_ENOMEM"):
        ctx.lanczos_bounds_noalloc(v, 4)
    lo, hi = ctx.lanczos_bounds(v, 4)
    assert np.isfinite(lo) and np.isfinite(hi)
    ctx.close()
