"""Device assembly of the plain cells' blocks (chebfilter_assemble_cells)
against the oracle's quadrature sum (oracle/assembly.py, pinned in
test_oracle_assembly.py).

Tolerance, entry by entry: the device sums the nq terms in blocks of four
(MFMA) where the oracle sums them one by one; both are within
nq * u * (|K| + sum_q |w_q V_q B_qa B_qb|) of the exact sum, so the test
allows twice that.  The device block is exactly symmetric by construction.
"""
import copy

import numpy as np
import pytest

from oracle.assembly import plain_cell_block
from oracle.operators import Operators

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

U = 2.0 ** -53


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def plain_cells(prob):
    ep = np.asarray(prob.enr_ptr)
    return np.nonzero(ep[1:] == ep[:-1])[0]


def potential_at(prob, cells, seed):
    """The problem's potential at the cells' Gauss points plus a seeded smooth
    relative perturbation (a different potential than the one assembled)."""
    from synth.assemble import plain_points
    pts = plain_points(prob, cells)
    V = prob.meta["potential"](pts.reshape(-1, 3)).reshape(len(cells), -1)
    rng = np.random.default_rng(seed)
    k = rng.standard_normal(3) * 0.2
    return V * (1.0 + 0.1 * np.sin(pts @ k)) + 0.05 * rng.standard_normal(V.shape)


def check_blocks(prob, cells, V, H_dev, K, B, w):
    worst = 0.0
    for i, e in enumerate(cells):
        Ho = plain_cell_block(K, B, w, V[i])
        bound = np.abs(K) + (np.abs(B) * np.abs(w * V[i])[:, None]).T @ np.abs(B)
        err = np.abs(H_dev[i] - Ho)
        assert np.all(err <= 2.0 * len(w) * U * bound + 1e-300), e
        assert np.array_equal(H_dev[i], H_dev[i].T), e
        worst = max(worst, float((err / (bound + 1e-300)).max()))
    return worst


def test_assemble_against_oracle(si_small):
    """A ragged list of plain cells (out of order) on the 5-atom cluster; the
    other cells keep their blocks; H X through the updated operator matches
    the oracle operator built from the oracle's blocks."""
    from paper_1610_02121_amd import Context
    from synth.assemble import plain_tables
    print("[assemble si_small]", flush=True)
    prob = si_small
    B, w, K, _ = plain_tables(prob)
    ctx = Context(prob, max_cols=16)
    ctx.assembly_tables(B, w, K)
    pc = plain_cells(prob)
    cells = np.random.default_rng(1).permutation(pc)[:37]
    V = potential_at(prob, cells, seed=2)
    ctx.assemble_cells(cells, dev(V))
    H = ctx.get_H_cc(cells)
    worst = check_blocks(prob, cells, V, H, K, B, w)
    print(f"  worst error / bound {worst:.2e}", flush=True)
    others = np.setdiff1d(np.arange(prob.n_cells), cells)[::97]
    assert np.array_equal(ctx.get_H_cc(others), np.asarray(prob.H_cc)[others])
    P = copy.deepcopy(prob)
    Hn = np.array(prob.H_cc, copy=True)
    for i, e in enumerate(cells):
        Ho = plain_cell_block(K, B, w, V[i])
        Hn[e] = 0.5 * (Ho + Ho.T)
    P.H_cc = Hn
    ops = Operators(P)
    X = np.random.default_rng(3).standard_normal((ops.n, 16))
    Y = ctx.apply_H(dev(X)).cpu().numpy()
    Yo = ops.apply_H(X)
    assert np.abs(Y - Yo).max() < 1e-12 * np.abs(Yo).max()
    ctx.close()


def test_assemble_all_plain_cells_refreshes_reduced_copies(hydrogen_small):
    """Every plain cell at once (the SCF-step update); the FP32 filter of the
    context afterwards equals, bit for bit, the FP32 filter of a fresh
    context built from the device blocks (so the reduced copies follow)."""
    from paper_1610_02121_amd import Context
    from synth.assemble import plain_tables
    print("[assemble all plain cells]", flush=True)
    prob = hydrogen_small
    B, w, K, _ = plain_tables(prob)
    ctx = Context(prob, max_cols=8)
    X = dev(np.random.default_rng(4).standard_normal((prob.n, 8)))
    ctx.filter(X, 4, -1.0, 50.0, prec="fp32")      # reduced copies exist before the update
    ctx.assembly_tables(B, w, K)
    cells = plain_cells(prob)
    V = potential_at(prob, cells, seed=5)
    ctx.assemble_cells(cells, dev(V))
    H_all = ctx.get_H_cc(np.arange(prob.n_cells))
    check_blocks(prob, cells[::7], V[::7], H_all[cells[::7]], K, B, w)
    P = copy.deepcopy(prob)
    P.H_cc = H_all
    fresh = Context(P, max_cols=8)
    for prec in ("fp64", "fp32"):
        Ya = ctx.filter(X, 6, -1.0, 50.0, prec=prec)
        Yb = fresh.filter(X, 6, -1.0, 50.0, prec=prec)
        torch.cuda.synchronize()
        assert torch.equal(Ya, Yb), prec
    ctx.close()
    fresh.close()


def test_assemble_errors(hydrogen_small):
    from paper_1610_02121_amd import ChebFilterError, Context
    from synth.assemble import plain_tables
    prob = hydrogen_small
    B, w, K, _ = plain_tables(prob)
    ctx = Context(prob, max_cols=4)
    V = dev(np.zeros((2, len(w))))
    pc = plain_cells(prob)
    with pytest.raises(ChebFilterError, match="CF_EINVAL.*tables"):
        ctx.assemble_cells(pc[:2], V)
    ctx.assembly_tables(B, w, K)
    ep = np.asarray(prob.enr_ptr)
    enriched = np.nonzero(ep[1:] > ep[:-1])[0]
    with pytest.raises(ChebFilterError, match="CF_EINVAL.*enrichment"):
        ctx.assemble_cells(np.array([pc[0], enriched[0]]), V)
    with pytest.raises(ChebFilterError, match="CF_EINVAL.*twice"):
        ctx.assemble_cells(np.array([pc[0], pc[0]]), V)
    with pytest.raises(ChebFilterError, match="CF_EINVAL.*range"):
        ctx.assemble_cells(np.array([pc[0], prob.n_cells]), V)
    Kbad = K.copy()
    Kbad[0, 1] += 1.0
    with pytest.raises(ChebFilterError, match="CF_EINVAL.*symmetric"):
        ctx.assembly_tables(B, w, Kbad)
    ctx.assemble_cells(pc[:0], V[:0])                 # empty list: nothing to do
    ctx.close()
