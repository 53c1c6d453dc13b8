"""Device assembly of the cells with an adaptive rule (chebfilter_assemble_enriched,
Sec. IV.C and Eq. HBlocks) against the oracle's element blocks
(oracle/enriched.py, pinned in test_oracle_enriched.py).

The grid is the generator's: the leaf boxes its divide-and-conquer rule
accepted on each enriched cell (and, for hydrogen, on the plain cells
touching the bare nucleus).  The potential at the grid's points is the
problem's own potential with a seeded smooth relative perturbation, so it is
a new potential, not the assembled one.

Tolerance, entry by entry: the device sums the point terms in steps of four
(MFMA), the oracle with numpy's matmul.  Both are within nq u sum|terms| of
the exact sum, where nq is the cell's point count and sum|terms| is the same
sum with every factor replaced by its absolute value.  The test allows 4
nq u sum|terms|, plus 4 u |K| for H^cc.  H^ee also sums over the cells: its
bound adds the cells' bounds.  The function values themselves differ by more
than u where they are ill-conditioned: in the cutoff's tail h = exp(-1/r~)
/ (...) has relative condition ~1/r~^2, and the two sides' exp and point
coordinates differ in the last bit.  Those entries are tiny (1e-21 at the
support's edge), so the bound adds 64 u times the largest entry of that
block over the problem.  Then the operator H^E and one three-term step
of the filter on the updated context are compared with the oracle's sparse
operator built from the oracle's blocks: H~ uses the rebuilt
H^ee - M^ec D^-1 H^ec^T.
"""
import copy

import numpy as np
import pytest

from oracle.enriched import atom_functions, box_points, cell_basis, enriched_cell_blocks
from oracle.filters import recurrence_filter
from oracle.operators import Operators

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

U = 2.0 ** -53


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def gauss01(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def grid_of(prob):
    """The generator's adaptive grid as chebfilter_enriched_tables takes it."""
    from synth.basis import gll_rule
    mesh, qb = prob.meta["mesh"], prob.meta["quad_boxes"]
    bp = np.asarray(qb["box_ptr"])
    cells = np.nonzero(bp[1:] > bp[:-1])[0].astype(np.int32)
    box_ptr = np.concatenate([bp[cells], [bp[-1]]]).astype(np.int64)
    gx, gw = gauss01(qb["ng"])
    enr = prob.meta.get("enr")
    g = dict(cells=cells, cell_lo=mesh.cell_lo()[cells], h=mesh.h,
             nodes=0.5 * (gll_rule(mesh.p)[0] + 1.0), gauss_x=gx, gauss_w=gw,
             box_ptr=box_ptr, box_lo=qb["box_lo"], box_size=qb["box_size"])
    if enr is not None:
        g.update(centers=enr.centers, shells=enr.shell_terms(), r0=enr.r0, t=enr.t)
    return g


def new_potential(prob, g, seed):
    pts, _, _ = box_points(g["box_lo"], g["box_size"], g["gauss_x"], g["gauss_w"])
    V = prob.meta["potential"](pts)
    rng = np.random.default_rng(seed)
    k = rng.standard_normal(3) * 0.2
    return V * (1.0 + 0.1 * np.sin(pts @ k)) + 0.05 * rng.standard_normal(V.shape)


def oracle_blocks(prob, g, V, K):
    """Per listed cell: the oracle's blocks and the entrywise bounds."""
    ep = np.asarray(prob.enr_ptr)
    idx = np.asarray(prob.enr_idx)
    npa = len(g.get("shells", ())) and sum(2 * l + 1 for l, _ in g["shells"])
    out = []
    off = 0
    for i, e in enumerate(g["cells"]):
        b0, b1 = g["box_ptr"][i], g["box_ptr"][i + 1]
        pts, w, ng = box_points(g["box_lo"][b0:b1], g["box_size"][b0:b1], g["gauss_x"],
                                g["gauss_w"])
        Vc = V[off:off + pts.shape[0]]
        off += pts.shape[0]
        fn = idx[ep[e]:ep[e + 1]]
        atoms = list(fn[::npa] // npa) if len(fn) else []
        blk = enriched_cell_blocks(K, g["nodes"], g["cell_lo"][i], g["h"], pts, w, Vc, atoms,
                                   g.get("centers"), g.get("shells"), g.get("r0", 1.0),
                                   g.get("t", 1.0))
        N, G = cell_basis(g["nodes"], g["cell_lo"][i], g["h"], pts)
        aw, awV = np.abs(w), np.abs(w * Vc)
        bnd = {"cc": np.abs(K) + (np.abs(N) * awV[:, None]).T @ np.abs(N)}
        if atoms:
            vals, grads = zip(*(atom_functions(g["centers"][I], g["shells"], g["r0"], g["t"], pts)
                                for I in atoms))
            E, EG = np.abs(np.concatenate(vals, axis=1)), np.abs(np.concatenate(grads, axis=1))
            EGd = [np.ascontiguousarray(EG[:, :, d]) for d in range(3)]
            aG = np.abs(G)
            bnd["ec"] = (E * awV[:, None]).T @ np.abs(N) + 0.5 * sum(
                (EGd[d] * aw[:, None]).T @ aG[d] for d in range(3))
            bnd["ee"] = (E * awV[:, None]).T @ E + 0.5 * sum(
                (EGd[d] * aw[:, None]).T @ EGd[d] for d in range(3))
        out.append((e, fn, pts.shape[0], blk, bnd))
    assert off == V.size
    return out


def run_assembly(prob, ctx, seed):
    from synth.assemble import plain_tables
    B, w, K, _ = plain_tables(prob)
    ctx.assembly_tables(B, w, K)
    g = grid_of(prob)
    ctx.enriched_tables(**g)
    assert ctx.adaptive_points() == int(g["box_ptr"][-1]) * len(g["gauss_x"]) ** 3
    V = new_potential(prob, g, seed)
    print(f"[assemble_enriched] {len(g['cells'])} cells, {V.size} points, n_e = {prob.n_e}",
          flush=True)
    ctx.assemble_enriched(dev(V))
    torch.cuda.synchronize()
    Kc = 0.5 * (K + K.T)
    return g, V, oracle_blocks(prob, g, V, Kc)


def check_blocks(prob, ctx, blocks):
    cells = np.array([b[0] for b in blocks], dtype=np.int32)
    Hcc = ctx.get_H_cc(cells)
    Hec, Hee = ctx.get_coupling()
    ep = np.asarray(prob.enr_ptr)
    worst = {"cc": 0.0, "ec": 0.0, "ee": 0.0}
    Hee_o = np.zeros_like(Hee)
    Hee_b = np.zeros_like(Hee)
    fl_cc = 64 * U * max(np.abs(b[3][0]).max() for b in blocks)
    fl_ec = 64 * U * max([np.abs(b[3][1]).max() for b in blocks if len(b[1])] + [0.0])
    for i, (e, fn, nq, blk, bnd) in enumerate(blocks):
        err = np.abs(Hcc[i] - blk[0])
        lim = 4 * nq * U * bnd["cc"] + fl_cc
        assert np.all(err <= lim), f"H_cc of cell {e}: {(err / lim).max():.2f} of the bound"
        assert np.array_equal(Hcc[i], Hcc[i].T)
        worst["cc"] = max(worst["cc"], float((err / lim).max()))
        if len(fn):
            err = np.abs(Hec[ep[e]:ep[e + 1]] - blk[1])
            lim = 4 * nq * U * bnd["ec"] + fl_ec
            assert np.all(err <= lim), f"H_ec of cell {e}: {(err / lim).max():.2f} of the bound"
            worst["ec"] = max(worst["ec"], float((err / lim).max()))
            Hee_o[np.ix_(fn, fn)] += blk[3]
            Hee_b[np.ix_(fn, fn)] += 4 * nq * U * bnd["ee"]
    if prob.n_e:
        Hee_o = 0.5 * (Hee_o + Hee_o.T)
        err = np.abs(Hee - Hee_o)
        lim = Hee_b + 64 * U * np.abs(Hee_o).max()
        assert np.all(err <= lim), f"H_ee: {(err / lim).max():.2f} of the bound"
        assert np.array_equal(Hee, Hee.T)
        worst["ee"] = float((err / lim).max())
    print(f"[assemble_enriched] worst error / bound: {worst}", flush=True)
    return Hcc, Hec, Hee


def oracle_problem(prob, blocks, Hec, Hee):
    """The problem with the oracle's blocks on the listed cells (H^ec, H^ee
    from the oracle too; the device's H^ec / H^ee are only used to check
    the shapes)."""
    p2 = copy.copy(prob)
    p2.H_cc = np.array(prob.H_cc, copy=True)
    p2.H_ec = np.array(prob.H_ec, copy=True)
    ep = np.asarray(prob.enr_ptr)
    Hee_o = np.zeros((prob.n_e, prob.n_e))
    for e, fn, _, blk, _ in blocks:
        p2.H_cc[e] = blk[0]
        if len(fn):
            p2.H_ec[ep[e]:ep[e + 1]] = blk[1]
            Hee_o[np.ix_(fn, fn)] += blk[3]
    p2.H_ee = 0.5 * (Hee_o + Hee_o.T)
    assert p2.H_ec.shape == Hec.shape and p2.H_ee.shape == Hee.shape
    return p2


@pytest.mark.parametrize("fixture", ["si_dense", "hydrogen_small"])
def test_assemble_enriched_against_oracle(fixture, request):
    """Every block of every listed cell; then H^E X and a degree-3 filter step
    through the updated context against the oracle's operator from the
    oracle's blocks.  si_dense: up to 90 functions per cell (two work items
    per cell).  hydrogen: a two-term radial (2s) and plain cells with the
    adaptive rule at the nucleus."""
    from paper_1610_02121_amd import Context
    prob = request.getfixturevalue(fixture)
    N = 24
    ctx = Context(prob, max_cols=N)
    g, V, blocks = run_assembly(prob, ctx, seed=11)
    Hcc, Hec, Hee = check_blocks(prob, ctx, blocks)
    p2 = oracle_problem(prob, blocks, Hec, Hee)
    ops = Operators(p2)
    X = np.random.default_rng(3).standard_normal((prob.n, N))
    Y = ctx.apply_H(dev(X)).cpu().numpy()
    Yo = ops.apply_H(X)
    scale = np.abs(Yo).max()
    rel = np.abs(Y - Yo).max() / scale
    print(f"[assemble_enriched] {fixture}: H X rel err {rel:.2e}", flush=True)
    assert rel < 1e-11
    a, b = -1.0, 50.0
    Z = ctx.filter(dev(X), 3, a, b).cpu().numpy()
    Zo = recurrence_filter(lambda v: ops.apply_Htilde(v), X, 3, a, b)
    relf = np.abs(Z - Zo).max() / np.abs(Zo).max()
    print(f"[assemble_enriched] {fixture}: filter m=3 rel err {relf:.2e}", flush=True)
    assert relf < 1e-9


def test_assemble_enriched_reproduces_generator_blocks(si_small):
    """With the assembled potential itself, the device recomputes the
    generator's blocks (host quadrature over the same grid) to rounding."""
    from paper_1610_02121_amd import Context
    from synth.assemble import plain_tables
    prob = si_small
    ctx = Context(prob, max_cols=8)
    B, w, K, _ = plain_tables(prob)
    ctx.assembly_tables(B, w, K)
    g = grid_of(prob)
    ctx.enriched_tables(**g)
    pts, _, _ = box_points(g["box_lo"], g["box_size"], g["gauss_x"], g["gauss_w"])
    ctx.assemble_enriched(dev(prob.meta["potential"](pts)))
    Hcc = ctx.get_H_cc(g["cells"])
    Hec, Hee = ctx.get_coupling()
    H0 = np.asarray(prob.H_cc)[g["cells"]]
    for name, a, b in (("H_cc", Hcc, H0), ("H_ec", Hec, np.asarray(prob.H_ec)),
                       ("H_ee", Hee, np.asarray(prob.H_ee))):
        rel = np.abs(a - b).max() / np.abs(b).max()
        print(f"[assemble_enriched] generator's {name}: rel diff {rel:.2e}", flush=True)
        assert rel < 1e-12


def test_assemble_enriched_twice_and_reduced_copies(si_small):
    """Two assemblies in a row with different potentials leave the blocks of
    the second (H^ee is cleared, not accumulated); the FP32 filter then
    follows the new operator."""
    from paper_1610_02121_amd import Context
    prob = si_small
    N = 16
    ctx = Context(prob, max_cols=N)
    run_assembly(prob, ctx, seed=5)
    g, V, blocks = run_assembly(prob, ctx, seed=6)
    check_blocks(prob, ctx, blocks)
    X = dev(np.random.default_rng(4).standard_normal((prob.n, N)))
    Z64 = ctx.filter(X, 4, -1.0, 60.0)
    Z32 = ctx.filter(X, 4, -1.0, 60.0, prec="fp32")
    rel = float((Z32 - Z64).abs().max() / Z64.abs().max())
    print(f"[assemble_enriched] FP32 filter after assembly: rel diff {rel:.2e}", flush=True)
    assert rel < 1e-4


def test_assemble_enriched_errors(si_small):
    from paper_1610_02121_amd import ChebFilterError, Context
    from synth.assemble import plain_tables
    prob = si_small
    ctx = Context(prob, max_cols=4)
    with pytest.raises(ChebFilterError, match="no grid"):
        ctx._check(ctx.lib.chebfilter_assemble_enriched(ctx._h, None))
    g = grid_of(prob)
    with pytest.raises(ChebFilterError, match="kinetic"):
        ctx.enriched_tables(**g)
    B, w, K, _ = plain_tables(prob)
    ctx.assembly_tables(B, w, K)
    bad = dict(g)
    bad["cells"] = g["cells"][1:]
    bad["cell_lo"] = g["cell_lo"][1:]
    bad["box_ptr"] = g["box_ptr"][1:] - g["box_ptr"][1]
    bad["box_lo"] = g["box_lo"][g["box_ptr"][1]:]
    bad["box_size"] = g["box_size"][g["box_ptr"][1]:]
    with pytest.raises(ChebFilterError, match="not listed"):
        ctx.enriched_tables(**bad)
    bad = dict(g)
    bad["box_lo"] = np.array(g["box_lo"], copy=True)
    bad["box_lo"][0, 0] -= g["h"]
    with pytest.raises(ChebFilterError, match="outside its cell"):
        ctx.enriched_tables(**bad)
    bad = dict(g)
    bad["shells"] = [(2, [(1.0, 2, 1.0)])] + list(g["shells"][1:])
    with pytest.raises(ChebFilterError, match="l = 0 or 1"):
        ctx.enriched_tables(**bad)
    ctx.enriched_tables(**g)
    with pytest.raises(ValueError, match="one value per point"):
        ctx.assemble_enriched(torch.zeros(5, dtype=torch.float64, device="cuda"))
