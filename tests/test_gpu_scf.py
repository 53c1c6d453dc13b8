"""The self-consistent field quantities on the device (chebfilter_scf_*)
against the oracle (oracle/scf.py, oracle/enriched.py, oracle/assembly.py,
pinned in test_oracle_scf.py and test_oracle_enriched.py).

The oracle builds the SCF points on its own side: the plain rule on the
plain cells in cell order, then the generator's leaf boxes with the Gauss
rule.  The device's coordinates and weights are compared with them.  Every
oracle field is computed from the oracle's points.

Tolerances:
* Density: the device forms D_e = Y diag(2f) Y^T and then Phi^T D_e Phi;
  the oracle forms (Phi Y) and squares.  The two differ by at most
  (K + N) u sum_j 2 f_j (sum_k |Phi_k Y_kj|)^2 at a point, K being the
  cell's basis size.  The test allows 4 times that.
* LDA: elementwise within 1e-13 relative (cbrt and log in the last bit).
* Poisson: the device CG stops at relative residual 1e-12 and the oracle
  solves directly.  V_H then agrees to ~cond(A) 1e-12, and the test allows
  1e-8 of max |V_eff|.
* Anderson: the same history through both sides, 1e-10 relative (the
  small linear system is solved by different eliminations).
* Whole SCF: the device iteration (Chebyshev-filtered subspace steps to
  convergence for every potential) and the oracle iteration (dense
  generalized eigensolve) from the same start agree on the eigenvalues and
  the energy terms after each of 6 steps, to 1e-8.
"""
import numpy as np
import pytest

from oracle.assembly import plain_cell_block
from oracle.enriched import atom_functions, box_points, cell_basis, enriched_cell_blocks
from oracle.scf import (anderson, density_at_points, fermi_level, gaussian_charge,
                        laplace_matrix, lda_xc, poisson_solve)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

U = 2.0 ** -53
KT = 0.01


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def gauss01(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


class Setup:
    """The problem's grid, the oracle's SCF points and a device context set up
    for the SCF entry points."""

    def __init__(self, prob, N, comp_width=1.5, mix_depth=3, mix_beta=0.6):
        from paper_1610_02121_amd import Context
        from synth.assemble import plain_tables
        from synth.basis import gll_rule
        from synth.quad import unit_cube_rule
        self.prob = prob
        mesh, qb = prob.meta["mesh"], prob.meta["quad_boxes"]
        self.mesh = mesh
        self.enr = prob.meta.get("enr")
        bp = np.asarray(qb["box_ptr"])
        self.acells = np.nonzero(bp[1:] > bp[:-1])[0].astype(np.int32)
        listed = np.zeros(mesh.n_cells, dtype=bool)
        listed[self.acells] = True
        self.pcells = np.nonzero(~listed)[0]
        self.gx, self.gw = gauss01(qb["ng"])
        self.nodes = 0.5 * (gll_rule(mesh.p)[0] + 1.0)
        B, w, K, ref = plain_tables(prob)
        self.B, self.wq, self.K, self.ref = B, w, 0.5 * (K + K.T), ref
        self.box_ptr = np.concatenate([bp[self.acells], [bp[-1]]])
        self.box_lo, self.box_size = qb["box_lo"], qb["box_size"]
        # oracle points: plain cells (cell order), then the adaptive grid
        lo = mesh.cell_lo()
        pts, wts, self.ranges = [], [], []
        off = 0
        for e in self.pcells:
            pts.append(lo[e] + mesh.h * ref)
            wts.append(w)
            self.ranges.append((e, off, len(w), None))
            off += len(w)
        for i, e in enumerate(self.acells):
            b0, b1 = self.box_ptr[i], self.box_ptr[i + 1]
            p, ww, _ = box_points(self.box_lo[b0:b1], self.box_size[b0:b1], self.gx, self.gw)
            pts.append(p)
            wts.append(ww)
            self.ranges.append((e, off, len(ww), i))
            off += len(ww)
        self.xyz = np.concatenate(pts)
        self.w = np.concatenate(wts)
        self.center = np.asarray(self.enr.centers).mean(axis=0) if self.enr is not None else np.zeros(3)
        self.comp_width = comp_width
        self.ctx = Context(prob, max_cols=N)
        self.ctx.assembly_tables(B, w, K)
        g = dict(cells=self.acells, cell_lo=lo[self.acells], h=mesh.h, nodes=self.nodes,
                 gauss_x=self.gx, gauss_w=self.gw, box_ptr=self.box_ptr, box_lo=self.box_lo,
                 box_size=self.box_size)
        if self.enr is not None:
            g.update(centers=self.enr.centers, shells=self.enr.shell_terms(), r0=self.enr.r0,
                     t=self.enr.t)
        self.ctx.enriched_tables(**g)
        self.ctx.scf_setup(lo, ref, self.center, comp_width, cg_max_iter=5000, cg_tol=1e-12,
                           mix_depth=mix_depth, mix_beta=mix_beta)
        self.mix_depth, self.mix_beta = mix_depth, mix_beta
        self.vext = prob.meta["potential"](self.xyz)
        ep, idx = np.asarray(prob.enr_ptr), np.asarray(prob.enr_idx)
        self.fn = [idx[ep[e]:ep[e + 1]] for e, _, _, _ in self.ranges]
        self._basis = {}

    def basis(self, k):
        """(N [Q, npc], E [Q, na] or None) at the points of SCF cell k (cached)."""
        if k not in self._basis:
            e, off, cnt, _ = self.ranges[k]
            pts = self.xyz[off:off + cnt]
            N, _ = cell_basis(self.nodes, self.mesh.cell_lo()[e], self.mesh.h, pts)
            E = None
            if len(self.fn[k]):
                npa = sum(2 * l + 1 for l, _ in self.enr.shell_terms())
                atoms = self.fn[k][::npa] // npa
                E = np.concatenate([atom_functions(self.enr.centers[I], self.enr.shell_terms(),
                                                   self.enr.r0, self.enr.t, pts)[0]
                                    for I in atoms], axis=1)
            self._basis[k] = (N, E)
        return self._basis[k]

    def rows(self, k, X):
        e = self.ranges[k][0]
        dofs = np.asarray(self.prob.cell_dof[e])
        Yc = np.where(dofs[:, None] >= 0, X[np.maximum(dofs, 0)], 0.0)
        if len(self.fn[k]):
            return np.concatenate([Yc, X[self.prob.n_h + self.fn[k]]])
        return Yc

    def density(self, X, f):
        """Oracle density at every point, and its bound for the device's form."""
        rho = np.zeros(len(self.w))
        bnd = np.zeros(len(self.w))
        for k, (e, off, cnt, _) in enumerate(self.ranges):
            N, E = self.basis(k)
            Phi = N if E is None else np.concatenate([N, E], axis=1)
            Y = self.rows(k, X)
            rho[off:off + cnt] = density_at_points(Phi, Y, f)
            Kb = 128 + (0 if E is None else ((E.shape[1] + 15) // 16) * 16)
            a = np.abs(Phi) @ np.abs(Y)
            bnd[off:off + cnt] = (Kb + X.shape[1]) * U * (2 * (a * a) @ f)
        return rho, bnd

    def potential(self, rho):
        """Oracle V_eff and terms for the density rho at the points."""
        eps, vxc = lda_xc(rho)
        Q = float(self.w @ rho)
        rg, vg = gaussian_charge(self.xyz, Q, self.center, self.comp_width)
        prob = self.prob
        b = np.zeros(prob.n_h)
        for k, (e, off, cnt, _) in enumerate(self.ranges):
            N, _ = self.basis(k)
            be = N.T @ (self.w[off:off + cnt] * (rho[off:off + cnt] - rg[off:off + cnt]))
            dofs = np.asarray(prob.cell_dof[e])
            m = dofs >= 0
            np.add.at(b, dofs[m], be[m])
        A = laplace_matrix(prob.cell_dof, self.K, prob.n_h)
        phi = poisson_solve(A, b)
        vh = np.empty_like(rho)
        for k, (e, off, cnt, _) in enumerate(self.ranges):
            N, _ = self.basis(k)
            dofs = np.asarray(prob.cell_dof[e])
            ph = np.where(dofs >= 0, phi[np.maximum(dofs, 0)], 0.0)
            vh[off:off + cnt] = N @ ph
        vh += vg
        veff = self.vext + vh + vxc
        terms = {"charge": Q, "E_xc": float(self.w @ (rho * eps)),
                 "int_rho_vxc": float(self.w @ (rho * vxc)),
                 "half_int_rho_vh": 0.5 * float(self.w @ (rho * vh))}
        return veff, terms

    def hamiltonian(self, veff):
        """The problem with the oracle's blocks for V_eff at the points."""
        import copy
        prob = self.prob
        p2 = copy.copy(prob)
        p2.H_cc = np.array(prob.H_cc, copy=True)
        p2.H_ec = np.array(prob.H_ec, copy=True)
        ep = np.asarray(prob.enr_ptr)
        Hee = np.zeros((prob.n_e, prob.n_e))
        for k, (e, off, cnt, slot) in enumerate(self.ranges):
            V = veff[off:off + cnt]
            if slot is None:
                p2.H_cc[e] = plain_cell_block(self.K, self.B, self.wq, V)
                continue
            b0, b1 = self.box_ptr[slot], self.box_ptr[slot + 1]
            pts, ww, _ = box_points(self.box_lo[b0:b1], self.box_size[b0:b1], self.gx, self.gw)
            npa = sum(2 * l + 1 for l, _ in self.enr.shell_terms()) if self.enr else 1
            atoms = list(self.fn[k][::npa] // npa) if len(self.fn[k]) else []
            blk = enriched_cell_blocks(self.K, self.nodes, self.mesh.cell_lo()[e], self.mesh.h, pts,
                                       ww, V, atoms, self.enr.centers if self.enr else None,
                                       self.enr.shell_terms() if self.enr else None,
                                       self.enr.r0 if self.enr else 1.0,
                                       self.enr.t if self.enr else 1.0)
            p2.H_cc[e] = blk[0]
            if len(self.fn[k]):
                p2.H_ec[ep[e]:ep[e + 1]] = blk[1]
                Hee[np.ix_(self.fn[k], self.fn[k])] += blk[3]
        p2.H_ee = 0.5 * (Hee + Hee.T)
        return p2


def test_scf_points_density_potential_mixing(hydrogen_small, si_small):
    """One pass of every SCF piece on two problems against the oracle."""
    for prob, ne in ((hydrogen_small, 1.0), (si_small, 70.0)):
        N = 40
        s = Setup(prob, N)
        ctx = s.ctx
        xyz, w = ctx.scf_geometry()
        assert xyz.shape == s.xyz.shape
        assert np.abs(xyz - s.xyz).max() <= 4 * U * np.abs(s.xyz).max()
        assert np.abs(w - s.w).max() <= 4 * U * np.abs(s.w).max()
        rng = np.random.default_rng(7)
        X = rng.standard_normal((prob.n, N)) * 0.05
        f = rng.uniform(0.0, 1.0, N)
        rho_d = ctx.scf_density(dev(X), f).cpu().numpy()
        rho_o, bnd = s.density(X, f)
        err = np.abs(rho_d - rho_o)
        print(f"[scf] n={prob.n} points={len(w)}: density worst {float((err / (4 * bnd + 1e-300)).max()):.3f}"
              f" of the bound", flush=True)
        assert np.all(err <= 4 * bnd + 1e-300)
        veff_d, terms_d, it = ctx.scf_potential(dev(rho_o), dev(s.vext))
        veff_o, terms_o = s.potential(rho_o)
        rel = np.abs(veff_d.cpu().numpy() - veff_o).max() / np.abs(veff_o).max()
        print(f"[scf] V_eff rel err {rel:.2e} after {it} CG iterations; terms {terms_d}", flush=True)
        assert rel < 1e-8
        for k, v in terms_o.items():
            assert terms_d[k] == pytest.approx(v, rel=1e-9, abs=1e-12), k
        # three mixing calls, history depth 3
        ins = [rng.uniform(0.0, 1.0, len(w)) for _ in range(3)]
        outs = [x + 0.1 * rng.standard_normal(len(w)) for x in ins]
        for k in range(3):
            nxt, r = ctx.scf_mix(dev(ins[k]), dev(outs[k]))
            ref = anderson(ins[:k + 1], outs[:k + 1], s.w, s.mix_beta)
            d = np.abs(nxt.cpu().numpy() - ref).max() / np.abs(ref).max()
            assert d < 1e-10, (k, d)
            assert r == pytest.approx(np.sqrt(s.w @ (outs[k] - ins[k]) ** 2), rel=1e-12)
        ctx.close()


def gpu_eigs(ctx, X, theta, v0, steps=40, m=12):
    """Chebyshev-filtered subspace iteration until the Ritz values settle."""
    _, b = ctx.lanczos_bounds(v0, 10)
    for _ in range(steps):
        Y = ctx.filter(X, m, float(theta[-1]), b)
        th = ctx.rayleigh_ritz(Y)
        X = Y
        if np.abs(th - theta).max() < 1e-13 * max(1.0, np.abs(th).max()):
            theta = th
            break
        theta = th
    return X, theta


def test_scf_iteration_against_oracle(tiny_enriched):
    """Six SCF steps of hydrogen (one electron, LDA) on the 2^3-cell degree-2
    mesh, device against oracle from the same start."""
    import scipy.linalg as sla
    from oracle.operators import Operators
    prob = tiny_enriched
    N = 8
    s = Setup(prob, N, comp_width=0.8, mix_depth=3, mix_beta=0.5)
    ctx = s.ctx
    # start: the generator's Hamiltonian (V_ext only), lowest N states
    Hd, Md = Operators(prob).dense()
    th0, V0 = sla.eigh(Hd, Md)
    X0 = V0[:, :N]
    f0, _ = fermi_level(th0[:N], 1.0, KT)
    rho_in_o, _ = s.density(X0, f0)
    rho_in_d = dev(rho_in_o)
    X = dev(X0)
    theta = th0[:N].copy()
    v0 = dev(np.random.default_rng(3).standard_normal(prob.n)).reshape(-1)
    hist_in, hist_out = [], []
    for step in range(6):
        # device: potential, blocks, eigenpairs, occupations, density, mixing
        veff_d, terms_d, _ = ctx.scf_potential(rho_in_d, dev(s.vext))
        ctx.scf_assemble(veff_d)
        X, theta = gpu_eigs(ctx, X, theta, v0)
        from paper_1610_02121_amd import fermi_level as lib_fermi
        f_d, mu_d = lib_fermi(theta, 1.0, KT)
        rho_out_d = ctx.scf_density(X, f_d)
        nxt_d, res_d = ctx.scf_mix(rho_in_d, rho_out_d)
        # oracle: the same step
        veff_o, terms_o = s.potential(rho_in_o)
        p2 = s.hamiltonian(veff_o)
        Ho, Mo = Operators(p2).dense()
        tho, Vo = sla.eigh(Ho, Mo)
        fo, _ = fermi_level(tho[:N], 1.0, KT)
        rho_out_o, _ = s.density(Vo[:, :N], fo)
        hist_in.append(rho_in_o)
        hist_out.append(rho_out_o)
        nxt_o = anderson(hist_in[-3:], hist_out[-3:], s.w, s.mix_beta)
        res_o = float(np.sqrt(s.w @ (rho_out_o - rho_in_o) ** 2))
        e_err = np.abs(theta - tho[:N]).max()
        print(f"[scf] step {step}: eigenvalue diff {e_err:.2e}, residual {res_d:.3e} / {res_o:.3e}, "
              f"E_xc {terms_d['E_xc']:.10f} / {terms_o['E_xc']:.10f}", flush=True)
        assert e_err < 1e-8
        assert res_d == pytest.approx(res_o, rel=1e-6, abs=1e-10)
        for k, v in terms_o.items():
            assert terms_d[k] == pytest.approx(v, rel=1e-8, abs=1e-10), k
        rho_in_o = nxt_o
        rho_in_d = nxt_d
        assert np.abs(nxt_d.cpu().numpy() - nxt_o).max() < 1e-7 * np.abs(nxt_o).max()
    ctx.close()


def test_scf_converges_on_hydrogen(hydrogen_small):
    """The device SCF loop on the 4^3-cell hydrogen problem: the density
    residual falls below 1e-7 within 20 steps."""
    prob = hydrogen_small
    N = 8
    s = Setup(prob, N, comp_width=1.5, mix_depth=4, mix_beta=0.6)
    ctx = s.ctx
    from paper_1610_02121_amd import fermi_level as lib_fermi
    from synth import configs
    X = dev(configs.initial_block(prob, N))
    theta = ctx.rayleigh_ritz(X)
    v0 = dev(np.random.default_rng(3).standard_normal(prob.n)).reshape(-1)
    X, theta = gpu_eigs(ctx, X, theta, v0)
    f, _ = lib_fermi(theta, 1.0, KT)
    rho_in = ctx.scf_density(X, f)
    vext = dev(s.vext)
    res = []
    for step in range(20):
        veff, terms, it = ctx.scf_potential(rho_in, vext)
        ctx.scf_assemble(veff)
        X, theta = gpu_eigs(ctx, X, theta, v0)
        f, mu = lib_fermi(theta, 1.0, KT)
        rho_out = ctx.scf_density(X, f)
        rho_in, r = ctx.scf_mix(rho_in, rho_out)
        res.append(r)
        e_tot = 2 * float(f @ theta) + terms["E_xc"] - terms["int_rho_vxc"] - terms["half_int_rho_vh"]
        print(f"[scf] hydrogen step {step}: residual {r:.3e}, eps_1 {theta[0]:.8f}, E {e_tot:.8f}, "
              f"CG {it}", flush=True)
        if r < 1e-7:
            break
    assert res[-1] < 1e-7
    assert terms["charge"] == pytest.approx(1.0, abs=1e-3)
    ctx.close()
