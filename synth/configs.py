"""Seeded synthetic workloads.

* hydrogen: one proton (V = -1/r) at a vertex in the centre of a Dirichlet
  cube, with the hydrogen 1s and 2s radials as enrichments.
* si_cluster: the n sites of a diamond lattice (a = 10.26 Bohr, an atom at
  the origin) nearest the origin, each jittered, with a softened nuclear
  potential -14/sqrt(r^2 + 0.01) per site and nine Slater-type enrichments
  per atom (1s, 2s, 2p, 3s, 3p).
* box: no potential and no enrichment (particle in a box).

Random numbers come from numpy's PCG64 `default_rng(seed)`, drawn in the
order: site jitter, Slater exponents, initial block.
"""
from __future__ import annotations

import numpy as np

from .assemble import assemble
from .enrich import EnrichmentSet, Radial
from .mesh import build_mesh
from .problem import Problem

SI_LATTICE = 10.26
SI_Z = 14.0
SOFTEN = 0.01


def diamond_sites(n_atoms: int, a: float = SI_LATTICE) -> np.ndarray:
    """The n_atoms diamond-lattice sites nearest the origin (an atom sits there).

    Sites are ordered by (distance rounded to 1e-9, x, y, z); ties on the last
    shell are broken by that order.
    """
    fcc = np.array([[0, 0, 0], [0, 0.5, 0.5], [0.5, 0, 0.5], [0.5, 0.5, 0]])
    basis = np.concatenate([fcc, fcc + 0.25])
    reach = int(np.ceil((3.0 * n_atoms / (4.0 * np.pi * 8.0)) ** (1.0 / 3.0))) + 2
    r = np.arange(-reach, reach + 1)
    cz, cy, cx = np.meshgrid(r, r, r, indexing="ij")
    cells = np.stack([cx.ravel(), cy.ravel(), cz.ravel()], axis=1).astype(np.float64)
    pts = (cells[:, None, :] + basis[None, :, :]).reshape(-1, 3) * a
    d = np.round(np.sqrt((pts ** 2).sum(axis=1)), 9)
    order = np.lexsort((pts[:, 2], pts[:, 1], pts[:, 0], d))
    return pts[order[:n_atoms]]


def softened_potential(centers: np.ndarray, z: float = SI_Z, eps: float = SOFTEN):
    def V(x: np.ndarray) -> np.ndarray:
        out = np.zeros(x.shape[0])
        for c in centers:
            d = x - c[None, :]
            out -= z / np.sqrt(np.einsum("qi,qi->q", d, d) + eps)
        return out
    return V


def coulomb_potential(center, z: float = 1.0):
    c = np.asarray(center, dtype=np.float64)

    def V(x: np.ndarray) -> np.ndarray:
        d = x - c[None, :]
        return -z / np.sqrt(np.einsum("qi,qi->q", d, d))
    return V


def zero_potential(x: np.ndarray) -> np.ndarray:
    return np.zeros(x.shape[0])


def hydrogen(nc: int = 8, length: float = 20.0, p: int = 4, r_c: float = 6.0,
             enrich: bool = True, **kw) -> Problem:
    mesh = build_mesh(p, nc, -0.5 * length, length)
    enr = None
    if enrich:
        enr = EnrichmentSet(centers=np.zeros((1, 3)),
                            shells=[Radial("h1s"), Radial("h2s")], r_c=r_c)
    V = coulomb_potential([0.0, 0.0, 0.0])
    prob = assemble(mesh, V, enr, singular_centers=np.zeros((1, 3)), **kw)
    prob.meta.update(kind="hydrogen", r_c=r_c, mesh=mesh, enr=enr, potential=V)
    return prob


def box(nc: int = 2, length: float = 2.0, p: int = 4, **kw) -> Problem:
    mesh = build_mesh(p, nc, -0.5 * length, length)
    prob = assemble(mesh, zero_potential, None, **kw)
    prob.meta.update(kind="box", mesh=mesh, potential=zero_potential)
    return prob


def si_shells(rng: np.random.Generator, lo: float = 0.5, hi: float = 14.0) -> list:
    z = np.sort(rng.uniform(lo, hi, 5))[::-1]
    return [Radial("slater", n=1, zeta=float(z[0]), l=0),
            Radial("slater", n=2, zeta=float(z[1]), l=0),
            Radial("slater", n=2, zeta=float(z[2]), l=1),
            Radial("slater", n=3, zeta=float(z[3]), l=0),
            Radial("slater", n=3, zeta=float(z[4]), l=1)]


def si_cluster(n_atoms: int = 30, length: float = 48.0, nc: int = 24, p: int = 4,
               r_c: float = 8.0, seed: int = 0, jitter: float = 0.05, enrich: bool = True,
               **kw) -> Problem:
    rng = np.random.default_rng(seed)
    sites = diamond_sites(n_atoms)
    sites = sites + rng.uniform(-jitter, jitter, sites.shape)
    shells = si_shells(rng)
    mesh = build_mesh(p, nc, -0.5 * length, length)
    enr = EnrichmentSet(centers=sites, shells=shells, r_c=r_c) if enrich else None
    V = softened_potential(sites)
    prob = assemble(mesh, V, enr, **kw)
    prob.meta.update(kind="si", sites=sites, shells=shells, r_c=r_c, mesh=mesh, enr=enr,
                     seed=seed, rng=rng, potential=V)
    return prob


def initial_block(prob: Problem, N: int, seed: int = 0) -> np.ndarray:
    """Starting subspace built from the atomic orbitals (the enrichment functions).

    The lowest N generalized eigenvectors of the enrichment pencil
    (H^ee, M^ee) are placed in the enrichment rows (classical rows zero);
    columns beyond n_e, or every column when there is no enrichment, are
    drawn N(0, 1) from `seed`.
    """
    import scipy.linalg as sla
    X = np.zeros((prob.n, N))
    k = min(N, prob.n_e)
    if k:
        _, V = sla.eigh(prob.H_ee, prob.M_ee)
        X[prob.n_h:, :k] = V[:, :k]
    if k < N:
        X[:, k:] = np.random.default_rng(seed).standard_normal((prob.n, N - k))
    return X


# Named workloads (sizes of the paper-shaped synthetic configurations).
def config1(**kw) -> Problem:
    """Hydrogen, 20 Bohr cube, 8^3 cells of degree 4, r_c = 6 (N = 16, m = 20)."""
    return hydrogen(nc=8, length=20.0, p=4, r_c=6.0, **kw)


def config2_classical(seed: int = 0, **kw) -> Problem:
    """The 30-atom Si cluster of config2 on the same mesh with no enrichment
    (classical finite elements only, n_e = 0)."""
    return si_cluster(n_atoms=30, length=48.0, nc=24, p=4, r_c=8.0, seed=seed, enrich=False, **kw)


def config2(seed: int = 0, **kw) -> Problem:
    """30-atom Si cluster, 48 Bohr cube, 24^3 cells of degree 4, r_c = 8 (N = 260, m = 40)."""
    return si_cluster(n_atoms=30, length=48.0, nc=24, p=4, r_c=8.0, seed=seed, **kw)


WORKLOADS = {
    "hydrogen-8c": dict(N=16, m=20, wanted=14),
    "si30-24c": dict(N=260, m=40, wanted=210),
}


def config3(seed: int = 0, plain_blocks: bool = False, **kw) -> Problem:
    """The 280-atom Si cluster: 80 Bohr cube, 48^3 degree-4 cells (n_h =
    6,967,871), 9 enrichments per atom (n_e = 2520).  By default the blocks of
    the cells without enrichment functions hold only the kinetic part: their
    potential term is assembled on the device (chebfilter_assemble_cells)
    from the potential at their Gauss points."""
    return si_cluster(n_atoms=280, length=80.0, nc=48, p=4, r_c=8.0, seed=seed,
                      plain_blocks=plain_blocks, **kw)


def si_cluster_meta(n_atoms: int = 30, length: float = 48.0, nc: int = 24, p: int = 4,
                    r_c: float = 8.0, seed: int = 0, jitter: float = 0.05) -> dict:
    """The meta entries si_cluster records (mesh, sites, shells, enrichment
    set, potential), rebuilt with the same draws and no assembly: for a
    problem whose element blocks were loaded from a file."""
    rng = np.random.default_rng(seed)
    sites = diamond_sites(n_atoms)
    sites = sites + rng.uniform(-jitter, jitter, sites.shape)
    shells = si_shells(rng)
    mesh = build_mesh(p, nc, -0.5 * length, length)
    enr = EnrichmentSet(centers=sites, shells=shells, r_c=r_c)
    return dict(kind="si", sites=sites, shells=shells, r_c=r_c, mesh=mesh, enr=enr, seed=seed,
                rng=rng, potential=softened_potential(sites))


def config3_meta(seed: int = 0) -> dict:
    """si_cluster_meta of config3."""
    return si_cluster_meta(n_atoms=280, length=80.0, nc=48, p=4, r_c=8.0, seed=seed)


def cluster_in_box(n_atoms: int, nc: int, seed: int, **kw) -> Problem:
    """An n_atoms Si cluster (diamond sites nearest the origin) in a cube of
    half-width R_cluster + 12 Bohr (R_cluster = the largest site coordinate)
    with nc degree-4 cells per axis, r_c = 8, nine Slater enrichments per atom."""
    sites = diamond_sites(n_atoms)
    R = float(np.abs(sites).max()) if n_atoms > 1 else 0.0
    return si_cluster(n_atoms=n_atoms, length=2.0 * (R + 12.0), nc=nc, p=4, r_c=8.0, seed=seed,
                      **kw)


def batch_cluster(n_atoms: int, seed: int = 0, **kw) -> Problem:
    """One problem of the batched workload: a cluster of 1-40 atoms in its
    own cube (cluster_in_box) with 8 + round(12 (n_atoms - 1) / 39) cells per
    axis (8^3 .. 20^3 cells); its own jitter and exponents (seed)."""
    return cluster_in_box(n_atoms, 8 + round(12 * (n_atoms - 1) / 39), 1000 + n_atoms + seed, **kw)


def batch_vectors(n_atoms: int) -> int:
    """Block width of a batched problem: 16 + round(334 (n_atoms - 1) / 39)
    (16 .. 350 vectors for 1 .. 40 atoms)."""
    return 16 + round(334 * (n_atoms - 1) / 39)


def batch_workload(count: int = 256, seed: int = 0, max_atoms: int = 40, progress=None, **kw):
    """Batched workload: `count` entries with atom counts drawn U{1..max_atoms}
    (seeded), batch_vectors(n_atoms) vectors each, filter degree 40.  The
    entries of one atom count share one generated problem (the pool), so the
    batch holds at most max_atoms distinct operators and `count` independent
    blocks and intervals.  Returns (pool dict n_atoms -> Problem, list of
    n_atoms per entry, list of N per entry).  progress(msg), if given, is
    called after each generated problem."""
    import time
    rng = np.random.default_rng(seed)
    atoms = [int(a) for a in rng.integers(1, max_atoms + 1, size=count)]
    pool = {}
    for a in sorted(set(atoms)):
        t0 = time.time()
        pool[a] = batch_cluster(a, seed, **kw)
        if progress:
            progress(f"pool problem {len(pool)}: {a} atoms, n = {pool[a].n}, "
                     f"{time.time() - t0:.1f}s")
    Ns = [batch_vectors(a) for a in atoms]
    return pool, atoms, Ns


def learned_cluster(n_atoms: int, seed: int = 0) -> Problem:
    """A small cluster of the learned-bounds study (1..8 atoms):
    cluster_in_box with 6 + round(6 (n_atoms - 1) / 7) cells per axis."""
    return cluster_in_box(n_atoms, 6 + round(6 * (n_atoms - 1) / 7), 1000 + n_atoms + seed)
