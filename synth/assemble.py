"""Element blocks of the enriched spectral-FE Kohn-Sham problem (Eq. HBlocks, MBlocks).

For every cell e with local nodes a, b and enrichment functions alpha, beta
meeting the cell:

    H_cc_e[a,b]   = 1/2 int grad N_a . grad N_b + int V N_a N_b
    H_ec_e[al,a]  = 1/2 int grad N_al . grad N_a + int V N_al N_a
    M_ec_e[al,a]  = int N_al N_a
    H_ee[al,be]  += 1/2 int grad N_al . grad N_be + int V N_al N_be
    M_ee[al,be]  += int N_al N_be

and the classical overlap is the GLL-lumped diagonal (Sec. III.B).  The
kinetic part of H_cc_e is a polynomial and is integrated exactly with the
1D tensor factors; every integral with V or an enrichment function uses the
cell's quadrature rule (plain n_g^3 Gauss, or the adaptive rule inside
enrichment supports).
"""
from __future__ import annotations

import time

import numpy as np

from .basis import gauss_rule, gll_rule, lagrange_eval
from .enrich import EnrichmentSet
from .mesh import Mesh
from .problem import Problem
from .quad import adaptive_rule, unit_cube_rule


def _tensor3(a1: np.ndarray, a2: np.ndarray, a3: np.ndarray) -> np.ndarray:
    """Operator on x-fastest local indices: a1 acts on x, a2 on y, a3 on z."""
    return np.kron(a3, np.kron(a2, a1))


def reference_kinetic(p: int, h: float) -> np.ndarray:
    """1/2 int grad N_a . grad N_b over a cube of side h (exact)."""
    xi, _ = gll_rule(p)
    gx, gw = gauss_rule(p + 2)
    L, dL = lagrange_eval(xi, gx)
    M1 = (L * gw[:, None]).T @ L
    K1 = (dL * gw[:, None]).T @ dL
    jac = (0.5 * h) ** 3
    s = (2.0 / h) ** 2
    K = _tensor3(K1, M1, M1) + _tensor3(M1, K1, M1) + _tensor3(M1, M1, K1)
    return 0.5 * jac * s * K


def shape_at(p: int, h: float, lo: np.ndarray, pts: np.ndarray, need_grad: bool):
    """Values [Q, npc] (and physical gradients, three arrays [Q, npc]) of a cell's basis."""
    xi, _ = gll_rule(p)
    ref = 2.0 * (pts - lo[None, :]) / h - 1.0
    Lx, dLx = lagrange_eval(xi, ref[:, 0])
    Ly, dLy = lagrange_eval(xi, ref[:, 1])
    Lz, dLz = lagrange_eval(xi, ref[:, 2])
    Q = pts.shape[0]
    k = p + 1

    def outer(ax, ay, az):
        return (az[:, :, None, None] * ay[:, None, :, None] * ax[:, None, None, :]).reshape(Q, k ** 3)

    N = outer(Lx, Ly, Lz)
    if not need_grad:
        return N, None
    s = 2.0 / h
    G = (outer(dLx * s, Ly, Lz), outer(Lx, dLy * s, Lz), outer(Lx, Ly, dLz * s))
    return N, G


def plain_tables(prob, ng: int = 6):
    """Reference tables of the plain rule of a generated problem: B [nq, npc]
    shape values at the ng^3 Gauss points (the same in every cell), w [nq]
    weights times the cell volume, K [npc, npc] the kinetic block, and the
    points in the unit cube [nq, 3] (x fastest)."""
    mesh = prob.meta["mesh"]
    ref, wref = unit_cube_rule(ng)
    B, _ = shape_at(mesh.p, 2.0, np.array([-1.0, -1.0, -1.0]), 2.0 * ref - 1.0, need_grad=False)
    return B, wref * mesh.h ** 3, reference_kinetic(mesh.p, mesh.h), ref


def plain_points(prob, cells, ng: int = 6) -> np.ndarray:
    """Physical Gauss points [len(cells), nq, 3] of the listed cells."""
    mesh = prob.meta["mesh"]
    ref, _ = unit_cube_rule(ng)
    return mesh.cell_lo()[np.asarray(cells)][:, None, :] + mesh.h * ref[None]


_POT: dict = {}


def _pot_chunk(bounds):
    a, b = bounds
    return _POT["V"](_POT["pts"][a:b])


def potential_at_points(V, pts: np.ndarray, nproc: int | None = None,
                        chunk: int = 1 << 20) -> np.ndarray:
    """V at pts [Q, 3], in chunks over forked workers (V may be a closure;
    the workers inherit it), or in-process chunk by chunk once the GPU is
    initialised.  Values do not depend on the chunking."""
    import multiprocessing as mp
    bounds = [(a, min(a + chunk, len(pts))) for a in range(0, len(pts), chunk)]
    nw = min(nproc or _workers(), len(bounds))
    if gpu_initialised():
        nw = 1
    if nw <= 1:
        return np.concatenate([V(pts[a:b]) for a, b in bounds]) if bounds else V(pts)
    _POT.update(V=V, pts=pts)
    try:
        with mp.get_context("fork").Pool(nw) as pool:
            parts = pool.map(_pot_chunk, bounds)
    finally:
        _POT.clear()
    return np.concatenate(parts)


def gll_lumped_diag(mesh: Mesh) -> np.ndarray:
    _, w = gll_rule(mesh.p)
    we = (0.5 * mesh.h) ** 3 * _tensor3(np.diag(w), np.diag(w), np.diag(w)).diagonal()
    D = np.zeros(mesh.n_h)
    cd = mesh.cell_dof
    m = cd >= 0
    np.add.at(D, cd[m], np.broadcast_to(we[None, :], cd.shape)[m])
    return D


def box_distance(lo: np.ndarray, h: float, c: np.ndarray) -> np.ndarray:
    """Euclidean distance from point c to each box [lo, lo+h]^3 (lo: [E,3])."""
    d = np.maximum(np.maximum(lo - c[None, :], c[None, :] - (lo + h)), 0.0)
    return np.sqrt(np.einsum("ei,ei->e", d, d))


# State shared with forked workers (set by assemble before the pool starts).
_W: dict = {}


def _trial(x: np.ndarray, atoms) -> np.ndarray:
    """Trial functions of Sec. IV.C: sum N^2, sum |grad N|^2 and |V| (1 + sum N^2)."""
    enr, potential = _W["enr"], _W["potential"]
    f3 = np.zeros(x.shape[0])
    f4 = np.zeros(x.shape[0])
    for I in atoms:
        a3, a4 = enr.trial_sums(I, x)
        f3 += a3
        f4 += a4
    return np.stack([f3, f4, np.abs(potential(x)) * (1.0 + f3)], axis=1)


def _plain_integrals(cells) -> np.ndarray:
    ref, wref = unit_cube_rule(_W["ng"])
    h, lo_all, cell_atoms = _W["h"], _W["lo_all"], _W["cell_atoms"]
    out = np.zeros(3)
    for e in cells:
        f = _trial(lo_all[e][None, :] + h * ref, cell_atoms[e])
        out += np.abs(wref @ f) * h ** 3
    return out


def _enriched_chunk(cells):
    """Element blocks of a chunk of enriched cells; H_ee / M_ee partial sums."""
    from threadpoolctl import threadpool_limits
    enr, potential = _W["enr"], _W["potential"]
    p, h, K = _W["p"], _W["h"], _W["K"]
    lo_all, cell_atoms, enr_ptr, enr_idx = _W["lo_all"], _W["cell_atoms"], _W["enr_ptr"], _W["enr_idx"]
    n_e, tau = _W["n_e"], _W["tau"]
    Hcc, Hec, Mec, boxes = [], [], [], []
    # the chunk's partial H_ee / M_ee on the enrichment indices it touches
    # (the other entries of the partial are zero)
    used = np.unique(np.concatenate([enr_idx[enr_ptr[e]:enr_ptr[e + 1]] for e in cells]))
    pos = np.full(n_e, -1, dtype=np.int64)
    pos[used] = np.arange(used.size)
    Hee = np.zeros((used.size, used.size))
    Mee = np.zeros((used.size, used.size))
    stats = np.zeros(3)
    with threadpool_limits(_W["blas_threads"]):
        for e in cells:
            lo = lo_all[e]
            atoms = cell_atoms[e]
            pts, w, leaves, blo, bsz = adaptive_rule(lo, h, lambda x: _trial(x, atoms), tau,
                                                     ng=_W["ng"], max_depth=_W["max_depth"],
                                                     boxes=True)
            boxes.append((blo, bsz))
            stats += (leaves, w.size, 0)
            stats[2] = max(stats[2], leaves)
            N, G = shape_at(p, h, lo, pts, need_grad=True)
            wV = w * potential(pts)
            Hcc.append(K + (N.T * wV[None, :]) @ N)
            vals, grads = [], []
            for I in atoms:
                v, g = enr.eval_atom(I, pts)
                vals.append(v)
                grads.append(g)
            Ev = np.concatenate(vals, axis=1)                   # [Q, na]
            Eg = np.concatenate(grads, axis=1)                  # [Q, na, 3]
            Egd = [np.ascontiguousarray(Eg[:, :, d]) for d in range(3)]
            EwT = (Ev * w[:, None]).T                           # [na, Q]
            EgwT = [(g * w[:, None]).T for g in Egd]
            Hec.append(0.5 * sum(EgwT[d] @ G[d] for d in range(3)) + (Ev * wV[:, None]).T @ N)
            Mec.append(EwT @ N)
            idx = pos[enr_idx[enr_ptr[e]:enr_ptr[e + 1]]]
            kin_ee = 0.5 * sum(EgwT[d] @ Egd[d] for d in range(3))
            Hee[np.ix_(idx, idx)] += kin_ee + (Ev * wV[:, None]).T @ Ev
            Mee[np.ix_(idx, idx)] += EwT @ Ev
    return Hcc, Hec, Mec, (used, Hee), (used, Mee), stats, boxes


def gpu_initialised() -> bool:
    """True once this process holds the GPU driver open (an open /dev/kfd):
    after any HIP call, and from the start under a profiler that initialises
    the GPU before the program runs.  A forked child of such a process shares
    the driver state, so the generator then works in-process."""
    import os
    try:
        fds = os.listdir("/proc/self/fd")
    except OSError:
        return False
    for fd in fds:
        try:
            if os.readlink(f"/proc/self/fd/{fd}") == "/dev/kfd":
                return True
        except OSError:
            continue
    return False


def _workers() -> int:
    import os
    if gpu_initialised():
        return 1
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return max(1, min(16, n))


def assemble(mesh: Mesh, potential, enr: EnrichmentSet | None, ng: int = 6,
             tol_rel: float = 1e-10, tol_abs: float = 1e-14, max_depth: int = 10,
             chunk: int = 16, workers: int | None = None, verbose: bool = False,
             plain_blocks: bool = True, progress=None, singular_centers=None) -> Problem:
    """Element blocks of the problem.

    The adaptive-quadrature tolerance of trial function nu is
    tau_nu = max(tol_abs, tol_rel * S_nu), S_nu = its integral over all
    enriched cells by the plain rule.  Enriched cells are integrated in fixed
    chunks (results combined in chunk order, so the output does not depend on
    the number of worker processes).  With plain_blocks=False the cells
    without enrichment functions get the kinetic block K only (their
    potential term is left to a device assembly from the potential at their
    Gauss points; meta["plain_blocks"] records it).  progress(msg), if given,
    is called at each stage and about every 30 s while the enriched cells
    are integrated.
    singular_centers [k, 3]: points where the potential is singular (bare
    nuclei); the cells without enrichment functions that touch one (box
    distance below h / 2) take the potential term by the adaptive rule with
    the trial function |V| (tolerance tol_rel times its plain-rule integral
    over those cells), as the enriched cells do.
    """
    t0 = time.time()
    p, h, E, npc = mesh.p, mesh.h, mesh.n_cells, mesh.npc
    lo_all = mesh.cell_lo()
    K = reference_kinetic(p, h)
    D = gll_lumped_diag(mesh)

    # ---- which enrichment functions meet which cell
    n_e = 0 if enr is None else enr.n_e
    cell_atoms: list[list[int]] = [[] for _ in range(E)]
    if enr is not None:
        box_lo, box_hi = mesh.lo, mesh.lo + mesh.length
        for I in range(enr.n_atoms):
            c = enr.centers[I]
            if np.any(c - enr.r_c <= box_lo) or np.any(c + enr.r_c >= box_hi):
                raise ValueError(f"enrichment support of atom {I} reaches the Dirichlet boundary")
            for e in np.nonzero(box_distance(lo_all, h, c) < enr.r_c)[0]:
                cell_atoms[e].append(I)
    npa = 0 if enr is None else enr.n_per_atom
    counts = np.array([len(a) * npa for a in cell_atoms], dtype=np.int64)
    enr_ptr = np.zeros(E + 1, dtype=np.int64)
    enr_ptr[1:] = np.cumsum(counts)
    nnz = int(enr_ptr[-1])
    enr_idx = np.empty(nnz, dtype=np.int64)
    for e in range(E):
        if counts[e]:
            enr_idx[enr_ptr[e]:enr_ptr[e + 1]] = (
                np.array(cell_atoms[e])[:, None] * npa + np.arange(npa)[None, :]).ravel()

    H_cc = np.empty((E, npc, npc))
    H_ec = np.zeros((nnz, npc))
    M_ec = np.zeros((nnz, npc))
    H_ee = np.zeros((n_e, n_e))
    M_ee = np.zeros((n_e, n_e))

    # leaf boxes of every cell with its own adaptive rule (Sec. IV.C)
    cell_boxes: dict = {}

    # ---- cells without enrichment: plain Gauss rule, batched
    ref, wref = unit_cube_rule(ng)
    Bref, _ = shape_at(p, 2.0, np.array([-1.0, -1.0, -1.0]), 2.0 * ref - 1.0, need_grad=False)
    plain = np.nonzero(counts == 0)[0]
    jac = h ** 3
    if singular_centers is not None and plain.size:
        near = np.zeros(E, dtype=bool)
        for c in np.asarray(singular_centers, dtype=np.float64).reshape(-1, 3):
            near |= box_distance(lo_all, h, c) < 0.5 * h
        sing = plain[near[plain]]
        plain = plain[~near[plain]]
        if sing.size:
            ref0, wref0 = unit_cube_rule(ng)
            fV = lambda x: np.abs(potential(x))[:, None]          # noqa: E731
            SV = sum(abs(float((wref0 * jac) @ fV(lo_all[e][None, :] + h * ref0)[:, 0]))
                     for e in sing)
            tauV = np.array([max(tol_abs, tol_rel * SV)])
            for e in sing:
                pts, w, _, blo, bsz = adaptive_rule(lo_all[e], h, fV, tauV, ng=ng,
                                                    max_depth=max_depth, boxes=True)
                cell_boxes[e] = (blo, bsz)
                Nq, _ = shape_at(p, h, lo_all[e], pts, need_grad=False)
                H_cc[e] = K + (Nq.T * (w * potential(pts))[None, :]) @ Nq
    if not plain_blocks:
        H_cc[plain] = K[None]
        plain = plain[:0]
    for s in range(0, plain.size, 256):
        cells = plain[s:s + 256]
        pts = lo_all[cells][:, None, :] + h * ref[None]
        wv = potential(pts.reshape(-1, 3)).reshape(cells.size, -1) * (wref * jac)[None, :]
        H_cc[cells] = K[None] + np.matmul(Bref.T[None] * wv[:, None, :], Bref[None])
    t1 = time.time()
    if progress:
        progress(f"cells without enrichment done ({t1 - t0:.0f}s)")

    # ---- enriched cells: adaptive rule, fixed chunks, forked workers
    stats = {"enriched_cells": 0, "leaves": 0, "points": 0, "max_leaves": 0}
    ecells = np.nonzero(counts)[0]
    if ecells.size:
        _W.clear()
        _W.update(enr=enr, potential=potential, p=p, h=h, K=K, lo_all=lo_all,
                  cell_atoms=cell_atoms, enr_ptr=enr_ptr, enr_idx=enr_idx, n_e=n_e, ng=ng,
                  max_depth=max_depth, blas_threads=1)
        chunks = [ecells[i:i + chunk] for i in range(0, ecells.size, chunk)]
        nw = 1 if gpu_initialised() else (workers or _workers())
        if nw > 1 and len(chunks) > 1:
            import multiprocessing as mp
            ctx = mp.get_context("fork")
            with ctx.Pool(nw) as pool:
                S = np.sum(pool.map(_plain_integrals, chunks), axis=0)
                _W["tau"] = np.maximum(tol_abs, tol_rel * S)
            pool = ctx.Pool(nw)
            results = pool.imap(_enriched_chunk, chunks)
        else:
            pool = None
            S = np.sum([_plain_integrals(c) for c in chunks], axis=0)
            _W["tau"] = np.maximum(tol_abs, tol_rel * S)
            results = (_enriched_chunk(c) for c in chunks)
        if progress:
            progress(f"tolerances set; {len(chunks)} chunks of enriched cells ({time.time() - t0:.0f}s)")
        t_last = time.time()
        for k, (cells, (hcc, hec, mec, hee, mee, st, bx)) in enumerate(zip(chunks, results)):
            if progress and time.time() - t_last > 30.0:
                progress(f"enriched cells: chunk {k + 1}/{len(chunks)} ({time.time() - t1:.0f}s)")
                t_last = time.time()
            for i, e in enumerate(cells):
                cell_boxes[e] = bx[i]
                H_cc[e] = hcc[i]
                H_ec[enr_ptr[e]:enr_ptr[e + 1]] = hec[i]
                M_ec[enr_ptr[e]:enr_ptr[e + 1]] = mec[i]
            (hu, hb), (mu, mb) = hee, mee
            H_ee[np.ix_(hu, hu)] += hb
            M_ee[np.ix_(mu, mu)] += mb
            stats["leaves"] += int(st[0])
            stats["points"] += int(st[1])
            stats["max_leaves"] = max(stats["max_leaves"], int(st[2]))
        if pool is not None:
            pool.close()
            pool.join()
        stats["enriched_cells"] = int(ecells.size)
        stats["tau"] = [float(x) for x in _W["tau"]]
        _W.clear()
    for c0 in range(0, E, 4096):           # symmetrise in slices (bounded temporaries)
        blk = H_cc[c0:c0 + 4096]
        blk[...] = (blk + np.swapaxes(blk, 1, 2)) * 0.5
    H_ee = 0.5 * (H_ee + H_ee.T)
    M_ee = 0.5 * (M_ee + M_ee.T)
    t2 = time.time()
    stats.update(t_plain=t1 - t0, t_enriched=t2 - t1)
    if verbose:
        print(f"[assemble] E={E} n_h={mesh.n_h} n_e={n_e} nnz={nnz} {stats}", flush=True)
    # the leaf boxes as one list (cell by cell, in cell order): cell e owns
    # boxes box_ptr[e] .. box_ptr[e+1]; each box carries the ng^3 Gauss rule
    counts_b = np.zeros(E, dtype=np.int64)
    for e, (blo, _) in cell_boxes.items():
        counts_b[e] = blo.shape[0]
    box_ptr = np.zeros(E + 1, dtype=np.int64)
    box_ptr[1:] = np.cumsum(counts_b)
    box_lo = np.zeros((int(box_ptr[-1]), 3))
    box_size = np.zeros(int(box_ptr[-1]))
    for e, (blo, bsz) in cell_boxes.items():
        box_lo[box_ptr[e]:box_ptr[e + 1]] = blo
        box_size[box_ptr[e]:box_ptr[e + 1]] = bsz
    meta = {"h": h, "nc": mesh.nc, "lo": mesh.lo, "length": mesh.length, "quad": stats,
            "plain_blocks": plain_blocks,
            "quad_boxes": {"ng": ng, "box_ptr": box_ptr, "box_lo": box_lo, "box_size": box_size}}
    return Problem(p=p, cell_dof=mesh.cell_dof, H_cc=H_cc, M_cc_diag=D, enr_ptr=enr_ptr,
                   enr_idx=enr_idx, H_ec=H_ec, M_ec=M_ec, H_ee=H_ee, M_ee=M_ee, meta=meta)
