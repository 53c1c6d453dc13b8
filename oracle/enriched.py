"""Element blocks of a cell inside enrichment supports (oracle; test
infrastructure only).

Eq. HBlocks and Eq. MBlocks restricted to one cell e, evaluated with the
cell's own quadrature points x_q and weights w_q (Jacobian included).  These
come from the adaptive rule of Sec. IV.C: a union of boxes, each carrying an
n-point Gauss rule per axis.  V_q is the potential at x_q.

    H^cc_e[a, b]   = K[a, b] + sum_q w_q V_q N_a N_b
    H^ec_e[al, a]  = sum_q w_q (1/2 grad N_al . grad N_a + V_q N_al N_a)
    M^ec_e[al, a]  = sum_q w_q N_al N_a
    H^ee_e[al, be] = sum_q w_q (1/2 grad N_al . grad N_be + V_q N_al N_be)
    M^ee_e[al, be] = sum_q w_q N_al N_be

N_a is the cell's tensor-product Lagrange basis of degree p through the 1D
nodes (Sec. III.B).  Local index a = i + (p+1) j + (p+1)^2 k puts x fastest.
K (the polynomial kinetic block) is an input.  H^ee and M^ee of the whole
problem are the sums of the cell terms over the cells.

N_al is an enrichment function (Sec. IV.A, IV.B).  Each one is centred on an
atom at R: the radial part R(r) times a real spherical harmonic, multiplied
by the smooth cutoff h of Eq. Moll1.  R(r) is given as a sum of Slater-type
terms c r^k exp(-zeta r).  The harmonics are Y_00 = 1/sqrt(4 pi) and, for
l = 1, sqrt(3/(4 pi)) (y, z, x)/r, in that order.  An atom's functions are
its shells in order, and within a p shell (y, z, x).  This is a labelling
convention that the generator and the library share.

Everything is written out point by point: values and gradients at every
point, then the weighted sums as plain contractions.
"""
from __future__ import annotations

from math import pi, sqrt

import numpy as np

Y00 = 1.0 / sqrt(4.0 * pi)
Y1 = sqrt(3.0 / (4.0 * pi))
P_AXES = (1, 2, 0)              # l = 1 components in function order: y, z, x


def lagrange_1d(nodes: np.ndarray, x: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Lagrange polynomials through `nodes` and their derivatives at x:
    l_i(x) = prod_{j != i} (x - x_j) / (x_i - x_j).  Returns [len(x), len(nodes)]
    each; the derivative is the sum over the left-out factor."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64).reshape(-1)
    k = nodes.size
    val = np.ones((x.size, k))
    der = np.zeros((x.size, k))
    for i in range(k):
        for j in range(k):
            if j == i:
                continue
            f = (x - nodes[j]) / (nodes[i] - nodes[j])
            der[:, i] = der[:, i] * f + val[:, i] / (nodes[i] - nodes[j])
            val[:, i] = val[:, i] * f
    return val, der


def cell_basis(nodes01: np.ndarray, lo: np.ndarray, h: float, pts: np.ndarray):
    """Values [Q, (p+1)^3] and physical gradients [3, Q, (p+1)^3] of the cell
    [lo, lo + h]^3's basis; nodes01 are the 1D nodes on [0, 1]."""
    s = (np.asarray(pts, dtype=np.float64) - np.asarray(lo, dtype=np.float64)[None, :]) / h
    L = [lagrange_1d(nodes01, s[:, d]) for d in range(3)]
    Q, k = s.shape[0], len(nodes01)

    def tp(fx, fy, fz):
        return np.einsum("qk,qj,qi->qkji", fz, fy, fx).reshape(Q, k ** 3)

    N = tp(L[0][0], L[1][0], L[2][0])
    G = np.stack([tp(L[0][1] / h, L[1][0], L[2][0]),
                  tp(L[0][0], L[1][1] / h, L[2][0]),
                  tp(L[0][0], L[1][0], L[2][1] / h)])
    return N, G


def smooth_cutoff(r: np.ndarray, r0: float, t: float) -> tuple[np.ndarray, np.ndarray]:
    """h(r~) of Eq. Moll1 with r~ = 1 - t (r - r0) / r0, u(s) = exp(-1/s) for
    s > 0 (else 0), h = u(r~) / (u(r~) + u(1 - r~)); returns h and dh/dr."""
    r = np.asarray(r, dtype=np.float64)
    rt = 1.0 - t * (r - r0) / r0

    def u(s):
        out = np.zeros_like(s)
        m = s > 0
        out[m] = np.exp(-1.0 / s[m])
        return out

    def du(s):
        out = np.zeros_like(s)
        m = s > 0
        out[m] = np.exp(-1.0 / s[m]) / (s[m] * s[m])
        return out

    a, b = u(rt), u(1.0 - rt)
    den = a + b
    hval = a / den
    dh_drt = (du(rt) * b + a * du(1.0 - rt)) / (den * den)
    return hval, dh_drt * (-t / r0)


def radial_terms(terms, r: np.ndarray, shift: int = 0) -> tuple[np.ndarray, np.ndarray]:
    """sum_(c, k, zeta) c r^(k - shift) exp(-zeta r) and its r-derivative.
    `terms` is a list of (c, k, zeta), and every k - shift must be >= 0."""
    r = np.asarray(r, dtype=np.float64)
    v = np.zeros_like(r)
    dv = np.zeros_like(r)
    for c, k, z in terms:
        kk = int(k) - shift
        if kk < 0:
            raise ValueError("radial term power below zero")
        e = c * np.exp(-z * r)
        pk = r ** kk
        v += pk * e
        dv += (kk * r ** (kk - 1) if kk > 0 else 0.0) * e - z * pk * e
    return v, dv


def atom_functions(center, shells, r0: float, t: float, pts: np.ndarray):
    """Values [Q, n] and gradients [Q, n, 3] of one atom's enrichment
    functions.  `shells` is a list of (l, terms) with l in {0, 1}."""
    d = np.asarray(pts, dtype=np.float64) - np.asarray(center, dtype=np.float64)[None, :]
    r = np.sqrt((d * d).sum(axis=1))
    rs = np.maximum(r, 1e-300)
    hc, dhc = smooth_cutoff(r, r0, t)
    n = sum(2 * l + 1 for l, _ in shells)
    val = np.empty((d.shape[0], n))
    grad = np.empty((d.shape[0], n, 3))
    k = 0
    for l, terms in shells:
        if l == 0:
            R, dR = radial_terms(terms, r)
            g, dg = hc * R, dhc * R + hc * dR           # g = h R
            val[:, k] = Y00 * g
            grad[:, k, :] = (Y00 * dg / rs)[:, None] * d
            k += 1
        elif l == 1:
            S, dS = radial_terms(terms, r, shift=1)      # S = R / r
            q, dq = hc * S, dhc * S + hc * dS           # q = h R / r
            for ax in P_AXES:
                val[:, k] = Y1 * d[:, ax] * q
                gr = (Y1 * d[:, ax] * dq / rs)[:, None] * d
                gr[:, ax] += Y1 * q
                grad[:, k, :] = gr
                k += 1
        else:
            raise ValueError("only l <= 1 shells")
    return val, grad


def box_points(boxes_lo: np.ndarray, boxes_size: np.ndarray, gx: np.ndarray, gw: np.ndarray):
    """Points [nbox * ng^3, 3] and weights of a union of boxes, each with the
    tensor Gauss rule (gx, gw on [0, 1], weights summing to 1), x fastest
    inside a box, boxes in the given order."""
    ng = len(gx)
    zz, yy, xx = np.meshgrid(gx, gx, gx, indexing="ij")
    ref = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1)
    wz, wy, wx = np.meshgrid(gw, gw, gw, indexing="ij")
    wref = (wx * wy * wz).ravel()
    lo = np.asarray(boxes_lo, dtype=np.float64).reshape(-1, 3)
    sz = np.asarray(boxes_size, dtype=np.float64).reshape(-1)
    pts = lo[:, None, :] + sz[:, None, None] * ref[None]
    w = (sz[:, None] ** 3) * wref[None]
    return pts.reshape(-1, 3), w.reshape(-1), ng


def enriched_cell_blocks(K, nodes01, lo, h, pts, w, V, atoms, centers, shells, r0, t):
    """The five blocks of one cell (module docstring).  atoms: the atoms whose
    functions meet the cell, in the order of the cell's enrichment list.
    Returns (H_cc [npc, npc], H_ec [na, npc], M_ec [na, npc], H_ee_e [na, na],
    M_ee_e [na, na])."""
    pts = np.asarray(pts, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    wV = w * np.asarray(V, dtype=np.float64)
    N, G = cell_basis(nodes01, lo, h, pts)
    H_cc = np.asarray(K, dtype=np.float64) + (N * wV[:, None]).T @ N
    if len(atoms) == 0:
        z = np.zeros((0, N.shape[1]))
        return H_cc, z, z, np.zeros((0, 0)), np.zeros((0, 0))
    vals, grads = zip(*(atom_functions(centers[I], shells, r0, t, pts) for I in atoms))
    E = np.concatenate(vals, axis=1)                         # [Q, na]
    EG = np.concatenate(grads, axis=1)                       # [Q, na, 3]
    EGd = [np.ascontiguousarray(EG[:, :, d]) for d in range(3)]
    kin_ec = 0.5 * sum((EGd[d] * w[:, None]).T @ G[d] for d in range(3))
    kin_ee = 0.5 * sum((EGd[d] * w[:, None]).T @ EGd[d] for d in range(3))
    H_ec = kin_ec + (E * wV[:, None]).T @ N
    M_ec = (E * w[:, None]).T @ N
    H_ee = kin_ee + (E * wV[:, None]).T @ E
    M_ee = (E * w[:, None]).T @ E
    return H_cc, H_ec, M_ec, H_ee, M_ee
