"""Atom-centred enrichment functions (Sec. IV.A, IV.B).

Each enrichment function is a radial function times a real spherical
harmonic, centred on an atom, and multiplied by the smooth cutoff of
Sec. IV.B so that it has compact support:

    h(rt) = u(rt) / (u(rt) + u(1 - rt)),  u(s) = exp(-1/s) for s > 0, else 0,
    rt = 1 - t (r - r0) / r0,

which equals 1 for r < r0 and 0 beyond r0 + r0/t.  Here the outer support
radius r_c is the configured cutoff, t = 1 and r0 = r_c / 2.

Radials are normalised before the cutoff (integral of R^2 r^2 dr = 1).  The
real harmonics are orthonormal; for l = 1 the three functions are ordered
(y, z, x) / r.  Function alpha of atom I is alpha = I * n_per_atom + k, k
running over the shells in order and, within a p shell, over (y, z, x).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from math import factorial, pi, sqrt

import numpy as np

Y00 = 1.0 / sqrt(4.0 * pi)
Y1C = sqrt(3.0 / (4.0 * pi))


# ---------------------------------------------------------------- radials
@dataclass(frozen=True)
class Radial:
    """Radial part R(r) and its derivative."""
    kind: str           # "slater" | "h1s" | "h2s"
    n: int = 1
    zeta: float = 1.0
    l: int = 0

    def terms(self) -> list[tuple[float, int, float]]:
        """R(r) as a sum of Slater-type terms c r^k exp(-zeta r): [(c, k, zeta)]."""
        if self.kind == "h1s":
            return [(2.0, 0, 1.0)]
        if self.kind == "h2s":
            c = 1.0 / (2.0 * sqrt(2.0))
            return [(2.0 * c, 0, 0.5), (-c, 1, 0.5)]
        if self.kind == "slater":
            n, z = self.n, self.zeta
            return [(sqrt((2.0 * z) ** (2 * n + 1) / factorial(2 * n)), n - 1, z)]
        raise ValueError(self.kind)

    def eval(self, r: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
        if self.kind == "h1s":          # hydrogen 1s: 2 e^{-r}
            e = np.exp(-r)
            return 2.0 * e, -2.0 * e
        if self.kind == "h2s":          # hydrogen 2s: (2 - r) e^{-r/2} / (2 sqrt 2)
            e = np.exp(-0.5 * r)
            c = 1.0 / (2.0 * sqrt(2.0))
            return c * (2.0 - r) * e, c * e * (-1.0 - 0.5 * (2.0 - r))
        if self.kind == "slater":       # N r^{n-1} e^{-zeta r}
            n, z = self.n, self.zeta
            norm = sqrt((2.0 * z) ** (2 * n + 1) / factorial(2 * n))
            e = np.exp(-z * r)
            if n == 1:
                return norm * e, -z * norm * e
            rn2 = r ** (n - 2)
            R = norm * rn2 * r * e
            dR = norm * e * ((n - 1) * rn2 - z * rn2 * r)
            return R, dR
        raise ValueError(self.kind)


# ---------------------------------------------------------------- cutoff
def _u(s: np.ndarray) -> np.ndarray:
    out = np.zeros_like(s)
    m = s > 0
    out[m] = np.exp(-1.0 / s[m])
    return out


def _du(s: np.ndarray) -> np.ndarray:
    out = np.zeros_like(s)
    m = s > 0
    out[m] = np.exp(-1.0 / s[m]) / (s[m] * s[m])
    return out


def cutoff(r: np.ndarray, r0: float, t: float = 1.0) -> tuple[np.ndarray, np.ndarray]:
    """Smooth cutoff h(r) of Sec. IV.B and dh/dr."""
    rt = 1.0 - t * (r - r0) / r0
    a, b = _u(rt), _u(1.0 - rt)
    den = a + b
    h = a / den
    dh_drt = (_du(rt) * b + a * _du(1.0 - rt)) / (den * den)
    return h, dh_drt * (-t / r0)


# ---------------------------------------------------------------- function set
@dataclass
class EnrichmentSet:
    centers: np.ndarray                 # [n_atoms, 3]
    shells: list                        # list[Radial], shared by all atoms
    r_c: float                          # outer support radius
    t: float = 1.0
    cache: dict = field(default_factory=dict, repr=False)

    @property
    def r0(self) -> float:
        return self.r_c / (1.0 + 1.0 / self.t)

    @property
    def n_atoms(self) -> int:
        return int(self.centers.shape[0])

    @property
    def n_per_atom(self) -> int:
        return sum(2 * s.l + 1 for s in self.shells)

    @property
    def n_e(self) -> int:
        return self.n_atoms * self.n_per_atom

    def shell_terms(self) -> list[tuple[int, list]]:
        """[(l, [(c, k, zeta), ...])] per shell: the radial as Slater-type terms."""
        return [(s.l, s.terms()) for s in self.shells]

    def func_table(self) -> list[tuple[int, int, int]]:
        """(atom, shell index, m-component) per alpha, in alpha order."""
        out = []
        for I in range(self.n_atoms):
            for si, s in enumerate(self.shells):
                for m in range(2 * s.l + 1):
                    out.append((I, si, m))
        return out

    def radial_g(self, si: int, r: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
        """g = h R and g' for shell si."""
        R, dR = self.shells[si].eval(r)
        h, dh = cutoff(r, self.r0, self.t)
        return h * R, dh * R + h * dR

    def eval_atom(self, I: int, pts: np.ndarray, need_grad: bool = True):
        """Values [Q, n_per_atom] (and gradients [Q, n_per_atom, 3]) of atom I's functions."""
        d = pts - self.centers[I][None, :]
        r = np.sqrt(np.einsum("qi,qi->q", d, d))
        r = np.maximum(r, 1e-300)
        val = np.empty((pts.shape[0], self.n_per_atom))
        grad = np.empty((pts.shape[0], self.n_per_atom, 3)) if need_grad else None
        k = 0
        for si, s in enumerate(self.shells):
            g, dg = self.radial_g(si, r)
            if s.l == 0:
                val[:, k] = Y00 * g
                if need_grad:
                    grad[:, k, :] = (Y00 * dg / r)[:, None] * d
                k += 1
            elif s.l == 1:
                q = g / r
                dq = (dg - q) / r
                for comp in (1, 2, 0):                     # y, z, x
                    xi = d[:, comp]
                    val[:, k] = Y1C * xi * q
                    if need_grad:
                        gr = (Y1C * xi * dq / r)[:, None] * d
                        gr[:, comp] += Y1C * q
                        grad[:, k, :] = gr
                    k += 1
            else:
                raise NotImplementedError("only l <= 1 shells are used")
        return val, grad

    def trial_sums(self, I: int, pts: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
        """Sum over atom I's functions of N^2 and |grad N|^2.

        Uses the addition theorem: summed over m, Y_lm^2 gives (2l+1)/(4 pi)
        and |grad_angular Y_lm|^2 gives l(l+1)(2l+1)/(4 pi).
        """
        d = pts - self.centers[I][None, :]
        r = np.maximum(np.sqrt(np.einsum("qi,qi->q", d, d)), 1e-300)
        f3 = np.zeros(pts.shape[0])
        f4 = np.zeros(pts.shape[0])
        for si, s in enumerate(self.shells):
            g, dg = self.radial_g(si, r)
            c = (2 * s.l + 1) / (4.0 * pi)
            f3 += c * g * g
            f4 += c * (dg * dg + s.l * (s.l + 1) * g * g / (r * r))
        return f3, f4
