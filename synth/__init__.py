"""Seeded synthetic input generator: the discrete enriched-FE problem.

Builds the element blocks (the hot path's input) from a uniform spectral
hexahedral mesh, analytic potentials and atom-centred enrichment functions
(Sec. III, IV.A-C).  It holds no part of the filter, the overlap inverse,
the orthonormalisation or the Rayleigh-Ritz step.
"""
from .problem import Problem  # noqa: F401
