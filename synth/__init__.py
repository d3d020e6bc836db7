"""Seeded synthetic CT/CBCT phantoms for DISC tests and benchmarks.

This package holds input generation only: analytic phantoms, known
deformations and CBCT artifact models. It contains none of the DISC
arithmetic and serves both the oracle-side tests and the HIP path.
"""
from .phantom import CONFIGS, Case, make_case, make_hn_pair, make_ellipsoid_pair  # noqa: F401
