"""Seeded synthetic inputs shared by the HIP path, the oracle and the benchmarks.

This package only *makes data*: mechanism files (species, stoichiometry, rate
parameters, NASA-7 coefficients) and per-cell fields (T, p, Y).  It evaluates
none of the chemistry step itself, so the two implementations that consume its
output (the CPU oracle and the GPU library) stay independent of each other.
"""
from .mechfile import Mechanism, read_mech, write_mech  # noqa: F401
from .mechgen import generate_h2_mechanism, H2_SPECIES  # noqa: F401
from . import fields  # noqa: F401
