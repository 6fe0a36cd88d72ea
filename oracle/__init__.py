"""FP64 CPU reference for the NEP loss-and-gradient hot path.

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the
benchmark's CPU-baseline leg; the library never imports it.
"""
from .nep_oracle import (NEPOracle, Sizes, adam_step, four_body, five_body, lr_schedule,
                         neighbor_pairs, radial_functions, chebyshev, cutoff, unpack, voigt)
from . import harmonics
