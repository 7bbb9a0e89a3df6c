"""Seeded synthetic Bethe-Salpeter inputs.

This module only draws random numbers and assembles input matrices. It holds
none of the solver's arithmetic, so both the CPU oracle and the GPU path can
use it without sharing any part of the method.
"""

from .generators import (  # noqa: F401
    BseProblem,
    gen_bse,
    gen_closed_form,
    gen_b_zero,
    gen_real,
    gen_real_closed_form,
    gen_not_definite,
    batched_sizes,
    serving_stream,
    omega_is_positive_definite,
)
