"""Seeded synthetic inputs shared by the CPU oracle, the tests and the benchmark.

This package only draws numbers: vibronic coupling constants, site orderings,
initial occupations and random tensors.  It contains none of the arithmetic of
the time-evolution method itself (no operators, no MPO, no contractions), so
that the oracle and the HIP path stay independent of each other.
"""
from .vibronic import (  # noqa: F401
    AU_TIME_FS,
    HBAR_EV_FS,
    config1_model,
    config2_model,
    config3_model,
    config5_model,
    debye_bath,
    sf_table1_model,
    per_state_model,
    superposed_excitation_state,
    lvc4_per_state_model,
    single_mode_model,
    site_dims,
    rabi_model,
)
from .tensors import heff_problem, heff_batch_shapes  # noqa: F401
