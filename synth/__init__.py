"""Seeded synthetic LAPW+LO inputs shared by the CPU oracle and the GPU path.

This module only draws and lays out inputs (geometry, G+k sets, grids,
matching coefficients, muffin-tin blocks, start blocks, pulse samples).  It
performs none of the method's arithmetic: no operator is applied, no matrix is
projected and nothing is propagated here.
"""

from .lapw_inputs import (  # noqa: F401
    C_LIGHT,
    WORKLOADS,
    Atom,
    KPoint,
    System,
    make_system,
    pulse_samples,
    hat_weights,
    td_potential,
    potential_scale,
)
