"""Seeded synthetic reservoir models (inputs only).

This package builds the discrete problems that both the FP64 oracle and the
HIP library consume: cells with pore volumes and depths, two-point
connections with their transmissibilities (Cartesian TPFA plus embedded
discrete fractures), well perforations, fluid parameters, initial states and
timestep schedules.  It contains none of the solver's arithmetic: no
residual, Jacobian, Newton, Krylov or active-set logic lives here.

The paper describes its models only through stripped figures and Table 1, so
every workload is a synthetic stand-in built from a seed.
"""
from .units import PSI, MD, DAY, CP, GRAV
from .model import Model, FLUID_SINGLE, FLUID_DEADOIL, FLUID_BLACKOIL
from .configs import (make_c1, make_c2, make_c3, make_c4_member, make_tiny,
                      make_chain, make_c1_variant, make_small_c2, make_small_c3,
                      c1_schedule, geometric_schedule)

__all__ = [
    "PSI", "MD", "DAY", "CP", "GRAV", "Model", "FLUID_SINGLE", "FLUID_DEADOIL",
    "FLUID_BLACKOIL", "make_c1", "make_c2", "make_c3", "make_c4_member",
    "make_tiny", "make_chain", "make_c1_variant", "make_small_c2",
    "make_small_c3", "c1_schedule", "geometric_schedule",
]
