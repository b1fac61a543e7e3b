"""Seeded synthetic inputs (feeders, load scenarios, request streams).

Shared by the CPU oracle and the GPU library's tests and benchmark; holds no
solver arithmetic.
"""
from .feeder import (SPECS, DEFAULT_SEEDS, FeederSpec, make_feeder, scale_loads,
                     scenario_factors, two_bus, perturb_extras)

__all__ = ["SPECS", "DEFAULT_SEEDS", "FeederSpec", "make_feeder", "scale_loads",
           "scenario_factors", "two_bus", "perturb_extras"]
