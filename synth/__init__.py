"""Seeded synthetic initial fields shared by the oracle checks, the tests and the benchmark.

This package only builds macroscopic initial conditions (density, velocity,
temperature on a uniform grid). It contains none of the kinetic method's
arithmetic: no populations, moments, equilibria or fluxes.
"""

from .fields import (  # noqa: F401
    Workload,
    acoustic_wave,
    gaussian_bump,
    isentropic_vortex,
    shear_wave,
    shock_vortex,
    smooth_random,
    sod_tube,
    thermal_wave,
    thermal_wave_1d,
    rankine_hugoniot,
    uniform,
)
