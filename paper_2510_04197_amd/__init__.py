"""MI355X-native hot path of the DDF-QE discrete velocity Boltzmann method.

``dvbm`` is the ctypes binding of the HIP library ``libdvbm.so`` (C ABI in
``include/dvbm.h``); ``build`` compiles that library for gfx950.
"""

from .dvbm import (  # noqa: F401
    BC,
    KERNEL,
    STORAGE,
    VISC,
    DVBMError,
    Params,
    Solver,
    load_library,
    make_params,
    num_populations,
    velocity_set,
)
from .autograd import rollout_temperature  # noqa: F401
