"""MI355X (gfx950) closed-form ADMM for linearized multi-phase OPF.

The solver lives in the HIP/C++ library ``libldopf.so`` (C ABI in
include/ldopf.h); ``ldopf`` is its Python binding.
"""
from .ldopf import (LdopfError, Network, Problem, ldopf_create, ldopf_create_lp,  # noqa: F401
                    ldopf_default_options, ldopf_describe_network)
