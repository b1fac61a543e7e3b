"""MI355X (gfx950) closed-form ADMM for linearized multi-phase OPF.

The solver lives in the HIP/C++ library ``libldopf.so`` (C ABI in
include/ldopf.h); ``ldopf`` is its Python binding.
"""
from .ldopf import (Batch, LdopfError, Network, Problem, Server, ldopf_batch_create, ldopf_create,  # noqa: F401
                    ldopf_create_lp, ldopf_default_options, ldopf_describe_network, ldopf_request_estimate,
                    ldopf_solve_many)
