"""Restarted PDHG for LP (arXiv 2311.12180) on one AMD MI355X.

The solver is the HIP library ``libpdlp_hip.so`` (C ABI: include/pdlp.h);
``paper_2311_12180_amd.pdlp`` is its Python binding with the same names.
"""
from . import pdlp  # noqa: F401
from .pdlp import (PdlpError, pdlp_create, pdlp_default_options, pdlp_destroy, pdlp_get_iterate,  # noqa: F401
                   pdlp_get_scaling, pdlp_get_solution, pdlp_get_trace, pdlp_last_error,
                   pdlp_profile_attempts, pdlp_set_termination, pdlp_set_warm_start, pdlp_solve, pdlp_step_bytes, solve)
