"""Seeded synthetic inputs for the split-form contour-integral moment path.

This package holds problem *data* only: the coefficient matrices A_i, the
scalar-function descriptors f_i (FN semantics), the contours and the probe
blocks V.  It contains none of the method's arithmetic (no quadrature, no
solves, no moments); both the FP64 oracle and the HIP path consume what it
builds.
"""
from .fn import (fn_rational, fn_exp, fn_log, fn_sqrt, fn_invsqrt, fn_phi,
                 fn_combine, COMB_ADD, COMB_MUL, COMB_DIV, COMB_COMPOSE)
from .problems import (Problem, Contour, probes, config0, config1, config2,
                       config3, config4_stream, loaded_string, delay_problem,
                       sqrt_problem, build_operator, CONFIGS)

__all__ = [
    "fn_rational", "fn_exp", "fn_log", "fn_sqrt", "fn_invsqrt", "fn_phi",
    "fn_combine", "COMB_ADD", "COMB_MUL", "COMB_DIV", "COMB_COMPOSE",
    "Problem", "Contour", "probes", "config0", "config1", "config2",
    "config3", "config4_stream", "loaded_string", "delay_problem",
    "sqrt_problem", "build_operator", "CONFIGS",
]
