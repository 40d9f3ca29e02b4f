"""FP64 CPU oracle for the contour-integral moment path and for NLEIGS
(submodule `oracle.nleigs`) -- TEST INFRASTRUCTURE.

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  The product path (the HIP library and its
Python binding) never imports, calls or links anything here, and shares no
code with it: the only common dependency is the seeded input generator
package `workloads`, which holds no arithmetic of the method.
"""
from .ciss import (NotHolomorphic, SingularNode, RankSaturated, fn_value, fn_derivative,
                   quadrature, t_matrix, node_solve, ciss_moments,
                   block_hankel, extract, backward_error, relative_residual,
                   inside_mask, t_derivative, rii_polish, eigenvalue_count,
                   left_eigenvector, apply_resolvent)

__all__ = ["NotHolomorphic", "SingularNode", "RankSaturated", "fn_value", "fn_derivative",
           "quadrature", "t_matrix", "node_solve", "ciss_moments",
           "block_hankel", "extract", "backward_error", "relative_residual",
           "inside_mask", "t_derivative", "rii_polish", "eigenvalue_count",
           "left_eigenvector", "apply_resolvent"]
