"""MI355X contour-integral moments for split-form nonlinear eigenproblems.

The product is the HIP library libnep.so (C ABI in include/nep.h).  This
package is its thin Python binding: `binding` mirrors the C entry points
(same names) and `SplitOperator` wraps a handle for convenience.  PyTorch is
used for device memory and streams only.
"""
import numpy as np

from . import binding
from .binding import (NepError, nep_split_create, nep_split_destroy, nep_ciss_moments, nep_ciss_wait,
                      nep_extract, nep_backward_error, nep_fn_eval, opts_struct, contour_struct)

__all__ = ["NepError", "SplitOperator", "binding", "nep_split_create", "nep_split_destroy",
           "nep_ciss_moments", "nep_ciss_wait", "nep_extract", "nep_backward_error", "nep_fn_eval",
           "device_probes", "moments_to_numpy", "Server"]


def device_probes(V, device="cuda"):
    """numpy (n x L) complex -> CUDA tensor holding the column-major block."""
    import torch
    V = np.asarray(V, dtype=np.complex128)
    return torch.from_numpy(np.ascontiguousarray(V.T)).to(device)


def moments_to_numpy(S):
    """CUDA tensor (2K, L, n) of column-major blocks -> numpy (2K, n, L)."""
    return np.ascontiguousarray(S.cpu().numpy().transpose(0, 2, 1))


class SplitOperator:
    """T(z) = sum_i f_i(z) A_i held on the device (nep_split handle)."""

    def __init__(self, mats, fns, stream=None):
        self.n = int(mats[0].shape[0])
        self.ell = len(mats)
        self.h = nep_split_create(mats, fns, stream)

    @classmethod
    def from_problem(cls, problem, stream=None):
        return cls(problem.mats, problem.fns, stream)

    def close(self):
        if self.h is not None and self.h.value:
            nep_split_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def moments(self, contour, V, N, L, K, prec="mixed", max_refine=None, fallback=True, tol=0.0, S=None,
                sync=True, stream=None):
        """Returns (S tensor (2K, L, n), stats).  V: CUDA tensor (L, n)."""
        import torch
        if S is None:
            S = torch.empty((2 * K, L, self.n), dtype=torch.complex128, device=V.device)
        o = opts_struct(N, L, K, prec, max_refine, fallback, tol, stream)
        st = nep_ciss_moments(self.h, contour, o, V, S, sync=sync)
        return S, st

    def wait(self):
        return nep_ciss_wait(self.h)

    def extract(self, contour, S, N, L, K, prec="mixed", max_eigs=64, rank_tol=0.0, X=None, stream=None,
                eta_tol=0.0, polish_its=0):
        import torch
        if X is None:
            X = torch.zeros((max_eigs, self.n), dtype=torch.complex128, device=S.device)
        o = opts_struct(N, L, K, prec, None, True, 0.0, stream)
        r = nep_extract(self.h, contour, o, S, X, max_eigs, rank_tol, eta_tol, polish_its)
        r["X_dev"] = X
        r["X"] = X[: r["m"]].cpu().numpy().T.copy()
        return r

    def backward_error(self, lam, X):
        return nep_backward_error(self.h, lam, X)

    def rii_polish(self, lam, X, tol=0.0, max_it=10):
        """X: device tensor (m, n) holding the eigenvectors; polished in place."""
        return binding.nep_rii_polish(self.h, lam, X, tol, max_it)

    def nleigs_interp(self, contour, dmax=50, npts=1024, tol=0.0, xi=()):
        return binding.nep_nleigs_interp(self.h, contour, dmax, npts, tol, xi)

    def nleigs(self, contour, W0, X, sigma, k, dmax=50, npts=1024, tol=0.0, xi=(), eta_tol=0.0, max_eigs=64,
               want_H=False):
        """NLEIGS eigenpairs near sigma inside contour (see nep_nleigs)."""
        return binding.nep_nleigs(self.h, contour, W0, X, sigma, k, dmax, npts, tol, xi, eta_tol, max_eigs,
                                  want_H)

    def fn_eval(self, z):
        return nep_fn_eval(self.h, self.ell, z)

    def fn_eval_derivative(self, z):
        return binding.nep_fn_eval_derivative(self.h, self.ell, z)


class Server:
    """Query server over the C ABI: submit (operator, contour, probes) and
    collect eigenvalues inside the contour; queries sharing (N, L, K,
    precision) are batched and run on several streams at once."""

    def __init__(self, hbm_budget, max_inflight=64, nstreams=4):
        self.s = binding.nep_server_create(hbm_budget, max_inflight, nstreams)
        self._out = {}

    def submit(self, op, contour, V, N, L, K, prec="mixed", max_eigs=64, want_X=False, rank_tol=0.0,
               eta_tol=0.0):
        o = binding.opts_struct(N, L, K, prec)
        t, out = binding.nep_server_submit(self.s, op.h, contour, o, V, max_eigs, rank_tol, want_X, eta_tol)
        self._out[t] = out
        return t

    def poll(self, ticket):
        r = binding.nep_server_poll(self.s, ticket, self._out[ticket])
        if r is not None:
            del self._out[ticket]
        return r

    def wait(self, ticket):
        r = binding.nep_server_wait(self.s, ticket, self._out[ticket])
        del self._out[ticket]
        return r

    def clock(self):
        return binding.nep_server_clock(self.s)

    def close(self):
        if self.s is not None and self.s.value:
            binding.nep_server_destroy(self.s)
        self.s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
