"""Banded and low-rank terms in the refinement's residual, through the C ABI.

When the operator is created from host matrices, a real A_i whose nonzeros
lie within a band of half-width up to 64 is marked banded, and a real dense
A_i of numerical rank up to 96 is kept as G H^T (a randomized range finder,
accepted only at the rounding level of the entries).  The FP64 residual of
the mixed path (the split-form T(z_j) Y_j of eq. (sressplit)) then runs a
banded term over its band only and a low-rank one as G (H^T Y).  Moments
match the oracle's for a non-symmetric banded problem in both precisions, for
a problem with a rank-20 term, and for twins of both whose terms stay dense
(one negligible entry outside the band; a 1e-12 dense perturbation)."""
import numpy as np
import pytest

import oracle
import workloads as wl
from workloads import Contour, Problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def nep():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1910_11712_amd as P
    P.binding.lib()
    return P


def _band(rng, n, lo, up, scale):
    A = np.zeros((n, n))
    for k in range(-lo, up + 1):
        i = np.arange(max(0, -k), min(n, n - k))
        A[i, i + k] = scale * rng.standard_normal(len(i))
    return A


def _problem(n, dense_twin=False):
    """T(z) = B0 - z I + exp(-z) B1: B0 lower half-width 3, upper 5, with a
    diagonal spread over [1, 10]; B1 lower 2, upper 1."""
    rng = np.random.default_rng(11)
    B0 = _band(rng, n, 3, 5, 0.3) + np.diag(np.linspace(1.0, 10.0, n))
    B1 = _band(rng, n, 2, 1, 0.2)
    if dense_twin:
        B0 = B0.copy()
        B0[0, n - 1] = 1e-30  # outside every band: B0 stays dense
    fns = [wl.fn_rational([1.0]), wl.fn_rational([-1.0, 0.0]), wl.fn_exp(alpha=-1.0, beta=1.0)]
    return Problem("band", [B0, np.eye(n), B1], fns)


@pytest.mark.parametrize("dense_twin", [False, True])
@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_banded_terms_moments_match_oracle(nep, prec, dense_twin):
    n, N, L, K = 300, 32, 8, 2
    p = _problem(n, dense_twin)
    con = Contour.circle(5.05, 0.7)
    V = wl.probes(n, L, 5)
    op = nep.SplitOperator.from_problem(p)
    S, st = op.moments(con, nep.device_probes(V), N, L, K, prec=prec)
    Sg = nep.moments_to_numpy(S)
    So = oracle.ciss_moments(p, con, N, K, V)
    for q in range(2 * K):
        err = np.linalg.norm(Sg[q] - So[q]) / np.linalg.norm(So[q])
        print(prec, "dense twin" if dense_twin else "banded", q, f"{err:.2e}")
        assert err <= 1e-10, (q, err)
    if prec == "mixed":
        assert st["n_fallback"] == 0 and st["max_rel_residual"] <= 1e-14, st
    op.close()


def _lowrank_problem(n, dense_twin=False):
    """T(z) = B0 - z I + exp(-z) W with W = G G^T / r (r = 20, exactly low
    rank up to the rounding of its entries).  The twin adds a 1e-12 relative
    dense perturbation: far above rounding, so W stays a dense product."""
    rng = np.random.default_rng(13)
    B0 = _band(rng, n, 2, 2, 0.3) + np.diag(np.linspace(1.0, 10.0, n))
    G = rng.standard_normal((n, 20))
    W = G @ G.T / 20.0
    if dense_twin:
        E = rng.standard_normal((n, n))
        W = W + 1e-12 * np.abs(W).max() * (E + E.T)
    fns = [wl.fn_rational([1.0]), wl.fn_rational([-1.0, 0.0]), wl.fn_exp(alpha=-1.0, beta=1.0)]
    return Problem("lowrank", [B0, np.eye(n), 0.05 * W], fns)


@pytest.mark.parametrize("dense_twin", [False, True])
def test_low_rank_term_moments_match_oracle(nep, dense_twin):
    """A term W = G G^T of rank 20 runs in the mixed path's residual as
    G (G^T Y) / 20; its moments match the oracle's, as do those of the twin
    whose W the range finder must reject."""
    n, N, L, K = 600, 32, 8, 2
    p = _lowrank_problem(n, dense_twin)
    con = Contour.circle(5.05, 0.7)
    V = wl.probes(n, L, 6)
    op = nep.SplitOperator.from_problem(p)
    S, st = op.moments(con, nep.device_probes(V), N, L, K, prec="mixed")
    Sg = nep.moments_to_numpy(S)
    So = oracle.ciss_moments(p, con, N, K, V)
    for q in range(2 * K):
        err = np.linalg.norm(Sg[q] - So[q]) / np.linalg.norm(So[q])
        print("dense twin" if dense_twin else "low rank", q, f"{err:.2e}")
        assert err <= 1e-10, (q, err)
    assert st["n_fallback"] == 0 and st["max_rel_residual"] <= 1e-14, st
    op.close()
