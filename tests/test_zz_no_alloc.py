"""nep_backward_error_noalloc (the allocation-free variant of
nep_backward_error, with its device scratch in a library-owned array)
against nep_backward_error, through the C ABI: two calls in a row, the
second with a smaller input, each equal to the allocating entry point's
result; and the size limits are refused before any device work."""
import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def nep():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1910_11712_amd as P
    P.binding.lib()
    return P


def _pairs(rng, n, m, c, r):
    lam = c + r * (rng.standard_normal(m) + 1j * rng.standard_normal(m))
    X = rng.standard_normal((n, m)) + 1j * rng.standard_normal((n, m))
    return lam, torch.from_numpy(np.ascontiguousarray(X.T)).to("cuda")


def test_noalloc_equals_backward_error(nep):
    B = nep.binding
    rng = np.random.default_rng(21)
    p = wl.sqrt_problem(300, seed=4)          # complex terms, square roots
    q = wl.loaded_string(120, sigma=1.2)      # real terms, a rational one
    op_p = nep.SplitOperator.from_problem(p)
    op_q = nep.SplitOperator.from_problem(q)
    cases = [(op_p, 40, 22600.0, 3000.0),     # first call: n=300, m=40
             (op_p, 7, 22600.0, 3000.0),      # second call, smaller m on the same handle
             (op_q, 3, 100.0, 50.0)]          # third, smaller n and m on another handle
    for op, m, c, r in cases:
        lam, Xd = _pairs(rng, op.n, m, c, r)
        ref = B.nep_backward_error(op.h, lam, Xd)
        got = B.nep_backward_error_noalloc(op.h, lam, Xd)
        print(op.n, m, np.max(np.abs(got - ref) / ref))
        assert np.all(np.isfinite(ref)) and np.all(ref > 0)
        # same kernels on the same inputs: the same bits
        assert np.array_equal(got, ref), (op.n, m, got, ref)


def test_noalloc_limits(nep):
    B = nep.binding
    op = nep.SplitOperator.from_problem(wl.loaded_string(2048, sigma=1.0))
    lam = np.full(200, 100.0 + 0j)
    Xd = torch.zeros((200, 2048), dtype=torch.complex128, device="cuda")
    with pytest.raises(B.NepError) as ei:       # n*m = 409600 > 262144
        B.nep_backward_error_noalloc(op.h, lam, Xd)
    assert ei.value.name == "NEP_ERR_ARG"
    lam = np.full(257, 100.0 + 0j)
    Xd = torch.zeros((257, 2048), dtype=torch.complex128, device="cuda")
    with pytest.raises(B.NepError) as ei:       # m > 256
        B.nep_backward_error_noalloc(op.h, lam, Xd)
    assert ei.value.name == "NEP_ERR_ARG"
