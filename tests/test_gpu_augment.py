"""Work on resident factors through the C ABI: moments of further probe
blocks without refactoring, probe augmentation when the moments' rank
saturates, and the eigenvalue count by the argument principle from the LU
log-determinants (eigenvalues are the zeros of det T, eq. (nep))."""
import os

import numpy as np
import pytest

import oracle
import workloads as wl
from workloads import Contour

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "cfg2_sqrt_n4096_oracle.npz")


@pytest.fixture(scope="module")
def nep():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1910_11712_amd as P
    P.binding.lib()
    return P


def _match(got, ref, tol):
    got = list(np.asarray(got))
    assert len(got) == len(ref), (np.sort_complex(np.asarray(got)), np.sort_complex(np.asarray(ref)))
    for r in ref:
        k = int(np.argmin([abs(g - r) for g in got]))
        assert abs(got[k] - r) <= tol * abs(r), (got[k], r)
        got.pop(k)


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_moments_more_on_resident_factors(nep, prec):
    """Moments of a second probe block on the resident factors equal a fresh
    call's bit for bit, land in the requested columns of an augmented moment
    array, and match the oracle."""
    B = nep.binding
    cfg = wl.config0()
    p, con, N, L, K = cfg["problem"], cfg["contour"], cfg["N"], cfg["L"], cfg["K"]
    V1, V2 = wl.probes(p.n, L, 0), wl.probes(p.n, L, 1)
    op = nep.SplitOperator.from_problem(p)
    op.moments(con, nep.device_probes(V1), N, L, K, prec=prec)
    Saug = torch.zeros((2 * K, 2 * L, p.n), dtype=torch.complex128, device="cuda")
    st = B.nep_ciss_moments_more(op.h, nep.device_probes(V2), Saug, s_stride=2 * L * p.n, offset=L * p.n)
    assert st["n_unconverged"] == 0 and st["ms_lu"] == 0.0, st   # no factorization in this call
    S2 = nep.moments_to_numpy(Saug)[:, :, L:]
    op2 = nep.SplitOperator.from_problem(p)
    S2ref, _ = op2.moments(con, nep.device_probes(V2), N, L, K, prec=prec)
    assert np.array_equal(S2, nep.moments_to_numpy(S2ref))
    assert np.all(nep.moments_to_numpy(Saug)[:, :, :L] == 0)    # other columns untouched
    So = oracle.ciss_moments(p, con, N, K, V2)
    for q in range(2 * K):
        assert np.linalg.norm(S2[q] - So[q]) <= 1e-10 * np.linalg.norm(So[q])
    op.close()
    op2.close()


def test_eigs_probe_augmentation_and_count(nep):
    """Delay problem with 9 eigenvalues inside circle(-1, 0.6) and K = 2:
    8 and then 16 probes saturate the moments' rank; nep_eigs solves further
    probe blocks on the resident factors until 24 resolve them, and its
    eigenvalues equal the oracle's from the same 24 probes.  The argument
    principle count from the factors at 256 nodes is 9, the oracle's too."""
    B = nep.binding
    p = wl.delay_problem(120, tau=1.0, seed=7)
    con = Contour.circle(-1.0, 0.6)
    N, L, K, Lmax = 32, 8, 2, 32
    V = wl.probes(120, Lmax, 20)
    op = nep.SplitOperator.from_problem(p)
    X = torch.zeros((64, 120), dtype=torch.complex128, device="cuda")
    r = B.nep_eigs(op.h, con, B.opts_struct(N, L, K, "mixed"), nep.device_probes(V), Lmax, X, max_eigs=64,
                   eta_tol=1e-10)
    print("L_used", r["L_used"], "m", r["m"], "inside", r["inside"].sum())
    assert r["L_used"] == 24
    So = oracle.ciss_moments(p, con, N, K, V[:, :24])
    ro = oracle.extract(p, con, So, K)
    assert r["m"] == ro["m"]
    ref = ro["lam"][ro["inside"] & (ro["eta"] <= 1e-10)]
    assert len(ref) == 9
    _match(r["lam"][r["inside"]], ref, 1e-10)
    assert np.all(r["eta"][r["inside"]] <= 1e-10)
    cnt, step, w = B.nep_count_eigs(op.h, con, 256, "mixed")
    co, so, wo = oracle.eigenvalue_count(p, con, 256)
    print("count", cnt, step, w, "oracle", co, so, wo)
    assert cnt == co == 9 and step < 2.5
    # from the factors resident after a moments call at 256 nodes
    op.moments(con, nep.device_probes(V[:, :8]), 256, 8, 2, prec="fp64")
    c2, s2, w2 = B.nep_ciss_count(op.h)
    assert c2 == 9 and abs(w2 - wo) < 1e-6, (c2, w2, wo)
    op.close()


def test_count_full_size_sqrt(nep):
    """The square-root workload at n=4096: the argument-principle count from
    complex-FP32 factors at 256 nodes equals the number of eigenvalues the
    oracle's extraction finds inside the ellipse."""
    B = nep.binding
    g = np.load(GOLDEN, allow_pickle=False)
    cfg = wl.config2()
    p, con = cfg["problem"], cfg["contour"]
    mu = (g["lam"] - con.c) / con.rho
    n_inside = int(np.sum(mu.real ** 2 + (mu.imag / con.v) ** 2 < 1.0))
    op = nep.SplitOperator.from_problem(p)
    cnt, step, w = B.nep_count_eigs(op.h, con, 256, "mixed")
    print("count", cnt, "max step", step, "winding", w, "oracle inside", n_inside)
    assert cnt == n_inside and abs(w - cnt) < 1e-3
    op.close()
