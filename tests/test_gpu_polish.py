"""FP64 eigenpair polish by residual inverse iteration (Section 4.1,
Algorithm "RII") on the device, through the C ABI, and the FN derivatives it
uses (FNEvaluateDerivative, Section 3.2.2).

Quadrature-limited pairs are made by a loose rank tolerance (1e-6): the
weakly filtered outside eigenvalues are truncated from the moments, which
leaves the inside pairs at eta ~ 1e-9 .. 1e-7.  Polish must take them to
eta <= 1e-12, to the closed-form eigenvalues (secular equation) and to the
oracle's own RII-polished eigenvalues to 1e-10.
"""
import numpy as np
import pytest

import oracle
import workloads as wl
from closed_forms import string_secular_roots
from workloads import Contour

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def nep():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1910_11712_amd as P
    P.binding.lib()
    return P


def test_fn_derivative_matches_oracle(nep):
    rng = np.random.default_rng(3)
    z = rng.standard_normal(64) * 40 + 1j * rng.standard_normal(64) * 40 + 100
    fns = [wl.fn_rational([1.0, -2.0, 3.0], [1.0, 0.5j]), wl.fn_exp(alpha=-0.7 + 0.1j, beta=2.0),
           wl.fn_log(), wl.fn_sqrt(beta=1j), wl.fn_invsqrt(alpha=2.0),
           wl.fn_phi(0), wl.fn_phi(1), wl.fn_phi(3, alpha=0.01),
           wl.fn_combine(wl.COMB_COMPOSE, wl.fn_rational([1.0, -108.8 ** 2]), wl.fn_sqrt(), beta=1j),
           wl.fn_combine(wl.COMB_DIV, wl.fn_exp(alpha=0.01), wl.fn_rational([1.0, 3.0])),
           wl.fn_combine(wl.COMB_MUL, wl.fn_rational([-1.0, 0.0]), wl.fn_exp(alpha=-0.05)),
           wl.fn_combine(wl.COMB_ADD, wl.fn_log(), wl.fn_sqrt())]
    op = nep.SplitOperator([np.eye(3)] * len(fns), fns)
    got = op.fn_eval_derivative(z)
    for i, f in enumerate(fns):
        ref = np.array([oracle.fn_derivative(f, zz) for zz in z])
        assert np.max(np.abs(got[i] - ref) / np.maximum(np.abs(ref), 1e-300)) < 1e-13, i
    op.close()


def _inside(con, lam):
    mu = (np.asarray(lam) - con.c) / con.rho
    return np.abs(mu) < 1.0 if con.kind == 0 else mu.real ** 2 + (mu.imag / con.v) ** 2 < 1.0


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_polish_quadrature_limited_string(nep, prec):
    cfg = wl.config0()
    p, con, N, L, K = cfg["problem"], cfg["contour"], cfg["N"], cfg["L"], cfg["K"]
    op = nep.SplitOperator.from_problem(p)
    S, st = op.moments(con, nep.device_probes(cfg["V"]), N, L, K, prec=prec)
    r0 = op.extract(con, S, N, L, K, prec=prec, max_eigs=16, rank_tol=1e-6, eta_tol=1e-10)
    ins0 = _inside(con, r0["lam"])
    print("unpolished eta", r0["eta"][ins0])
    assert ins0.sum() == 3 and np.max(r0["eta"][ins0]) > 1e-9   # quadrature-limited
    r = op.extract(con, S, N, L, K, prec=prec, max_eigs=16, rank_tol=1e-6, eta_tol=1e-10, polish_its=5)
    ins = r["inside"]
    print("polished eta", r["eta"][ins])
    assert ins.sum() == 3 and np.all(r["eta"][ins] <= 1e-12)
    roots = string_secular_roots(200, 1.0, 10.0, 190.0)
    got = np.sort(r["lam"][ins].real)
    assert np.max(np.abs(got - roots) / roots) <= 1e-12, (got, roots)
    assert np.all(np.abs(r["lam"][ins].imag) <= 1e-12 * np.abs(r["lam"][ins]))
    # the oracle's RII from the oracle's own quadrature-limited pairs
    So = oracle.ciss_moments(p, con, N, K, cfg["V"])
    ro = oracle.extract(p, con, So, K, rank_tol=1e-6)
    ref = []
    for lam0, x0 in zip(ro["lam"][_inside(con, ro["lam"])], ro["X"][:, _inside(con, ro["lam"])].T):
        lam, x, eta, k = oracle.rii_polish(p, lam0, x0, 1e-14)
        ref.append(lam)
    ref = np.sort(np.real(ref))
    assert np.max(np.abs(got - ref) / ref) <= 1e-10, (got, ref)
    # polished eigenvectors: unit norm, same normalization as the oracle's
    for lam, x in zip(r["lam"][ins], r["X"][:, ins].T):
        assert abs(np.linalg.norm(x) - 1.0) < 1e-13
        k = int(np.argmax(np.abs(x)))
        assert abs(x[k].imag) < 1e-14 and x[k].real > 0
    op.close()


def test_rii_polish_entry_point_delay_and_sqrt(nep):
    """nep_rii_polish on given pairs: the delay problem's quadrature-limited
    pairs, and perturbed eigenpairs of the square-root problem (complex T,
    sqrt terms), each against the oracle's RII from the same start."""
    p = wl.delay_problem(120, tau=1.0, seed=7)
    con = Contour.circle(-1.0, 0.4)
    V = wl.probes(120, 8, 20)
    So = oracle.ciss_moments(p, con, 32, 4, V)
    ro = oracle.extract(p, con, So, 4, rank_tol=1e-6)
    ins = _inside(con, ro["lam"])
    lam0, X0 = ro["lam"][ins], ro["X"][:, ins]
    assert len(lam0) >= 3 and np.max(ro["eta"][ins]) > 1e-10
    op = nep.SplitOperator.from_problem(p)
    Xd = torch.from_numpy(np.ascontiguousarray(X0.T)).to("cuda")
    lam, eta, its = op.rii_polish(lam0, Xd, tol=1e-14, max_it=8)
    print("delay polished", eta, its)
    assert np.all(eta <= 1e-12) and np.all(its >= 1)
    for l0, x0, l in zip(lam0, X0.T, lam):
        lo, xo, eo, ko = oracle.rii_polish(p, l0, x0, 1e-14)
        assert abs(l - lo) <= 1e-10 * abs(lo), (l, lo)
    eta_check = oracle.backward_error(p, lam, Xd.cpu().numpy().T)
    assert np.all(eta_check <= 1e-12)
    op.close()
    # square root problem: eigenpairs of the n=256 version, perturbed
    q = wl.sqrt_problem(256, seed=5)
    con2 = Contour.ellipse(22600.0, 1000.0, 1.0 / 3.0)
    V2 = wl.probes(256, 16, 9)
    S2 = oracle.ciss_moments(q, con2, 48, 2, V2)
    r2 = oracle.extract(q, con2, S2, 2)
    good = r2["inside"] & (r2["eta"] < 1e-12)
    assert good.sum() >= 2
    rng = np.random.default_rng(8)
    lam0 = r2["lam"][good] * (1 + 1e-7 * rng.standard_normal(good.sum()))
    X0 = r2["X"][:, good] + 1e-5 * (rng.standard_normal((256, good.sum())) + 1j * rng.standard_normal((256, good.sum())))
    op2 = nep.SplitOperator.from_problem(q)
    Xd2 = torch.from_numpy(np.ascontiguousarray(X0.T)).to("cuda")
    lam, eta, its = op2.rii_polish(lam0, Xd2, tol=1e-14, max_it=8)
    print("sqrt polished", eta, its)
    assert np.all(eta <= 1e-12)
    for l0, x0, l in zip(lam0, X0.T, lam):
        lo, xo, eo, ko = oracle.rii_polish(q, l0, x0, 1e-14)
        assert abs(l - lo) <= 1e-10 * abs(lo), (l, lo)
    op2.close()
