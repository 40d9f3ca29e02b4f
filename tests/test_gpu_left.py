"""Left eigenvectors and the resolvent on the device, through the C ABI
(Section 2, eqs. (nep-left), (resolvent); Section 3.2.5): the adjoint
operator T^*, left eigenvectors by residual inverse iteration on it, the
moment path run on T^* (left eigenpairs as its right eigenpairs), the
Keldysh resolvent action and exact shifted solves."""
import numpy as np
import pytest
import scipy.linalg

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


def _dev(M):
    """numpy (n, m) -> device tensor (m, n) holding the column-major block."""
    return torch.from_numpy(np.ascontiguousarray(np.asarray(M, dtype=np.complex128).T)).to("cuda")


def _host(T):
    return T.cpu().numpy().T.copy()


def _delay_pairs(n=120):
    """A non-symmetric delay problem and oracle eigenvalues inside
    circle(-1, 0.4), polished by the oracle's RII to full accuracy."""
    p = wl.delay_problem(n, tau=1.0, seed=7)
    con = Contour.circle(-1.0, 0.4)
    S = oracle.ciss_moments(p, con, 32, 4, wl.probes(n, 8, 20))
    r = oracle.extract(p, con, S, 4)
    ins = r["inside"] & (r["eta"] < 1e-10)
    lam = np.array([oracle.rii_polish(p, l, x, 1e-15)[0] for l, x in zip(r["lam"][ins], r["X"][:, ins].T)])
    return p, con, lam


def test_adjoint_functions_and_left_eigenvectors(nep):
    B = nep.binding
    p, con, lam = _delay_pairs()
    n = p.n
    op = nep.SplitOperator.from_problem(p)
    adj = B.nep_split_adjoint(op.h)
    # f^*(z) = conj(f(conj z)) for every term
    z = np.array([-0.7 + 0.3j, 1.2 - 2.0j, 0.1 + 0.05j])
    got = B.nep_fn_eval(adj, p.ell, z)
    for i, f in enumerate(p.fns):
        ref = np.array([np.conj(oracle.fn_value(f, np.conj(zz))) for zz in z])
        assert np.max(np.abs(got[i] - ref) / np.abs(ref)) < 1e-14
    # left eigenvectors from random start vectors
    rng = np.random.default_rng(31)
    Y0 = rng.standard_normal((n, len(lam))) + 1j * rng.standard_normal((n, len(lam)))
    Yd = _dev(Y0)
    lam_l, eta = B.nep_left_eigenvectors(op.h, lam, Yd, max_it=10)
    print("left eta", eta)
    assert np.all(eta <= 1e-12)
    Y = _host(Yd)
    for k, l in enumerate(lam):
        assert abs(lam_l[k] - l) <= 1e-10 * abs(l)
        y_ref = oracle.left_eigenvector(p, l)
        assert np.linalg.norm(Y[:, k] - y_ref) < 1e-8, (k, np.linalg.norm(Y[:, k] - y_ref))
        res = Y[:, k].conj() @ oracle.t_matrix(p, l)
        assert np.abs(res).max() <= 1e-12 * sum(np.abs(A).sum(axis=0).max() for A in p.mats)
    B.nep_split_destroy(adj)
    op.close()


def test_moments_on_the_adjoint(nep):
    """The whole moment path and the extraction on T^* with the conjugated
    contour return conj of T's eigenvalues and T's left eigenvectors."""
    B = nep.binding
    p, con, lam = _delay_pairs()
    op = nep.SplitOperator.from_problem(p)
    adj_h = B.nep_split_adjoint(op.h)
    conj_con = Contour.circle(np.conj(con.c), con.rho)
    N, L, K = 32, 8, 4
    V = wl.probes(p.n, L, 21)
    S = torch.empty((2 * K, L, p.n), dtype=torch.complex128, device="cuda")
    B.nep_ciss_moments(adj_h, conj_con, B.opts_struct(N, L, K, "mixed"), nep.device_probes(V), S)
    X = torch.zeros((64, p.n), dtype=torch.complex128, device="cuda")
    r = B.nep_extract(adj_h, conj_con, B.opts_struct(N, L, K, "mixed"), S, X, max_eigs=64, eta_tol=1e-10)
    got = np.conj(r["lam"][r["inside"]])
    assert len(got) == len(lam)
    Y = _host(X)[:, :r["m"]][:, r["inside"]]
    for l in lam:
        k = int(np.argmin(np.abs(got - l)))
        assert abs(got[k] - l) <= 1e-10 * abs(l)
        assert np.linalg.norm(Y[:, k] - oracle.left_eigenvector(p, l)) < 1e-8
    B.nep_split_destroy(adj_h)
    op.close()


def test_keldysh_resolvent_linear_full_spectrum(nep):
    """T(z) = A - z I, n = 12, every eigenvalue inside the contour: right
    eigenvectors from the moment path, left ones from RII on T^*, and the
    Keldysh sum equals (A - z I)^{-1} V (R = 0) and the oracle's sum."""
    B = nep.binding
    rng = np.random.default_rng(33)
    n = 12
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    p = Problem("linear", [A, np.eye(n)], [wl.fn_rational([1.0]), wl.fn_rational([-1.0, 0.0])])
    ev = scipy.linalg.eigvals(A)
    con = Contour.circle(0.0, 1.5 * np.abs(ev).max())
    op = nep.SplitOperator.from_problem(p)
    N, L, K = 64, 8, 2
    S, st = op.moments(con, nep.device_probes(wl.probes(n, L, 3)), N, L, K, prec="fp64")
    r = op.extract(con, S, N, L, K, prec="fp64", max_eigs=16, eta_tol=1e-10)
    assert r["inside"].sum() == n
    lam = r["lam"][r["inside"]]
    Xd = _dev(r["X"][:, r["inside"]])
    Yd = _dev(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    lam_l, eta_l = B.nep_left_eigenvectors(op.h, lam, Yd, max_it=10)
    assert np.all(eta_l <= 1e-12)
    z = 0.3 + 0.25j * np.abs(ev).max()
    V = rng.standard_normal((n, 3)) + 1j * rng.standard_normal((n, 3))
    Wd = torch.zeros((3, n), dtype=torch.complex128, device="cuda")
    B.nep_apply_resolvent(op.h, lam, Xd, Yd, z, _dev(V), Wd)
    W = _host(Wd)
    ref = np.linalg.solve(A - z * np.eye(n), V)
    assert np.linalg.norm(W - ref) <= 1e-10 * np.linalg.norm(ref), np.linalg.norm(W - ref) / np.linalg.norm(ref)
    Wo = oracle.apply_resolvent(p, lam, _host(Xd), _host(Yd), z, V)
    assert np.linalg.norm(W - Wo) <= 1e-10 * np.linalg.norm(Wo)
    op.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_solve_at_points(nep, prec):
    """T(z_k)^{-1} V at explicit points (the full resolvent) against the
    oracle's LAPACK solves, both precisions (the mixed path refined to a
    normwise backward error of 1e-15)."""
    B = nep.binding
    p = wl.delay_problem(200, tau=1.0, seed=3)
    op = nep.SplitOperator.from_problem(p)
    z = np.array([-1.0 + 0.5j, 0.3 - 0.2j, 2.0 + 1.0j, -2.5 + 0.1j, 0.9j])
    L = 4
    V = wl.probes(p.n, L, 12)
    Y = torch.zeros((len(z), L, p.n), dtype=torch.complex128, device="cuda")
    st = B.nep_solve_at(op.h, z, nep.device_probes(V), Y, prec=prec)
    assert st["n_unconverged"] == 0
    Yh = Y.cpu().numpy()
    for k, zk in enumerate(z):
        T = oracle.t_matrix(p, zk)
        ref = np.linalg.solve(T, V)
        got = Yh[k].T
        kappa = np.linalg.cond(T)
        bound = max(1e-12, 100 * kappa * 1.1e-16 if prec == "fp64" else 10 * kappa * 1e-15)
        assert np.linalg.norm(got - ref) <= bound * np.linalg.norm(ref), (k, np.linalg.norm(got - ref) / np.linalg.norm(ref), kappa)
    op.close()
