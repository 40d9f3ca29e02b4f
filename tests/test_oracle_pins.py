"""Pins of the FP64 oracle against facts fixed by the paper and by
mathematics, independent of the oracle's own code.

Each test names what it pins.  A plausible mistake in the oracle (a dropped
term, a wrong sign, a transposed operand, a wrong node offset or weight, a
wrong branch) fails at least one of them.
"""
import cmath
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg
import scipy.special

import oracle
import workloads as wl
from closed_forms import string_secular_roots
from workloads import Contour, Problem

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# FN semantics (Section 3.2.2)
# ---------------------------------------------------------------------------

def test_fig_split_worked_example():
    """Figure 'split': coefficients highest degree first; FNSetScale(-tau,1)."""
    with open(os.path.join(GOLDEN, "fig_split_fn.json")) as fh:
        g = json.load(fh)
    tau = g["tau_paper"]
    f1, f2, f3 = g["functions"]
    d1 = wl.fn_rational(f1["num"])
    d2 = wl.fn_rational(f2["num"])
    d3 = wl.fn_exp(alpha=-tau, beta=f3["beta"])
    for z in [0.3, -2.0 + 1.5j, 7.0 - 3.0j, 1e3 + 1j]:
        assert oracle.fn_value(d1, z) == -z
        assert oracle.fn_value(d2, z) == 1.0
        assert abs(oracle.fn_value(d3, z) - cmath.exp(-tau * z)) <= 1e-15 * abs(cmath.exp(-tau * z))


def test_rational_horner_order_and_scale():
    # (2x^2 - 3x + 1)/(x + 4), with alpha and beta scaling: beta*g(alpha*z)
    d = wl.fn_rational([2.0, -3.0, 1.0], [1.0, 4.0], alpha=0.5j, beta=-2.0)
    for z in [1.0, 2.0 - 1.0j, -3.5 + 0.25j]:
        x = 0.5j * z
        ref = -2.0 * (2 * x * x - 3 * x + 1) / (x + 4)
        assert abs(oracle.fn_value(d, z) - ref) <= 1e-14 * abs(ref)


def test_sqrt_log_principal_branch():
    rng = np.random.default_rng(5)
    pts = rng.standard_normal(50) * 10 + 1j * rng.standard_normal(50) * 10
    for z in pts:
        assert abs(oracle.fn_value(wl.fn_sqrt(), z) - cmath.sqrt(z)) <= 1e-15 * abs(z) ** 0.5
        assert abs(oracle.fn_value(wl.fn_invsqrt(), z) - 1 / cmath.sqrt(z)) <= 1e-15 / abs(z) ** 0.5
        assert abs(oracle.fn_value(wl.fn_log(), z) - cmath.log(z)) <= 1e-14 * max(1, abs(cmath.log(z)))
    # just above / below the cut: the two sides of the principal branch
    assert abs(oracle.fn_value(wl.fn_sqrt(), complex(-4, 1e-300)) - 2j) < 1e-15
    assert abs(oracle.fn_value(wl.fn_sqrt(), complex(-4, -1e-300)) + 2j) < 1e-15
    for f in (wl.fn_sqrt(), wl.fn_invsqrt(), wl.fn_log()):
        with pytest.raises(oracle.NotHolomorphic):
            oracle.fn_value(f, -4.0)
        with pytest.raises(oracle.NotHolomorphic):
            oracle.fn_value(f, 0.0)
    with pytest.raises(oracle.NotHolomorphic):
        oracle.fn_value(wl.fn_rational([1.0], [1.0, -2.0]), 2.0)


def test_phi_functions():
    """phi_0 = e^x, phi_1 = (e^x-1)/x, phi_2 = (e^x-1-x)/x^2, phi_3 = ..."""
    for x in [2.0, -1.5 + 0.7j, 3j, 0.3, -0.2 + 0.1j, 1e-6]:
        e = cmath.exp(x)
        em1 = complex(np.expm1(x)) if isinstance(x, float) else e - 1
        assert abs(oracle.fn_value(wl.fn_phi(0), x) - e) <= 1e-15 * abs(e)
        p1 = em1 / x
        assert abs(oracle.fn_value(wl.fn_phi(1), x) - p1) <= 2e-14 * abs(p1) + 1e-15
        if abs(x) > 0.1:
            p2 = (e - 1 - x) / x ** 2
            p3 = (e - 1 - x - x * x / 2) / x ** 3
            tol = 1e-13 / abs(x) ** 3
            assert abs(oracle.fn_value(wl.fn_phi(2), x) - p2) <= tol
            assert abs(oracle.fn_value(wl.fn_phi(3), x) - p3) <= tol
    # series limit at 0: phi_k(0) = 1/k!
    for k in range(5):
        assert abs(oracle.fn_value(wl.fn_phi(k), 1e-12) - 1 / math.factorial(k)) < 1e-11


def _cauchy_derivative(f, z0, r, N=96):
    """f'(z0) = (1/(2 pi i)) oint f(z)/(z - z0)^2 dz on |z - z0| = r, by the
    trapezoid rule: uses only values of f (error ~ (r/R)^N for a function
    holomorphic in |z - z0| < R)."""
    th = 2 * np.pi * np.arange(N) / N
    e = np.exp(1j * th)
    vals = np.array([oracle.fn_value(f, z0 + r * ee) for ee in e])
    return np.sum(vals / (r * e)) / N


@pytest.mark.parametrize("fn,z0,r", [
    (wl.fn_rational([1.0, -2.0, 3.0], [1.0, 0.5j]), 1.3 + 0.4j, 0.3),
    (wl.fn_rational([1.0, 0.0], [1.0, -1.0]), 3.0 - 1.0j, 0.5),
    (wl.fn_exp(alpha=-0.7 + 0.1j, beta=2.0), 0.4 - 0.2j, 0.5),
    (wl.fn_log(), 2.0 + 1.0j, 0.5),
    (wl.fn_sqrt(beta=1j), 3.0 - 2.0j, 0.8),
    (wl.fn_invsqrt(alpha=2.0), 1.0 + 1.0j, 0.5),
    (wl.fn_phi(0), 0.3 + 0.2j, 0.2),
    (wl.fn_phi(1), 1.5 - 0.5j, 0.5),
    (wl.fn_phi(3, alpha=0.01), 20.0 + 5.0j, 2.0),
    (wl.fn_combine(wl.COMB_COMPOSE, wl.fn_rational([1.0, -108.8 ** 2]), wl.fn_sqrt(), beta=1j),
     22600.0 + 300.0j, 200.0),
    (wl.fn_combine(wl.COMB_DIV, wl.fn_exp(alpha=0.01), wl.fn_rational([1.0, 3.0])), 4.0 + 2.0j, 1.0),
    (wl.fn_combine(wl.COMB_MUL, wl.fn_rational([-1.0, 0.0]), wl.fn_exp(alpha=-100.0)), -1.0 + 0.05j, 0.01),
    (wl.fn_combine(wl.COMB_ADD, wl.fn_log(), wl.fn_sqrt()), 1.0 + 2.0j, 0.5),
])
def test_fn_derivative_cauchy_integral(fn, z0, r):
    """FNEvaluateDerivative (Section 3.2.2): the oracle's derivative of every FN
    type and combination equals Cauchy's integral formula evaluated from the
    function values alone."""
    ref = _cauchy_derivative(fn, z0, r)
    got = oracle.fn_derivative(fn, z0)
    assert abs(got - ref) <= 1e-11 * abs(ref), (got, ref)


def test_fn_derivative_closed_forms():
    """The derivatives of the workloads' functions in closed form: the delay
    term e^{-tau z}, the gun-like i sqrt(z - s^2), the string's z/(z - sigma),
    and phi_1."""
    z = 0.7 - 1.3j
    assert oracle.fn_derivative(wl.fn_exp(alpha=-1.0), z) == pytest.approx(-cmath.exp(-z), rel=1e-15)
    f = wl.fn_combine(wl.COMB_COMPOSE, wl.fn_rational([1.0, -108.8 ** 2]), wl.fn_sqrt(), beta=1j)
    zz = 22600.0 + 40.0j
    assert oracle.fn_derivative(f, zz) == pytest.approx(0.5j / cmath.sqrt(zz - 108.8 ** 2), rel=1e-14)
    sig = 1.4
    g = wl.fn_rational([1.0, 0.0], [1.0, -sig])
    assert oracle.fn_derivative(g, z) == pytest.approx(-sig / (z - sig) ** 2, rel=1e-14)
    assert oracle.fn_derivative(wl.fn_phi(1), z) == pytest.approx(
        (z * cmath.exp(z) - cmath.exp(z) + 1) / z ** 2, rel=1e-13)


def test_combine_ops():
    a = wl.fn_rational([1.0, -3.0])            # x - 3
    b = wl.fn_exp(alpha=0.5)                    # exp(x/2)
    for z in [1.0 + 1j, -2.0, 4.0 - 0.5j]:
        av, bv = z - 3, cmath.exp(z / 2)
        assert abs(oracle.fn_value(wl.fn_combine(wl.COMB_ADD, a, b), z) - (av + bv)) < 1e-14 * abs(av + bv)
        assert abs(oracle.fn_value(wl.fn_combine(wl.COMB_MUL, a, b), z) - av * bv) < 1e-14 * abs(av * bv)
        assert abs(oracle.fn_value(wl.fn_combine(wl.COMB_DIV, a, b), z) - av / bv) < 1e-14 * abs(av / bv)
        comp = cmath.exp((z - 3) / 2)           # b(a(z))
        assert abs(oracle.fn_value(wl.fn_combine(wl.COMB_COMPOSE, a, b, beta=2j), z) - 2j * comp) < 1e-14 * abs(comp)


# ---------------------------------------------------------------------------
# Quadrature and moments in closed form
# ---------------------------------------------------------------------------

def _diag_linear(d):
    n = len(d)
    return Problem("diag", [np.diag(d).astype(complex), np.eye(n)],
                   [wl.fn_rational([1.0]), wl.fn_rational([-1.0, 0.0])])


@pytest.mark.parametrize("N", [8, 32, 33])
def test_moments_discrete_filter_identity(N):
    """P1: for T(z) = diag(d) - zI on a circle with half-offset trapezoid
    nodes, (1/N) sum_j w^{p+1}/(w - mu) = mu^p/(1+mu^N) for 0 <= p <= N-1, so
    S_p = -diag(mu^p/(1+mu^N)) V exactly (geometric series + the roots of -1).
    """
    c, rho, K = 3.0 - 1.0j, 2.0, 3
    rng = np.random.default_rng(0)
    d = np.array([3.3 - 0.9j, 1.5 - 1.2j, 4.1 + 0.3j, 6.5 + 1j, -0.5 - 3j, 3 + 2.5j])
    prob = _diag_linear(d)
    V = rng.standard_normal((6, 3)) + 1j * rng.standard_normal((6, 3))
    S = oracle.ciss_moments(prob, Contour.circle(c, rho), N, K, V)
    mu = (d - c) / rho
    for p in range(2 * K):
        ref = -(mu ** p / (1 + mu ** N))[:, None] * V
        assert np.abs(S[p] - ref).max() <= 1e-13 * np.abs(ref).max()


def test_quadrature_nodes_weights():
    """Nodes at theta_j = 2 pi (j+1/2)/N; weights integrate dz/(2 pi i)."""
    for con in [Contour.circle(1 + 1j, 2.0), Contour.ellipse(-3.0, 4.0, 0.25)]:
        N = 64
        z, zeta, w = oracle.quadrature(con, N)
        # (1/2 pi i) oint z^k dz = 0 for k >= 0 (polynomial, exact for k < N-1)
        for k in range(5):
            assert abs(np.sum(w * z ** k)) < 1e-12 * np.sum(np.abs(w * z ** k))
        # (1/2 pi i) oint dz/(z-a) = 1 inside, 0 outside (geometric convergence)
        zz, _, ww = oracle.quadrature(con, 512)
        a_in, a_out = con.c + 0.3 * con.rho * con.v, con.c + 1.8 * con.rho
        assert abs(np.sum(ww / (zz - a_in)) - 1) < 1e-13
        assert abs(np.sum(ww / (zz - a_out))) < 1e-13
        # no node on the real axis through the centre (half offset)
        assert np.all(np.abs(z.imag - con.c.imag) > 1e-3 * con.rho * con.v)
        # counter-clockwise orientation: angles increase
        ang = np.unwrap(np.angle(zeta))
        assert np.all(np.diff(ang) > 0)


def test_moments_ellipse_converge_to_residues():
    """Ellipse moments converge to -mu^p (inside) and 0 (outside) as N grows."""
    con = Contour.ellipse(2.0, 3.0, 0.5)
    d = np.array([2.5 + 0.3j, 0.5 - 0.4j, 6.0, 2.0 + 3.0j])
    prob = _diag_linear(d)
    V = np.eye(4, dtype=complex)
    S = oracle.ciss_moments(prob, con, 400, 2, V)
    mu = (d - con.c) / con.rho
    ins = oracle.inside_mask(con, d)
    assert list(ins) == [True, True, False, False]
    for p in range(4):
        ref = np.where(ins, -mu ** p, 0)
        assert np.abs(np.diag(S[p]) - ref).max() < 1e-12


# ---------------------------------------------------------------------------
# Extraction against library routines and closed forms
# ---------------------------------------------------------------------------

def _match(a, b, tol):
    a, b = np.sort_complex(np.asarray(a)), np.asarray(b)
    assert len(a) == len(b), (a, b)
    used = set()
    for x in a:
        k = int(np.argmin([abs(x - y) if i not in used else np.inf for i, y in enumerate(b)]))
        used.add(k)
        assert abs(x - b[k]) <= tol * max(abs(b[k]), 1e-2), (x, b[k])


def test_linear_pencil_vs_generalized_eig():
    """P2: T = A - zB; extraction returns the generalized eigenvalues inside
    (scipy's QZ, an independent routine) and their eigenvectors."""
    rng = np.random.default_rng(11)
    n = 10
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    B = np.eye(n) + 0.1 * rng.standard_normal((n, n))
    prob = Problem("pencil", [A, B], [wl.fn_rational([1.0]), wl.fn_rational([-1.0, 0.0])])
    lam_all, vec = scipy.linalg.eig(A, B)
    con = Contour.circle(0.0, 3.0)
    inside = oracle.inside_mask(con, lam_all)
    assert 2 <= inside.sum() <= 8
    mu = np.abs(lam_all / 3.0)
    assert np.all(np.abs(mu - 1) > 0.05)
    # L > n: every pole of the pencil has a nonzero discrete-filter weight,
    # so the moment rank is n < K*L and all n eigenvalues are recovered.
    V = wl.probes(n, n + 2, 3)
    S = oracle.ciss_moments(prob, con, 64, 1, V)
    r = oracle.extract(prob, con, S, 1)
    assert r["m"] == n
    _match(r["lam"], lam_all, 1e-4)      # far-outside poles: tiny weights
    got = r["lam"][r["inside"]]
    _match(got, lam_all[inside], 1e-10)
    assert np.all(r["eta"][r["inside"]] < 1e-12)
    for lam, x in zip(r["lam"][r["inside"]], r["X"][:, r["inside"]].T):
        k = int(np.argmin(np.abs(lam_all - lam)))
        y = vec[:, k] / np.linalg.norm(vec[:, k])
        assert abs(abs(np.vdot(y, x)) - 1) < 1e-9


def _lambert_roots(a, b, tau, ks=range(-6, 6)):
    # -l + a + b exp(-tau l) = 0  <=>  l = a + W_k(tau b exp(-tau a)) / tau
    return np.array([a + scipy.special.lambertw(tau * b * np.exp(-tau * a), k) / tau for k in ks])


def test_scalar_delay_lambert_w():
    """P3: scalar delay roots from every branch of Lambert W."""
    a, b, tau = 0.5, -2.0, 1.0
    roots = _lambert_roots(a, b, tau)
    for l in roots:   # the closed form really solves the equation
        assert abs(-l + a + b * np.exp(-tau * l)) < 1e-12 * max(1, abs(l))
    con = Contour.circle(0.5, 2.0)
    ins = roots[oracle.inside_mask(con, roots)]
    assert len(ins) == 2
    prob = Problem("scalar_delay", [np.array([[1.0]]), np.array([[a]]), np.array([[b]])],
                   [wl.fn_rational([-1.0, 0.0]), wl.fn_rational([1.0]), wl.fn_exp(alpha=-tau)])
    S = oracle.ciss_moments(prob, con, 48, 4, np.array([[1.0 + 0.5j]]))
    r = oracle.extract(prob, con, S, 4)
    _match(r["lam"][r["inside"]], ins, 1e-10)


def test_diagonal_delay_lambert_w():
    """P4: diagonal delay = union of the scalar roots; x = e_i."""
    a = np.array([0.5, -0.3, 0.2])
    b = np.array([-2.0, -1.5, 0.8])
    tau = 1.0
    con = Contour.circle(0.0, 2.5)
    allr, owner = [], []
    for i in range(3):
        r = _lambert_roots(a[i], b[i], tau)
        allr.extend(r)
        owner.extend([i] * len(r))
    allr = np.array(allr)
    ins = oracle.inside_mask(con, allr)
    assert np.all(np.abs(np.abs(allr / 2.5) - 1) > 0.05)
    prob = Problem("diag_delay", [np.eye(3), np.diag(a), np.diag(b)],
                   [wl.fn_rational([-1.0, 0.0]), wl.fn_rational([1.0]), wl.fn_exp(alpha=-tau)])
    V = wl.probes(3, 3, 7)
    S = oracle.ciss_moments(prob, con, 64, 4, V)
    r = oracle.extract(prob, con, S, 4)
    _match(r["lam"][r["inside"]], allr[ins], 1e-10)
    for lam, x in zip(r["lam"][r["inside"]], r["X"][:, r["inside"]].T):
        i = owner[int(np.argmin(np.abs(allr - lam)))]
        assert abs(abs(x[i]) - 1) < 1e-10


def test_diagonal_rational_quadratic():
    """P5: (a - l b)(l - sigma) + l c = 0 solved by the quadratic formula."""
    a = np.array([2.0, 5.0, 9.0])
    b = np.array([1.0, 0.5, 2.0])
    c = np.array([0.3, -0.7, 1.1])
    sigma = 1.0
    roots, owner = [], []
    for i in range(3):
        # -b l^2 + (a + b sigma + c) l - a sigma = 0
        qa, qb, qc = -b[i], a[i] + b[i] * sigma + c[i], -a[i] * sigma
        disc = cmath.sqrt(qb * qb - 4 * qa * qc)
        for s in (1, -1):
            roots.append((-qb + s * disc) / (2 * qa))
            owner.append(i)
    roots = np.array(roots)
    con = Contour.circle(4.5, 3.0)
    ins = oracle.inside_mask(con, roots)
    assert 2 <= ins.sum() <= 5
    assert np.all(np.abs(np.abs((roots - 4.5) / 3.0) - 1) > 0.03)
    prob = Problem("diag_rational", [np.diag(a), np.diag(b), np.diag(c)],
                   [wl.fn_rational([1.0]), wl.fn_rational([-1.0, 0.0]),
                    wl.fn_rational([1.0, 0.0], [1.0, -sigma])])
    V = wl.probes(3, 3, 8)
    S = oracle.ciss_moments(prob, con, 64, 3, V)
    r = oracle.extract(prob, con, S, 3)
    _match(r["lam"][r["inside"]], roots[ins], 1e-10)


def test_scalar_sqrt_closed_form():
    """P6: k - l m + i w sqrt(l - s^2) = 0; t = sqrt(l - s^2) solves
    m t^2 - i w t - (k - s^2 m) = 0 with Re t > 0 on the principal branch."""
    k, m, w, s = 10.0, 1.0, 1.0, 1.0
    disc = cmath.sqrt(-w * w + 4 * m * (k - s * s * m))
    ts = [(1j * w + disc) / (2 * m), (1j * w - disc) / (2 * m)]
    lam = [t * t + s * s for t in ts if t.real > 0]
    assert len(lam) == 1
    con = Contour.circle(lam[0] + 0.3 - 0.2j, 2.0)
    f_sqrt = wl.fn_combine(wl.COMB_COMPOSE, wl.fn_rational([1.0, -s * s]), wl.fn_sqrt(), beta=1j)
    prob = Problem("scalar_sqrt", [np.array([[k]]), np.array([[m]]), np.array([[w]])],
                   [wl.fn_rational([1.0]), wl.fn_rational([-1.0, 0.0]), f_sqrt])
    S = oracle.ciss_moments(prob, con, 64, 2, np.array([[0.7 - 1.1j]]))
    r = oracle.extract(prob, con, S, 2)
    _match(r["lam"][r["inside"]], lam, 1e-10)


def test_config0_secular_equation():
    """P7: config 0 inside eigenvalues equal the secular-equation roots."""
    cfg = wl.config0()
    roots = string_secular_roots(200, 1.0, 10.0, 190.0)
    assert len(roots) == 3
    S = oracle.ciss_moments(cfg["problem"], cfg["contour"], cfg["N"], cfg["K"], cfg["V"])
    r = oracle.extract(cfg["problem"], cfg["contour"], S, cfg["K"])
    got = r["lam"][r["inside"]]
    _match(got, roots, 1e-12)
    assert np.all(np.abs(got.imag) < 1e-9)          # real eigenvalues (Section 6)
    assert np.all(r["eta"][r["inside"]] < 1e-13)


def test_secular_roots_scaled_string_vs_linearization():
    """The scaled-string secular roots (A scale s != 1, sigma != 1, as in the
    256-problem batch) equal the eigenvalues of the quadratic
    (l - sigma)(sA - l B) + l C = 0, computed by SciPy's dense generalized
    eig of its companion linearization (a third-party routine), and the
    oracle's extraction inside circle(100, 90)."""
    n, sigma, s = 64, 1.3, 0.7
    p = wl.loaded_string(n, sigma=sigma, a_scale=s)
    A, B, Cm = p.mats
    # -B l^2 + (A + sigma B + C) l - sigma A = 0  ->  first companion form
    M0, M1, M2 = -sigma * A, A + sigma * B + Cm, -B
    Z, I = np.zeros((n, n)), np.eye(n)
    lin_A = np.block([[Z, I], [-M0, -M1]])
    lin_B = np.block([[I, Z], [Z, M2]])
    ev = scipy.linalg.eigvals(lin_A, lin_B)
    # multiplying by (l - sigma) adds sigma with multiplicity n - 1 (Q(sigma) =
    # sigma C has rank one); those are not eigenvalues of T
    ev = ev[np.isfinite(ev) & (np.abs(ev - sigma) > 1e-6)]
    assert np.all(np.abs(ev.imag) < 1e-8 * np.abs(ev))
    ev = np.sort(ev.real)
    roots = string_secular_roots(n, sigma, 0.0, 400.0, a_scale=s)
    ref = ev[(ev > 0.0) & (ev < 400.0)]
    assert len(roots) == len(ref) >= 4
    assert np.max(np.abs(roots - ref) / ref) < 1e-9
    con = Contour.circle(100.0, 90.0)
    S = oracle.ciss_moments(p, con, 32, 2, wl.probes(n, 8, 3))
    r = oracle.extract(p, con, S, 2)
    _match(r["lam"][r["inside"]], roots[(roots > 10.0) & (roots < 190.0)], 1e-10)


def test_node_solve_diagonal_closed_form():
    """oracle.node_solve at a diagonal linear problem T(z) = diag(d) - z I:
    Y_j = V / (d - z_j) row by row, with z_j the half-offset trapezoid node
    c + rho e^{i 2 pi (j + 1/2)/N}; and it equals the node solve inside the
    moment loop."""
    d = np.array([0.3 + 0.1j, -0.5, 2.0j, 4.0])
    prob = _diag_linear(d)
    con = Contour.circle(0.2 - 0.1j, 1.3)
    N = 12
    V = wl.probes(4, 3, 11)
    _, Ys = oracle.ciss_moments(prob, con, N, 1, V, return_y=True)
    for j in (0, 5, 11):
        z = con.c + con.rho * np.exp(2j * np.pi * (j + 0.5) / N)
        Y = oracle.node_solve(prob, con, N, j, V)
        np.testing.assert_allclose(Y, V / (d - z)[:, None], rtol=1e-14, atol=0)
        assert np.array_equal(Y, Ys[j])


def test_eigenvalue_count_argument_principle():
    """Argument principle (zeros of det T, eq. (nep)): the oracle's winding
    count equals the secular equation's number of roots inside cfg0's circle,
    and SciPy's eigenvalue count of a random complex pencil inside a circle."""
    cfg = wl.config0()
    roots = string_secular_roots(200, 1.0, 10.0, 190.0)
    for N in (32, 128):
        cnt, step, w = oracle.eigenvalue_count(cfg["problem"], cfg["contour"], N)
        assert cnt == len(roots) == 3 and abs(w - 3) < 1e-8, (N, cnt, w)
    rng = np.random.default_rng(17)
    n = 40
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    B = np.eye(n) + 0.1 * rng.standard_normal((n, n))
    ev = scipy.linalg.eigvals(A, B)
    prob = Problem("pencil", [A, B], [wl.fn_rational([1.0]), wl.fn_rational([-1.0, 0.0])])
    con = Contour.circle(0.5 + 0.5j, 4.5)
    d = np.abs(ev - con.c)
    assert np.min(np.abs(d - con.rho)) > 0.05           # none on the contour
    cnt, step, w = oracle.eigenvalue_count(prob, con, 512)
    assert step < 2.0 and cnt == int(np.sum(d < con.rho)) >= 3, (cnt, int(np.sum(d < con.rho)), step)


def _linear(A):
    n = A.shape[0]
    return Problem("linear", [A, np.eye(n)], [wl.fn_rational([1.0]), wl.fn_rational([-1.0, 0.0])])


def test_left_eigenvectors_vs_scipy():
    """eq. (nep-left): for T(z) = A - z I the oracle's left eigenvectors equal
    SciPy's left eigenvectors of A (up to the common normalization)."""
    rng = np.random.default_rng(23)
    A = rng.standard_normal((15, 15)) + 1j * rng.standard_normal((15, 15))
    w, vl = scipy.linalg.eig(A, left=True, right=False)
    p = _linear(A)
    for k in (0, 4, 9):
        y = oracle.left_eigenvector(p, w[k])
        ref = vl[:, k] / np.linalg.norm(vl[:, k])
        j = int(np.argmax(np.abs(ref)))
        ref = ref * np.conj(ref[j]) / abs(ref[j])
        assert np.linalg.norm(y - ref) < 1e-10
        assert np.abs(y.conj() @ oracle.t_matrix(p, w[k])).max() < 1e-12 * np.abs(A).sum()


def test_keldysh_resolvent_exact_for_linear_full_spectrum():
    """eq. (resolvent): for T(z) = A - z I with every eigenvalue included the
    holomorphic remainder vanishes, so the Keldysh sum (normalization
    y^* T'(lambda) x = 1) is (A - z I)^{-1} exactly."""
    rng = np.random.default_rng(29)
    n = 12
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    w, vl, vr = scipy.linalg.eig(A, left=True, right=True)
    p = _linear(A)
    z = 0.3 + 5.0j
    V = rng.standard_normal((n, 3)) + 1j * rng.standard_normal((n, 3))
    W = oracle.apply_resolvent(p, w, vr, vl, z, V)
    ref = np.linalg.solve(A - z * np.eye(n), V)
    assert np.linalg.norm(W - ref) <= 1e-11 * np.linalg.norm(ref)


def test_config0_invariants():
    """P8: eigenvalues independent of V; conjugate symmetry of node solves."""
    cfg = wl.config0()
    p, con = cfg["problem"], cfg["contour"]
    r0 = oracle.extract(p, con, oracle.ciss_moments(p, con, 32, 2, wl.probes(200, 8, 0)), 2)
    r1 = oracle.extract(p, con, oracle.ciss_moments(p, con, 32, 2, wl.probes(200, 8, 1)), 2)
    _match(r0["lam"][r0["inside"]], r1["lam"][r1["inside"]], 1e-10)
    Vr = np.asfortranarray(wl.probes(200, 8, 0).real.astype(complex))
    _, Ys = oracle.ciss_moments(p, con, 32, 2, Vr, return_y=True)
    for j in range(32):
        assert np.abs(Ys[31 - j] - np.conj(Ys[j])).max() <= 1e-12 * np.abs(Ys[j]).max()


# ---------------------------------------------------------------------------
# Backward error (eq. (sressplit), infinity norms)
# ---------------------------------------------------------------------------

def test_backward_error_hand_example():
    A1 = np.array([[1.0, 2.0], [0.0, 3.0]])
    prob = Problem("tiny", [A1, np.eye(2)], [wl.fn_rational([1.0]), wl.fn_rational([-1.0, 0.0])])
    # exact eigenpair (1, e_1): eta = 0
    assert oracle.backward_error(prob, [1.0], np.array([[1.0], [0.0]]))[0] == 0.0
    # l = 2, x = (1,1): T x = (1, 1); denominator (1*3 + 2*1) * 1 = 5
    assert oracle.backward_error(prob, [2.0], np.array([[1.0], [1.0]]))[0] == pytest.approx(0.2, rel=1e-15)
    # relative residual of the callback example: ||T x||_2 / |l|
    assert oracle.relative_residual(prob, [2.0], np.array([[1.0], [1.0]]))[0] == pytest.approx(np.sqrt(2) / 2, rel=1e-15)


def test_singular_node_and_rank_saturation():
    # node exactly on an eigenvalue: circle(0,1), N=4 puts z_0 at e^{i pi/4}
    z0 = np.exp(1j * np.pi / 4)
    prob = _diag_linear(np.array([z0, 5.0]))
    with pytest.raises(oracle.SingularNode):
        oracle.ciss_moments(prob, Contour.circle(0.0, 1.0), 4, 1, np.eye(2, dtype=complex))
    # three eigenvalues inside but K*L = 2 -> rank saturated
    prob = _diag_linear(np.array([0.1, -0.2j, 0.3 + 0.1j]))
    S = oracle.ciss_moments(prob, Contour.circle(0.0, 1.0), 32, 1, wl.probes(3, 2, 0))
    with pytest.raises(oracle.RankSaturated):
        oracle.extract(prob, Contour.circle(0.0, 1.0), S, 1)
