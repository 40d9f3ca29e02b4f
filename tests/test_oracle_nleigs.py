"""Pins of the NLEIGS oracle (Section 4.5) against facts fixed by the paper and
by mathematics, independent of the oracle's own code.

* Leja points of the unit circle from 1 are the van der Corput sequence.
* The greedy conditions of eq. (nleigsleja), checked by brute force with
  products evaluated from scratch in log form.
* The basis scaling of eq. (nleigsbj) and its zeros at earlier nodes.
* Scalar divided differences against the classical Newton divided-difference
  table (polynomial case), exactness for a rational function whose pole is
  in the singularity set, and interpolation of T.
* The linearization of eq. (nleigsmatlin): a quadratic eigenproblem against
  its textbook companion pencil, and the rational string against the roots
  of its secular equation.
* The recurrences of eqs. (nleigstoarreca), (nleigstoarrecb) against an
  explicit dense (A - sigma B)^{-1} B, and the Arnoldi relation of eq.
  (arnoldi) for the TOAR basis.
"""
import math

import numpy as np
import scipy.linalg

import oracle
import oracle.nleigs as nl
import workloads as wl
from closed_forms import string_secular_roots
from workloads import Contour, Problem


def _vdc(j):
    """Base-2 van der Corput fraction of j (bit reversal)."""
    f, b = 0.0, 0.5
    while j:
        f += b * (j & 1)
        j >>= 1
        b /= 2
    return f


def test_leja_points_of_the_unit_circle():
    """With no poles and sigma_0 = 1, the Leja points of the unit circle are
    the van der Corput sequence exp(2 pi i vdc(j)) (ties, exact in exact
    arithmetic, go to the lowest index: the first of the equal candidates
    counter-clockwise from 1)."""
    _, idx, sigma, xi = nl.leja_bagby(Contour.circle(0.0, 1.0), (), 15, 64)
    want = np.array([round(64 * _vdc(j)) for j in range(16)])
    assert list(idx) == list(want)
    assert np.all(np.isinf(xi[1:]))


def _log_s(z, sigma, xi, j):
    """log |s_j(z)| from its definition (products of eq. (nleigsleja))."""
    with np.errstate(divide="ignore"):
        v = np.sum(np.log(np.abs(z[:, None] - sigma[None, :j + 1])), axis=1)
    for k in range(1, j + 1):
        if not np.isinf(xi[k]):
            v = v - np.log(np.abs(1.0 - z / xi[k]))
    return v


def test_leja_bagby_greedy_conditions():
    """Every node maximizes |s_j| over the boundary points and every finite
    pole minimizes it over the unused points of the singularity set."""
    con = Contour.ellipse(22600.0, 3000.0, 1.0 / 3.0)
    xs = 108.8 ** 2 - np.logspace(-3, 6, 16)
    zb, idx, sigma, xi = nl.leja_bagby(con, xs, 24, 256)
    used = set()
    for j in range(24):
        lb = _log_s(zb, sigma, xi, j)
        assert lb[idx[j + 1]] >= lb.max() - 1e-9
        if np.isinf(xi[j + 1]):
            assert len(used) == len(xs)
            continue
        k = int(np.nonzero(xs == xi[j + 1])[0][0])
        assert k not in used
        free = np.array(sorted(set(range(len(xs))) - used))
        lx = _log_s(xs[free], sigma, xi, j)
        assert _log_s(xs[[k]], sigma, xi, j)[0] <= lx.min() + 1e-9
        used.add(k)
    assert len(used) == len(xs)     # 16 finite poles, then infinite ones


def _string(n=40):
    return wl.loaded_string(n, sigma=1.0)


def test_basis_scaling_and_zeros():
    """max over the boundary points of |b_j| is 1, and b_j vanishes at the
    nodes sigma_0..sigma_{j-1} (eq. (nleigsbj))."""
    con = Contour.circle(100.0, 90.0)
    it = nl.interpolant(_string(), con, xi_pts=(1.0, -5.0), tol=1e-14, dmax=8, npts=512)
    zb = nl.boundary_points(con, 512)
    B = np.array([nl.basis_values(it, z) for z in zb])
    assert np.allclose(np.abs(B).max(axis=0), 1.0, rtol=1e-12, atol=0)
    for j in range(1, it["d"] + 1):
        for k in range(j):
            assert abs(nl.basis_values(it, it["sigma"][k])[j]) < 1e-14


def _newton_table(f, x):
    """Classical divided differences f[x_0..x_j] by the triangular table."""
    c = np.array([f(v) for v in x], dtype=np.complex128)
    out = [c[0]]
    for lev in range(1, len(x)):
        c = (c[1:] - c[:-1]) / (x[lev:] - x[:-lev])
        out.append(c[0])
    return np.array(out)


def test_divided_differences_match_newton_table():
    """All poles infinite: b_j = prod_{k<j} (z - sigma_k) / prod_{k<=j} beta_k,
    so d^j / prod_{k<=j} beta_k = f[sigma_0, .., sigma_j] (classical Newton
    table)."""
    p = Problem("t", [np.eye(2)], [wl.fn_exp(alpha=0.7 + 0.2j)])
    con = Contour.circle(0.5, 2.0)
    it = nl.interpolant(p, con, tol=1e-15, dmax=12, npts=256)
    d = it["d"]
    tab = _newton_table(lambda z: np.exp((0.7 + 0.2j) * z), it["sigma"])
    scaled = it["dd"][0] / np.cumprod(it["beta"])
    assert np.allclose(scaled[:d], tab[:d], rtol=1e-9, atol=1e-12 * abs(tab[0]))


def test_rational_function_is_exact_with_its_pole():
    """f = 1/(z - p) lies in span{b_0, b_1} once xi_1 = p: every later
    divided difference vanishes and the degree test stops at d = 2."""
    pole = 3.0 + 1.0j
    p = Problem("t", [np.eye(2)], [wl.fn_rational([1.0], [1.0, -pole])])
    con = Contour.circle(-2.0, 2.5)
    it = nl.interpolant(p, con, xi_pts=(pole, 40.0), tol=1e-12, dmax=10, npts=256)
    assert it["xi"][1] == pole
    assert it["d"] == 2 and it["met"]
    assert abs(it["dd"][0, 2]) < 1e-13 * abs(it["dd"][0, 0])


def test_interpolant_reproduces_t():
    """R_d equals T at the nodes and approximates it inside the region."""
    p = wl.sqrt_problem(24, seed=2, bw=6, rank=6)
    con = Contour.ellipse(22600.0, 3000.0, 1.0 / 3.0)
    xs = 108.8 ** 2 - np.logspace(-3, 6, 100)
    it = nl.interpolant(p, con, xi_pts=xs, tol=1e-13, dmax=40, npts=1024)
    assert it["met"]
    for z in it["sigma"][:-1]:
        T = oracle.t_matrix(p, z)
        assert np.linalg.norm(nl.rd_matrix(p, it, z) - T) <= 1e-12 * np.linalg.norm(T)
    rng = np.random.default_rng(0)
    for _ in range(8):
        r, t = math.sqrt(rng.uniform()) * 0.95, rng.uniform(0, 2 * math.pi)
        z = con.c + con.rho * (r * math.cos(t) + 1j * con.v * r * math.sin(t))
        T = oracle.t_matrix(p, z)
        assert np.linalg.norm(nl.rd_matrix(p, it, z) - T) <= 1e-10 * np.linalg.norm(T)
        rho = nl.rd_coefficients(it, z)
        assert np.linalg.norm(sum(c * A for c, A in zip(rho, p.mats)) - nl.rd_matrix(p, it, z)) \
            <= 1e-13 * np.linalg.norm(T)


def test_quadratic_linearization_matches_companion_pencil():
    """T(z) = A0 + z A1 + z^2 A2 is interpolated exactly at degree 2: the
    eigenvalues of the pencil of eq. (nleigsmatlin) inside the region are
    those of the textbook companion pencil."""
    rng = np.random.default_rng(11)
    n = 6
    A0, A1, A2 = (rng.standard_normal((n, n)) for _ in range(3))
    p = Problem("quad", [A0, A1, A2], [wl.fn_rational([1.0]), wl.fn_rational([1.0, 0.0]),
                                        wl.fn_rational([1.0, 0.0, 0.0])])
    con = Contour.circle(0.0, 2.0)
    it = nl.interpolant(p, con, tol=1e-12, dmax=10, npts=256)
    assert it["d"] == 3 and np.max(np.abs(it["dd"][:, 3])) < 1e-13
    w, _ = nl.dense_eigs(p, it, con)
    Z, I = np.zeros((n, n)), np.eye(n)
    lc = scipy.linalg.eigvals(np.block([[Z, I], [-A0, -A1]]), np.block([[I, Z], [Z, A2]]))
    lc = lc[np.isfinite(lc)]
    lc = lc[oracle.inside_mask(con, lc)]
    lc = lc[np.lexsort((lc.imag, lc.real))]
    assert len(w) == len(lc) and len(w) > 0
    assert np.max(np.abs(w - lc) / np.abs(lc)) < 1e-10


def test_string_eigenvalues_are_secular_roots():
    """The rational string with its pole in the singularity set: the
    linearization's eigenvalues inside the region are the roots of the
    string's secular equation."""
    n = 40
    p = _string(n)
    con = Contour.circle(100.0, 90.0)
    it = nl.interpolant(p, con, xi_pts=(1.0,), tol=1e-12, dmax=20, npts=512)
    assert it["d"] == 3
    w, X = nl.dense_eigs(p, it, con)
    roots = string_secular_roots(n, 1.0, 10.0, 190.0)
    assert len(w) == len(roots)
    assert np.max(np.abs(w - roots) / roots) < 1e-12
    eta = oracle.backward_error(p, w, X / np.linalg.norm(X, axis=0))
    assert np.max(eta) < 1e-13


def _sqrt_case(n=80):
    p = wl.sqrt_problem(n, seed=2, bw=8, rank=8)
    con = Contour.ellipse(22600.0, 3000.0, 1.0 / 3.0)
    xs = 108.8 ** 2 - np.logspace(-3, 6, 100)
    return p, con, nl.interpolant(p, con, xi_pts=xs, tol=1e-12, dmax=40, npts=1024)


def test_shift_invert_recurrences_match_dense_operator():
    """S x by eqs. (nleigstoarreca), (nleigstoarrecb) and the permutation Pi
    equals (A - sigma B)^{-1} B x with the explicit pencil."""
    p, con, it = _sqrt_case()
    A, B = nl.linearization(p, it)
    rng = np.random.default_rng(1)
    d, n = it["d"], p.n
    x = rng.standard_normal((d, n)) + 1j * rng.standard_normal((d, n))
    for sig in (con.c, con.c + 700.0 + 150.0j):
        w = nl.apply_s(p, it, sig, x)
        ref = np.linalg.solve(A - sig * B, B @ x.reshape(-1)).reshape(d, n)
        assert np.linalg.norm(w - ref) <= 1e-10 * np.linalg.norm(ref)


def test_arnoldi_relation_in_toar_form():
    """The TOAR basis V_k = (I_d (x) U) G satisfies S V_k = V_{k+1} H with
    orthonormal columns, and the converged Ritz values are eigenvalues of the
    pencil."""
    p, con, it = _sqrt_case()
    A, B = nl.linearization(p, it)
    d, n, k = it["d"], p.n, 40
    rng = np.random.default_rng(2)
    w0 = rng.standard_normal((d, n)) + 1j * rng.standard_normal((d, n))
    H, U, G = nl.arnoldi(p, it, con.c, w0, k)
    # a y^0 within 1e-12 (relative) of span(U) does not extend the basis
    assert d + k // 2 <= U.shape[1] <= d + k
    assert np.linalg.norm(U.conj().T @ U - np.eye(U.shape[1])) < 1e-12
    V = np.concatenate([U @ G[i] for i in range(d)], axis=0)
    assert np.linalg.norm(V.conj().T @ V - np.eye(k + 1)) < 1e-12
    S = np.linalg.solve(A - con.c * B, B)
    assert np.linalg.norm(S @ V[:, :k] - V @ H) <= 1e-11 * np.linalg.norm(H)
    lam, est, _ = nl.ritz(H, U, G, con.c, n)
    good = lam[(est < 1e-12) & oracle.inside_mask(con, lam)]
    assert len(good) >= 4
    wall = scipy.linalg.eigvals(A, B)
    for z in good:
        assert np.min(np.abs(wall - z)) < 1e-9 * abs(z)
