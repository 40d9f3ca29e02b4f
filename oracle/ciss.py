"""Plain, slow FP64 reference of the split-form contour-integral path.

TEST INFRASTRUCTURE ONLY (see the package docstring): nothing in the product
path may import this module.

What it computes, step by step, with the passage each step follows:

* Split form T(z) = sum_i f_i(z) A_i                    -- Section 2, eq. (split)
* f_i under the FN semantics: rational p/q with coefficients highest degree
  first, exp, log, principal sqrt and inverse sqrt, the phi_k recurrence,
  scaling beta*g(alpha*z) and combinations            -- Section 3.2.2 (FN list,
  Figure "split")
* Trapezoid quadrature of the contour integral of eq. (invpair) over a circle
  or ellipse (the RG region of Section 3.2.4), nodes at half-offset angles.
* Moments S_p = (1/(2 pi i)) oint phi(z)^p T(z)^{-1} V dz with
  phi(z) = (z-c)/rho.  By Keldysh's expansion (eq. (resolvent)) only the
  poles inside the contour contribute: S_p = sum mu_i^p x_i y_i^* V.
* Block Hankel matrices of the moments have the row space of the block matrix
  V_p(X, H) of eq. (invpair-split); an SVD gives its rank, and the projected
  matrix V0^* B1 W0 Sigma0^{-1} is similar to H, so its eigenvalues are the
  eigenvalues inside and the first block of its eigenvectors (mapped by V0)
  gives X (minimal invariant pair, Section 2).
* Backward error of eq. (sressplit) with infinity norms (Section 6).
* Eigenvalues outside the region are flagged (RG filter, Section 3.2.4).

* Eigenpair polish by residual inverse iteration (Section 4.1, Algorithm
  "RII", eqs. (rii), (rii-scalar)) with the derivatives of the FN functions
  (FNEvaluateDerivative, Section 3.2.2).

Library primitives used as single steps: numpy.linalg.solve (one LU solve of
T(z_j) Y = V), numpy.linalg.svd and numpy.linalg.eig.  No blocking or fusion.
"""
import math

import numpy as np

COMB_ADD, COMB_MUL, COMB_DIV, COMB_COMPOSE = 0, 1, 2, 3


class NotHolomorphic(ValueError):
    """A quadrature node (or eigenvalue) lies on a pole or branch cut of f_i."""


class SingularNode(ArithmeticError):
    """T(z_j) is exactly singular at node j."""

    def __init__(self, j):
        super().__init__(f"T(z_j) singular at node {j}")
        self.node = j


class RankSaturated(ArithmeticError):
    """All K*L singular values are significant: L or K is too small."""


# ---------------------------------------------------------------------------
# FN semantics (Section 3.2.2)
# ---------------------------------------------------------------------------

def _horner(coeffs, x):
    acc = 0j
    for c in coeffs:          # highest degree first
        acc = acc * x + c
    return acc


def _on_cut(x):
    # principal branch of sqrt/log: cut along the non-positive real axis
    return x.imag == 0.0 and x.real <= 0.0


def _phi(k, x):
    """phi_0 = e^x, phi_1 = (e^x - 1)/x, phi_k = (phi_{k-1} - 1/(k-1)!)/x.

    For |x| < 1/2 the recurrence cancels; there the defining power series
    phi_k(x) = sum_m x^m/(m+k)! is summed instead (same function)."""
    if abs(x) < 0.5:
        s, term = 0j, 1.0 / math.factorial(k)
        for m in range(40):
            s += term
            term = term * x / (m + k + 1)
        return s
    v = complex(np.exp(x))
    for j in range(1, k + 1):
        v = (v - 1.0 / math.factorial(j - 1)) / x
    return v


def fn_value(fn, z):
    """beta * g(alpha * z) for one complex scalar z."""
    x = complex(fn["alpha"]) * complex(z)
    t = fn["type"]
    if t == "rational":
        num = _horner(fn["num"], x)
        if fn["den"]:
            den = _horner(fn["den"], x)
            if den == 0:
                raise NotHolomorphic("pole of a rational function")
            g = num / den
        else:
            g = num
    elif t == "exp":
        g = complex(np.exp(x))
    elif t == "log":
        if _on_cut(x):
            raise NotHolomorphic("log branch cut")
        g = complex(np.log(x))
    elif t == "sqrt":
        if _on_cut(x):
            raise NotHolomorphic("sqrt branch cut")
        g = complex(np.sqrt(x))
    elif t == "invsqrt":
        if _on_cut(x):
            raise NotHolomorphic("inverse sqrt branch cut")
        g = 1.0 / complex(np.sqrt(x))
    elif t == "phi":
        g = _phi(int(fn["k"]), x)
    elif t == "combine":
        op = fn["op"]
        a = fn_value(fn["a"], x)
        if op == COMB_COMPOSE:
            g = fn_value(fn["b"], a)
        else:
            b = fn_value(fn["b"], x)
            if op == COMB_ADD:
                g = a + b
            elif op == COMB_MUL:
                g = a * b
            elif op == COMB_DIV:
                if b == 0:
                    raise NotHolomorphic("division by zero in combine")
                g = a / b
            else:
                raise ValueError("unknown combine op")
    else:
        raise ValueError(f"unknown FN type {t}")
    return complex(fn["beta"]) * g


def fn_derivative(fn, z):
    """f'(z) for f(z) = beta * g(alpha * z): alpha * beta * g'(alpha * z)
    (FNEvaluateDerivative, Section 3.2.2), by the rules of differentiation:
    (p/q)' = (p' q - p q')/q^2 with p' from the coefficient list, exp' = exp,
    log' = 1/x, sqrt' = 1/(2 sqrt x), (x^(-1/2))' = -x^(-3/2)/2,
    phi_k' = phi_k - k phi_{k+1}, and the sum, product, quotient and chain
    rules for combinations."""
    a = complex(fn["alpha"])
    x = a * complex(z)
    t = fn["type"]
    if t == "rational":
        num, den = fn["num"], fn["den"]
        dnum = [c * (len(num) - 1 - k) for k, c in enumerate(num[:-1])]
        p, dp = _horner(num, x), _horner(dnum, x)
        if den:
            dden = [c * (len(den) - 1 - k) for k, c in enumerate(den[:-1])]
            q, dq = _horner(den, x), _horner(dden, x)
            if q == 0:
                raise NotHolomorphic("pole of a rational function")
            dg = (dp * q - p * dq) / (q * q)
        else:
            dg = dp
    elif t == "exp":
        dg = complex(np.exp(x))
    elif t == "log":
        if _on_cut(x):
            raise NotHolomorphic("log branch cut")
        dg = 1.0 / x
    elif t == "sqrt":
        if _on_cut(x):
            raise NotHolomorphic("sqrt branch cut")
        dg = 0.5 / complex(np.sqrt(x))
    elif t == "invsqrt":
        if _on_cut(x):
            raise NotHolomorphic("inverse sqrt branch cut")
        dg = -0.5 / (x * complex(np.sqrt(x)))
    elif t == "phi":
        k = int(fn["k"])
        dg = _phi(k, x) - k * _phi(k + 1, x)
    elif t == "combine":
        op = fn["op"]
        ga, da = fn_value(fn["a"], x), fn_derivative(fn["a"], x)
        if op == COMB_COMPOSE:
            dg = fn_derivative(fn["b"], ga) * da
        else:
            gb, db = fn_value(fn["b"], x), fn_derivative(fn["b"], x)
            if op == COMB_ADD:
                dg = da + db
            elif op == COMB_MUL:
                dg = da * gb + ga * db
            elif op == COMB_DIV:
                if gb == 0:
                    raise NotHolomorphic("division by zero in combine")
                dg = (da * gb - ga * db) / (gb * gb)
            else:
                raise ValueError("unknown combine op")
    else:
        raise ValueError(f"unknown FN type {t}")
    return a * complex(fn["beta"]) * dg


# ---------------------------------------------------------------------------
# Contour and quadrature
# ---------------------------------------------------------------------------

def quadrature(contour, N):
    """Trapezoid rule for (1/(2 pi i)) oint g(z) dz on the contour.

    theta_j = 2 pi (j + 1/2)/N, zeta_j = cos theta_j + i v sin theta_j,
    z_j = c + rho zeta_j, w_j = rho (v cos theta_j + i sin theta_j)/N so that
    (1/(2 pi i)) oint g dz ~= sum_j w_j g(z_j) (counter-clockwise)."""
    j = np.arange(N)
    th = 2.0 * np.pi * (j + 0.5) / N
    v = contour.v if contour.kind == 1 else 1.0
    zeta = np.cos(th) + 1j * v * np.sin(th)
    z = contour.c + contour.rho * zeta
    w = contour.rho * (v * np.cos(th) + 1j * np.sin(th)) / N
    return z, zeta, w


def inside_mask(contour, lam):
    mu = (np.asarray(lam) - contour.c) / contour.rho
    if contour.kind == 0:
        return np.abs(mu) < 1.0
    return mu.real ** 2 + (mu.imag / contour.v) ** 2 < 1.0


# ---------------------------------------------------------------------------
# Moments
# ---------------------------------------------------------------------------

def t_matrix(problem, z):
    """T(z) = sum_i f_i(z) A_i, summed in order i = 1..ell (eq. (split))."""
    T = np.zeros(problem.mats[0].shape, dtype=np.complex128)
    for A, f in zip(problem.mats, problem.fns):
        T += fn_value(f, z) * A
    return T


def node_solve(problem, contour, N, j, V):
    """Y_j = T(z_j)^{-1} V for one quadrature node."""
    z, _, _ = quadrature(contour, N)
    T = t_matrix(problem, z[j])
    try:
        return np.linalg.solve(T, V)
    except np.linalg.LinAlgError:
        raise SingularNode(j)


def ciss_moments(problem, contour, N, K, V, return_y=False):
    """S[p] = sum_j w_j zeta_j^p T(z_j)^{-1} V, p = 0..2K-1, j ascending."""
    z, zeta, w = quadrature(contour, N)
    V = np.asarray(V, dtype=np.complex128)
    S = np.zeros((2 * K,) + V.shape, dtype=np.complex128)
    Ys = []
    for j in range(N):
        T = t_matrix(problem, z[j])
        try:
            Y = np.linalg.solve(T, V)
        except np.linalg.LinAlgError:
            raise SingularNode(j)
        if return_y:
            Ys.append(Y)
        for p in range(2 * K):
            S[p] += (w[j] * zeta[j] ** p) * Y
    return (S, Ys) if return_y else S


# ---------------------------------------------------------------------------
# Extraction
# ---------------------------------------------------------------------------

def block_hankel(S, K):
    """B0 = [S_{r+s}], B1 = [S_{r+s+1}], r, s = 0..K-1 (Kn x KL)."""
    B0 = np.block([[S[r + s] for s in range(K)] for r in range(K)])
    B1 = np.block([[S[r + s + 1] for s in range(K)] for r in range(K)])
    return B0, B1


def _normalize(X):
    X = X / np.linalg.norm(X, axis=0, keepdims=True)
    for r in range(X.shape[1]):
        k = int(np.argmax(np.abs(X[:, r])))     # first index of the max
        X[:, r] *= np.conj(X[k, r]) / abs(X[k, r])
    return X


def extract(problem, contour, S, K, rank_tol=1e-12):
    """Eigenpairs from the moments (see the module docstring)."""
    n = S.shape[1]
    L = S.shape[2]
    B0, B1 = block_hankel(S, K)
    U, sig, Wh = np.linalg.svd(B0, full_matrices=False)
    m = int(np.sum(sig > rank_tol * sig[0]))
    if m == K * L:
        raise RankSaturated(f"rank {m} == K*L")
    V0 = U[:, :m]
    W0 = Wh[:m].conj().T
    M = (V0.conj().T @ B1 @ W0) / sig[:m][None, :]
    mu, s = np.linalg.eig(M)
    lam = contour.c + contour.rho * mu
    X = _normalize(V0[:n] @ s)
    order = np.lexsort((lam.imag, lam.real))
    lam, X = lam[order], X[:, order]
    eta = backward_error(problem, lam, X)
    return {"lam": lam, "X": X, "eta": eta,
            "inside": inside_mask(contour, lam), "sigma": sig, "m": m}


# ---------------------------------------------------------------------------
# Eigenvalue count (argument principle)
# ---------------------------------------------------------------------------

def eigenvalue_count(problem, contour, N):
    """Number of eigenvalues inside the contour as the winding number of
    det T(z) along it: eigenvalues are the zeros of det T (eq. (nep)).  The
    phase of det T(z_j) at the N trapezoid nodes (numpy.linalg.slogdet), the
    steps between consecutive nodes taken in (-pi, pi], summed and divided
    by 2 pi.  Returns (count, largest step, unrounded winding number)."""
    z, _, _ = quadrature(contour, N)
    ph = [np.angle(np.linalg.slogdet(t_matrix(problem, zz))[0]) for zz in z]
    steps = [math.remainder(ph[(j + 1) % N] - ph[j], 2.0 * math.pi) for j in range(N)]
    w = sum(steps) / (2.0 * math.pi)
    return int(round(w)), max(abs(s) for s in steps), w


# ---------------------------------------------------------------------------
# Eigenpair polish: residual inverse iteration (Section 4.1, Algorithm "RII")
# ---------------------------------------------------------------------------

def t_derivative(problem, z):
    """T'(z) = sum_i f_i'(z) A_i."""
    T = np.zeros(problem.mats[0].shape, dtype=np.complex128)
    for A, f in zip(problem.mats, problem.fns):
        T += fn_derivative(f, z) * A
    return T


def rii_polish(problem, lam0, x0, tol, max_it=10, max_newton=30):
    """Neumaier's residual inverse iteration as in Algorithm "RII": target
    sigma = lam0 (the eigenvalue to polish), T(sigma) kept fixed, initial
    vector x0.  Each outer step solves the scalar equation
    x^* T(sigma)^{-1} T(z) x = 0 (eq. (rii-scalar)) by Newton's method,
    mu = x^* T(sigma)^{-1} T(z) x / x^* T(sigma)^{-1} T'(z) x, stopping when
    |mu|/|z| < sqrt(eps) (or after max_newton steps); then forms the residual
    r = T(lambda) x, stops when eta(x, lambda) < tol, and otherwise updates
    x <- (x - T(sigma)^{-1} r)/||x - T(sigma)^{-1} r||.  Returns (lambda, x,
    eta, outer steps taken), x normalized as the extraction's eigenvectors."""
    sigma = complex(lam0)
    Ts = t_matrix(problem, sigma)
    x = np.asarray(x0, dtype=np.complex128)
    x = x / np.linalg.norm(x)
    lam = sigma
    eps = np.finfo(float).eps
    eta = np.inf
    k = 0
    for k in range(max_it):
        for _ in range(max_newton):
            num = np.vdot(x, np.linalg.solve(Ts, t_matrix(problem, lam) @ x))
            den = np.vdot(x, np.linalg.solve(Ts, t_derivative(problem, lam) @ x))
            mu = num / den
            lam = lam - mu
            if abs(mu) < np.sqrt(eps) * abs(lam):
                break
        eta = backward_error(problem, [lam], x[:, None])[0]
        if eta < tol:
            break
        r = t_matrix(problem, lam) @ x
        v = np.linalg.solve(Ts, r)
        x = x - v
        x = x / np.linalg.norm(x)
    return lam, _normalize(x[:, None])[:, 0], eta, k + 1


# ---------------------------------------------------------------------------
# Left eigenvectors and the resolvent (Section 2, eqs. (nep-left), (resolvent))
# ---------------------------------------------------------------------------

def left_eigenvector(problem, lam):
    """y with y^* T(lambda) = 0 (eq. (nep-left)): the left singular vector of
    T(lambda) for its smallest singular value (numpy.linalg.svd), normalized
    as the extraction's eigenvectors."""
    U, s, Wh = np.linalg.svd(t_matrix(problem, lam))
    return _normalize(U[:, -1:].copy())[:, 0]


def apply_resolvent(problem, lam, X, Y, z, V):
    """sum_i (z - lambda_i)^{-1} x_i y_i^* V / (y_i^* T'(lambda_i) x_i): the
    sum of Keldysh's expansion (eq. (resolvent)) with its normalization
    y_i^* T'(lambda_i) x_i = 1 applied explicitly."""
    W = np.zeros(np.asarray(V).shape, dtype=np.complex128)
    for l, x, y in zip(np.atleast_1d(lam), np.asarray(X).T, np.asarray(Y).T):
        c = np.vdot(y, t_derivative(problem, l) @ x)
        W += np.outer(x, y.conj() @ V) / ((z - l) * c)
    return W


# ---------------------------------------------------------------------------
# Residuals
# ---------------------------------------------------------------------------

def backward_error(problem, lam, X):
    """eta = ||T(l)x||_inf / (sum_i |f_i(l)| ||A_i||_inf ||x||_inf),
    eq. (sressplit) with infinity norms (Section 6)."""
    norms = [np.abs(A).sum(axis=1).max() for A in problem.mats]
    X = np.asarray(X).reshape(problem.n, -1)
    out = np.empty(len(lam))
    for r, l in enumerate(np.atleast_1d(lam)):
        try:
            fv = [fn_value(f, l) for f in problem.fns]
        except NotHolomorphic:
            out[r] = np.nan
            continue
        x = X[:, r]
        res = sum(f * (A @ x) for f, A in zip(fv, problem.mats))
        den = sum(abs(f) * a for f, a in zip(fv, norms)) * np.abs(x).max()
        out[r] = np.abs(res).max() / den
    return out


def relative_residual(problem, lam, X):
    """||T(l)x|| / |l| as printed by the callback example (Section 3.2.1)."""
    X = np.asarray(X).reshape(problem.n, -1)
    out = np.empty(len(lam))
    for r, l in enumerate(np.atleast_1d(lam)):
        res = t_matrix(problem, l) @ X[:, r]
        out[r] = np.linalg.norm(res) / abs(l)
    return out
