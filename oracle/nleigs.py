"""Plain FP64 reference of the NLEIGS path (Section 4.5) -- TEST INFRASTRUCTURE.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this module; the product path never does.

What it computes, with the passage each step follows:

* The target set Sigma is the region inside a circle or ellipse (the RG
  region, Section 3.2.4); its boundary is discretized at npts points
  z_k = c + rho (cos t_k + i v sin t_k), t_k = 2 pi k / npts.
* Leja--Bagby nodes sigma_j on the discretized boundary and poles xi_j from a
  given discretization of the singularity set Xi (eq. (nleigsleja)): sigma_0
  is the boundary point at t = 0; sigma_{j+1} maximizes |s_j| over the
  boundary points and xi_{j+1} minimizes |s_j| over the points of Xi.  |s_j|
  is infinite at a point already taken as a pole, so each point of Xi serves
  at most once; once every point of Xi is taken (or with Xi empty) the poles
  are infinite (with Xi empty: Newton polynomial interpolation).
* The rational Newton basis b_j of eq. (nleigsbj), with b_0 = 1 (so beta_0 =
  1) and beta_j making the maximum of |b_j| over the boundary points 1.
* The scalar rational divided differences d_i^j of each f_i by the
  interpolation conditions of eq. (nleigsdd) written for scalars:
  d^0 = f(sigma_0), d^j = (f(sigma_j) - sum_{k<j} b_k(sigma_j) d^k) / b_j(sigma_j).
  This is the plain definition of the quantity that eq. (nleigsfdd) computes
  through a matrix function; D_j = sum_i d_i^j A_i (eq. (nleigsdsplit)).
* The degree d: the first j >= 2 with delta^j / delta^0 < tol, delta^j =
  max_i |d_i^j| (the split-form norm estimate), at most dmax.  The last pole
  is then set to infinity (the simplification before eq. (nleigsmatlin)):
  beta_d, b_d and d_i^d are recomputed with xi_d = infinity.
* The linearization pencil (A, B) of eq. (nleigsmatlin), built explicitly,
  and its eigenvalues by a dense generalized eigensolver (the plain
  definition of what the Krylov method approximates).
* The shift-and-invert operator S = (A - sigma B)^{-1} B applied through the
  block recurrences eqs. (nleigstoarreca), (nleigstoarrecb), with one dense
  solve of R_d(sigma).
* Arnoldi in the TOAR representation (Algorithm "Arnoldi for NLEIGS with
  TOAR representation", eqs. (toarblocksd), (nleigs-toar1)--(nleigs-toar4)),
  classical Gram--Schmidt with one reorthogonalization in both the basis U
  and the coefficients G (a new y^0 whose remainder is below 1e-12 of its
  norm does not extend U), and the Ritz values lambda = sigma + 1/theta.

Ties in the greedy selections (exact in exact arithmetic, e.g. symmetric
points of a circle) are resolved to the lowest-indexed candidate among those
within a relative 1e-10 of the extreme value.

Library primitives used as single steps: numpy.linalg.solve, numpy.linalg.qr,
scipy.linalg.eig.  No blocking or fusion.
"""
import numpy as np
import scipy.linalg

from .ciss import fn_value, inside_mask

TIE_REL = 1e-10
DEP_REL = 1e-12   # a new vector this small (relative) after Gram--Schmidt does
                  # not extend U (it lies in the span of U)


def boundary_points(contour, npts):
    """npts points on the region's boundary, t_k = 2 pi k / npts."""
    t = 2.0 * np.pi * np.arange(npts) / npts
    v = contour.v if contour.kind == 1 else 1.0
    return contour.c + contour.rho * (np.cos(t) + 1j * v * np.sin(t))


def _argmax_tie(a):
    m = np.max(a)
    return int(np.nonzero(a >= m * (1.0 - TIE_REL))[0][0])


def _argmin_tie(a):
    """Lowest index within the tie window of the minimum, or -1 if every
    value is infinite."""
    m = np.min(a)
    if not np.isfinite(m):
        return -1
    return int(np.nonzero(a <= m * (1.0 + TIE_REL))[0][0])


def _pole_factor(z, xi):
    """1 - z/xi (1 for an infinite pole)."""
    if np.isinf(xi):
        return np.ones_like(z)
    return 1.0 - z / xi


def leja_bagby(contour, xi_pts, dmax, npts):
    """Nodes sigma_0..sigma_dmax (boundary indices and values) and poles
    xi_1..xi_dmax (xi[0] is unused and infinite), eq. (nleigsleja)."""
    zb = boundary_points(contour, npts)
    xs = np.asarray(xi_pts, dtype=np.complex128).ravel()
    idx = [0]
    sigma = [zb[0]]
    xi = [complex(np.inf)]
    sb = zb - sigma[0]
    sx = xs - sigma[0]
    used = np.zeros(xs.size, dtype=bool)      # |s_j| is infinite at a pole
    for j in range(dmax):
        scale = np.max(np.abs(sb))
        sb = sb / scale
        sx = sx / scale
        k = _argmax_tie(np.abs(sb))
        idx.append(k)
        sigma.append(zb[k])
        xnew = complex(np.inf)
        if xs.size:
            k = _argmin_tie(np.where(used, np.inf, np.abs(sx)))
            if k >= 0:
                xnew = xs[k]
                used |= xs == xnew
        xi.append(xnew)
        sb = sb * (zb - sigma[-1]) / _pole_factor(zb, xnew)
        free = ~used
        sx[free] = sx[free] * (xs[free] - sigma[-1]) / _pole_factor(xs[free], xnew)
    return zb, np.array(idx), np.array(sigma), np.array(xi)


def _basis_on_boundary(zb, sigma, xi, dmax):
    """b_j at every boundary point and beta_j (eq. (nleigsbj), max |b_j| = 1)."""
    bb = np.zeros((dmax + 1, zb.size), dtype=np.complex128)
    beta = np.ones(dmax + 1)
    bb[0] = 1.0
    for j in range(1, dmax + 1):
        t = bb[j - 1] * (zb - sigma[j - 1]) / _pole_factor(zb, xi[j])
        beta[j] = np.max(np.abs(t))
        bb[j] = t / beta[j]
    return bb, beta


def interpolant(problem, contour, xi_pts=(), tol=1e-12, dmax=40, npts=512):
    """The rational interpolant R_d of eq. (nleigsq) in split form: returns a
    dict with d, sigma[0..d], xi[0..d] (xi[0] unused, xi[d] infinite),
    beta[0..d], dd[i, j] = d_i^j, and whether the degree test was met."""
    zb, idx, sigma, xi = leja_bagby(contour, xi_pts, dmax, npts)
    bb, beta = _basis_on_boundary(zb, sigma, xi, dmax)
    ell = problem.ell
    fvals = np.array([[fn_value(f, s) for s in sigma] for f in problem.fns])
    dd = np.zeros((ell, dmax + 1), dtype=np.complex128)
    for j in range(dmax + 1):
        bj = bb[:, idx[j]]                        # b_k(sigma_j), k = 0..dmax
        dd[:, j] = (fvals[:, j] - dd[:, :j] @ bj[:j]) / bj[j]
    delta = np.max(np.abs(dd), axis=0)
    d, met = dmax, False
    for j in range(2, dmax + 1):
        if delta[j] / delta[0] < tol:
            d, met = j, True
            break
    # last pole at infinity: recompute beta_d, b_d and d^d
    xi = xi[:d + 1].copy()
    xi[d] = complex(np.inf)
    t = bb[d - 1] * (zb - sigma[d - 1])
    beta = beta[:d + 1].copy()
    beta[d] = np.max(np.abs(t))
    bd = t / beta[d]
    bj = bb[:d, idx[d]]
    dd = dd[:, :d + 1].copy()
    dd[:, d] = (fvals[:, d] - dd[:, :d] @ bj) / bd[idx[d]]
    return {"d": d, "sigma": sigma[:d + 1], "xi": xi, "beta": beta, "dd": dd,
            "met": met, "delta": delta}


def basis_values(it, lam):
    """b_0(lam)..b_d(lam) (eq. (nleigsbj))."""
    d = it["d"]
    b = np.zeros(d + 1, dtype=np.complex128)
    b[0] = 1.0
    for j in range(1, d + 1):
        xi = it["xi"][j]
        pf = 1.0 if np.isinf(xi) else 1.0 - lam / xi
        b[j] = b[j - 1] * (lam - it["sigma"][j - 1]) / (it["beta"][j] * pf)
    return b


def dd_matrices(problem, it):
    """D_j = sum_i d_i^j A_i, j = 0..d (eq. (nleigsdsplit))."""
    return [sum(it["dd"][i, j] * problem.mats[i] for i in range(problem.ell))
            for j in range(it["d"] + 1)]


def rd_matrix(problem, it, lam):
    """R_d(lam) = sum_j b_j(lam) D_j (eq. (nleigsq))."""
    b = basis_values(it, lam)
    return sum(b[j] * D for j, D in enumerate(dd_matrices(problem, it)))


def rd_coefficients(it, lam):
    """rho_i with R_d(lam) = sum_i rho_i A_i: rho_i = sum_j b_j(lam) d_i^j."""
    return it["dd"] @ basis_values(it, lam)


def linearization(problem, it):
    """The pencil (A, B) of eq. (nleigsmatlin), dense (d n x d n)."""
    d, n = it["d"], problem.n
    D = dd_matrices(problem, it)
    s, be, xi = it["sigma"], it["beta"], it["xi"]
    A = np.zeros((d * n, d * n), dtype=np.complex128)
    B = np.zeros((d * n, d * n), dtype=np.complex128)
    I = np.eye(n)
    for j in range(d - 1):
        A[:n, j * n:(j + 1) * n] = D[j]
    A[:n, (d - 1) * n:] = D[d - 1] - (s[d - 1] / be[d]) * D[d]
    B[:n, (d - 1) * n:] = -D[d] / be[d]
    for r in range(1, d):
        A[r * n:(r + 1) * n, (r - 1) * n:r * n] = s[r - 1] * I
        A[r * n:(r + 1) * n, r * n:(r + 1) * n] = be[r] * I
        B[r * n:(r + 1) * n, (r - 1) * n:r * n] = I
        B[r * n:(r + 1) * n, r * n:(r + 1) * n] = (0.0 if np.isinf(xi[r]) else be[r] / xi[r]) * I
    return A, B


def dense_eigs(problem, it, contour):
    """Eigenvalues of the linearization inside the region, sorted by real
    then imaginary part, with the first blocks of their eigenvectors."""
    A, B = linearization(problem, it)
    w, Y = scipy.linalg.eig(A, B)
    ok = np.isfinite(w)
    w, Y = w[ok], Y[:, ok]
    ins = inside_mask(contour, w)
    w, Y = w[ins], Y[:problem.n, ins]
    order = np.lexsort((w.imag, w.real))
    return w[order], Y[:, order]


def apply_s(problem, it, sigma, x):
    """w = S x, S = (A - sigma B)^{-1} B, by the recurrences of eqs.
    (nleigstoarreca), (nleigstoarrecb) and the permutation Pi.  x: d blocks
    (d x n array); returns d x n."""
    d = it["d"]
    s, be, xi = it["sigma"], it["beta"], it["xi"]
    D = dd_matrices(problem, it)
    y = [None] * d

    def xr(j):
        return 0.0 if np.isinf(xi[j]) else be[j] / xi[j]

    def om(j):
        return 1.0 if np.isinf(xi[j]) else 1.0 - sigma / xi[j]

    y[d - 1] = (x[d - 2] + xr(d - 1) * x[d - 1]) / (s[d - 2] - sigma)
    for j in range(d - 2, 0, -1):
        y[j] = (x[j - 1] + xr(j) * x[j] - be[j] * om(j) * y[j + 1]) / (s[j - 1] - sigma)
    rhs = -sum(D[j] @ y[j + 1] for j in range(d - 1)) - (D[d] @ x[d - 1]) / be[d]
    y[0] = np.linalg.solve(rd_matrix(problem, it, sigma), rhs)
    b = basis_values(it, sigma)
    wt = [b[d - 1] * y[0]] + [y[j] + b[j - 1] * y[0] for j in range(1, d)]
    return np.array(wt[1:] + wt[:1])


def arnoldi(problem, it, sigma, w0, k):
    """k steps of Arnoldi on S in the TOAR representation.  w0: d x n
    starting blocks.  Returns H ((k+1) x k), U (n x m, m <= k+d) and G (d
    blocks of m x (k+1) coefficients, column j = g_{j+1}), so that the Krylov
    basis block i is U @ G[i]."""
    d = it["d"]
    s, be, xi = it["sigma"], it["beta"], it["xi"]
    D = dd_matrices(problem, it)
    Rs = rd_matrix(problem, it, sigma)
    bsig = basis_values(it, sigma)

    def xr(j):
        return 0.0 if np.isinf(xi[j]) else be[j] / xi[j]

    def om(j):
        return 1.0 if np.isinf(xi[j]) else 1.0 - sigma / xi[j]

    Q, R = np.linalg.qr(np.array(w0).T)
    U = Q
    g = R / np.linalg.norm(R)                    # column i: g_1^i
    G = np.zeros((d, d + k, k + 1), dtype=np.complex128)
    G[:, :d, 0] = g.T
    H = np.zeros((k + 1, k), dtype=np.complex128)
    for j in range(k):
        m = U.shape[1]
        gj = G[:, :m, j]                         # d x m
        gt = [None] * d
        gt[d - 1] = (gj[d - 2] + xr(d - 1) * gj[d - 1]) / (s[d - 2] - sigma)
        for i in range(d - 2, 0, -1):
            gt[i] = (gj[i - 1] + xr(i) * gj[i] - be[i] * om(i) * gt[i + 1]) / (s[i - 1] - sigma)
        rhs = -sum(D[i] @ (U @ gt[i + 1]) for i in range(d - 1)) - (D[d] @ (U @ gj[d - 1])) / be[d]
        y0 = np.linalg.solve(Rs, rhs)
        c1 = U.conj().T @ y0
        r = y0 - U @ c1
        c2 = U.conj().T @ r
        r = r - U @ c2
        nr = np.linalg.norm(r)
        if nr > DEP_REL * np.linalg.norm(y0):    # else y^0 lies in span(U): no new column
            U = np.column_stack([U, r / nr])
            g0 = np.concatenate([c1 + c2, [nr]])  # y^0 = U g0
        else:
            g0 = c1 + c2
        mn = U.shape[1]
        gn = np.zeros((d, mn), dtype=np.complex128)
        for i in range(d - 1):
            gn[i, :m] = gt[i + 1]
            gn[i] += bsig[i] * g0
        gn[d - 1] = bsig[d - 1] * g0
        Gj = G[:, :mn, :j + 1].reshape(d * mn, j + 1)
        v = gn.reshape(-1)
        h1 = Gj.conj().T @ v
        v = v - Gj @ h1
        h2 = Gj.conj().T @ v
        v = v - Gj @ h2
        H[:j + 1, j] = h1 + h2
        H[j + 1, j] = np.linalg.norm(v)
        G[:, :mn, j + 1] = (v / H[j + 1, j]).reshape(d, mn)
    return H, U, G[:, :U.shape[1], :]


def ritz(H, U, G, sigma, n):
    """Ritz values lambda = sigma + 1/theta of the k x k Hessenberg block,
    the residual estimates |h_{k+1,k} e_k^* s| and the Ritz vectors' first
    blocks x = U G^0 s (unit 2-norm)."""
    k = H.shape[1]
    th, S = np.linalg.eig(H[:k, :k])
    lam = sigma + 1.0 / th
    est = np.abs(H[k, k - 1] * S[k - 1, :])
    X = U @ (G[0, :U.shape[1], :k] @ S)
    X = X / np.linalg.norm(X, axis=0)
    return lam, est, X
