"""Closed-form eigenvalues used as pins (test infrastructure).

Nothing here calls the oracle or the HIP path: these are the mathematical
facts both are checked against.
"""
import numpy as np


def string_secular_roots(n, sigma, lo, hi, a_scale=1.0):
    """Eigenvalues in (lo, hi) of the rational string
    T(l) = a_scale A - l B + l/(l - sigma) e_n e_n^T, with
    A = n tridiag(-1, 2, -1) and B = tridiag(1, 4, 1)/(6n).

    A and B share the eigenvectors sin(j theta_k), theta_k = k pi/(n+1), with
    a_k = a_scale 2n (1 - cos theta_k) and b_k = (4 + 2 cos theta_k)/(6n).  In
    that basis the rank-one term gives det T(l) = 0 iff the secular equation
    1 + (l/(l - sigma)) sum_k c_k/(a_k - l b_k) = 0 holds, with
    c_k = (2/(n+1)) sin^2(n theta_k).  Its roots interlace the poles sigma and
    a_k/b_k: one below the first pole and one between each pair of
    consecutive poles.  Each root is found
    by bisection to a few ulps."""
    k = np.arange(1, n + 1)
    th = k * np.pi / (n + 1)
    ak = a_scale * 2.0 * n * (1 - np.cos(th))
    bk = (4 + 2 * np.cos(th)) / (6.0 * n)
    ck = 2.0 / (n + 1) * np.sin(n * th) ** 2

    def h(x):
        x = np.atleast_1d(np.asarray(x, dtype=float))
        g = (ck[None, :] / (ak[None, :] - x[:, None] * bk[None, :])).sum(axis=1)
        return 1.0 + x / (x - sigma) * g

    poles = np.sort(np.concatenate([[sigma], ak / bk]))
    # h(0) = 1, so the interval (0, first pole) holds the smallest root
    edges = np.concatenate([[0.0], poles]) if poles[0] > 0 else poles
    roots = []
    for p0, p1 in zip(edges[:-1], edges[1:]):
        if p1 <= lo or p0 >= hi:
            continue
        eps = 1e-9 * (p1 - p0)
        xs = np.linspace(p0 + eps, p1 - eps, 257)
        hs = h(xs)
        for i in np.nonzero(np.sign(hs[:-1]) != np.sign(hs[1:]))[0]:
            x0, x1 = xs[i], xs[i + 1]
            s0 = np.sign(hs[i])
            for _ in range(200):
                xm = 0.5 * (x0 + x1)
                if np.sign(h(xm)[0]) == s0:
                    x0 = xm
                else:
                    x1 = xm
                if x1 - x0 <= 4 * np.finfo(float).eps * abs(xm):
                    break
            roots.append(0.5 * (x0 + x1))
    return np.array(sorted(r for r in roots if lo < r < hi))
