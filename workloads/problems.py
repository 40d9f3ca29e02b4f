"""Problem, contour and probe generators for the benchmark configurations.

Every generator is seeded and synthetic.  The paper's own matrices (the NLEVP
loaded_string and gun problems, the delay PDE of its Section 3.2.2 and
Section 6) are not available; the generators below build problems of the same
*form* (split form, eq. (split)) and of the stated sizes and structure.

Matrices are returned as dense numpy arrays (float64 or complex128); callers
choose the memory order they need.  Nothing in this module evaluates the
method's arithmetic.
"""
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from .fn import (fn_rational, fn_exp, fn_sqrt, fn_combine, COMB_COMPOSE)


@dataclass
class Problem:
    """T(z) = sum_i f_i(z) A_i  (split form, eq. (split))."""
    name: str
    mats: List[np.ndarray]
    fns: List[dict]
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.mats[0].shape[0])

    @property
    def ell(self) -> int:
        return len(self.mats)


@dataclass
class Contour:
    """Closed contour: kind 0 = circle |z-c| = rho; kind 1 = ellipse with
    horizontal semi-axis rho and vertical semi-axis v*rho (the RG ellipse)."""
    kind: int
    c: complex
    rho: float
    v: float = 1.0

    @staticmethod
    def circle(c, rho):
        return Contour(0, complex(c), float(rho), 1.0)

    @staticmethod
    def ellipse(c, rho, v):
        return Contour(1, complex(c), float(rho), float(v))


def probes(n: int, L: int, seed: int) -> np.ndarray:
    """Complex probe block V (n x L): real and imaginary parts i.i.d. N(0,1),
    drawn as standard_normal((2, n, L)) from default_rng(seed)."""
    g = np.random.default_rng(seed).standard_normal((2, n, L))
    return np.asfortranarray(g[0] + 1j * g[1])


def _tridiag(n, lo, d, up):
    m = np.zeros((n, n))
    i = np.arange(n)
    m[i, i] = d
    m[i[1:], i[:-1]] = lo
    m[i[:-1], i[1:]] = up
    return m


def loaded_string(n: int, sigma: float = 1.0, a_scale: float = 1.0) -> Problem:
    """Rational problem of the loaded_string form (Section 6, problem list):
    T(l) = A - l B + l/(l - sigma) C with A = a_scale * n * tridiag(-1,2,-1),
    B = tridiag(1,4,1)/(6n), C = e_n e_n^T (corners unmodified)."""
    A = a_scale * n * _tridiag(n, -1.0, 2.0, -1.0)
    B = _tridiag(n, 1.0, 4.0, 1.0) / (6.0 * n)
    C = np.zeros((n, n))
    C[n - 1, n - 1] = 1.0
    fns = [fn_rational([1.0]),                     # 1
           fn_rational([-1.0, 0.0]),               # -l
           fn_rational([1.0, 0.0], [1.0, -sigma])]  # l / (l - sigma)
    return Problem("loaded_string", [A, B, C], fns,
                   {"sigma": sigma, "a_scale": a_scale})


def delay_problem(n: int, tau: float = 1.0, seed: int = 1) -> Problem:
    """Delay form of eq. (delay): T(l) = -l I + A0 + A1 exp(-tau l), with
    A0 = 2 G0, A1 = G1, G entries N(0, 1/n) drawn G0 then G1 from
    default_rng(seed).  Term order as in the paper's split-form example."""
    rng = np.random.default_rng(seed)
    G0 = rng.standard_normal((n, n)) / np.sqrt(n)
    G1 = rng.standard_normal((n, n)) / np.sqrt(n)
    fns = [fn_rational([1.0]), fn_rational([-1.0, 0.0]),
           fn_exp(alpha=-tau, beta=1.0)]
    return Problem("delay", [2.0 * G0, np.eye(n), G1], fns,
                   {"tau": tau, "seed": seed})


def _sym_band(rng, n, bw):
    R = np.zeros((n, n))
    for k in range(1, bw + 1):
        d = rng.standard_normal(n - k)
        i = np.arange(n - k)
        R[i, i + k] = d
        R[i + k, i] = d
    return R


def sqrt_problem(n: int, s1: float = 0.0, s2: float = 108.8, seed: int = 2,
                 lo: float = 140.0 ** 2, hi: float = 160.0 ** 2,
                 bw: int = 32, rank: int = 64) -> Problem:
    """Square-root (gun-like) form: T(l) = K - l M + i sqrt(l - s1^2) W1
    + i sqrt(l - s2^2) W2.  K, M symmetric banded (bandwidth bw) with N(0,1)
    off-diagonals made diagonally dominant; K gets a graded diagonal so that
    about 24 pencil eigenvalues fall in [lo, hi]; W_k = G_k G_k^T / rank with
    G_k (n x rank) N(0,1).  Draw order from default_rng(seed): R_K, R_M, G_1,
    G_2."""
    rng = np.random.default_rng(seed)
    RK = _sym_band(rng, n, bw)
    RM = _sym_band(rng, n, bw)
    G1 = rng.standard_normal((n, rank))
    G2 = rng.standard_normal((n, rank))
    M = RM + np.diag(np.abs(RM).sum(axis=1) + 1.0)
    grade = np.mean(np.diag(M)) * (hi - lo) / 24.0 * n
    K = RK + np.diag(np.abs(RK).sum(axis=1) + 1.0) \
        + np.diag(grade * np.arange(1, n + 1) / n)
    W1 = G1 @ G1.T / rank
    W2 = G2 @ G2.T / rank
    if s1 == 0.0:
        f3 = fn_sqrt(beta=1j)
    else:
        f3 = fn_combine(COMB_COMPOSE, fn_rational([1.0, -s1 * s1]), fn_sqrt(),
                        beta=1j)
    f4 = fn_combine(COMB_COMPOSE, fn_rational([1.0, -s2 * s2]), fn_sqrt(),
                    beta=1j)
    fns = [fn_rational([1.0]), fn_rational([-1.0, 0.0]), f3, f4]
    return Problem("sqrt", [K, M, W1, W2], fns,
                   {"s1": s1, "s2": s2, "seed": seed})


# ---------------------------------------------------------------------------
# Benchmark configurations.  Each returns a dict with the problem(s), the
# contour(s), quadrature size N, probe count L, Hankel block count K and V.
# ---------------------------------------------------------------------------

def config0():
    """Rational string, n=200, circle(100, 90), N=32, L=8, K=2, V seed 0."""
    p = loaded_string(200, sigma=1.0)
    return {"name": "cfg0_rational_n200", "problem": p,
            "contour": Contour.circle(100.0, 90.0), "N": 32, "L": 8, "K": 2,
            "V": probes(p.n, 8, 0)}


def config1(n: int = 1000):
    """Delay, n=1000, tau=1, circle(-1, 2), N=64, L=16, K=16, V seed 101."""
    p = delay_problem(n, tau=1.0, seed=1)
    return {"name": f"cfg1_delay_n{n}", "problem": p,
            "contour": Contour.circle(-1.0, 2.0), "N": 64, "L": 16, "K": 16,
            "V": probes(p.n, 16, 101)}


def config2(n: int = 4096):
    """Square root, n=4096, ellipse c=22600, semi-axes 3000 and 1000,
    N=64, L=32, K=2, V seed 102."""
    p = sqrt_problem(n, seed=2)
    return {"name": f"cfg2_sqrt_n{n}", "problem": p,
            "contour": Contour.ellipse(22600.0, 3000.0, 1.0 / 3.0), "N": 64,
            "L": 32, "K": 2, "V": probes(p.n, 32, 102)}


def config3(nprob: int = 256, nmin: int = 64, nmax: int = 1024):
    """Batch of rational-string problems: n ~ U{nmin..nmax}, sigma ~ U[0.5,2],
    A-scale ~ U[0.5,2] (drawn in that order per problem from default_rng(3));
    problem p's V from default_rng(3000+p).  circle(100, 90), N=32, L=8, K=2."""
    rng = np.random.default_rng(3)
    probs, Vs = [], []
    for p in range(nprob):
        n = int(rng.integers(nmin, nmax + 1))
        sigma = float(rng.uniform(0.5, 2.0))
        s = float(rng.uniform(0.5, 2.0))
        probs.append(loaded_string(n, sigma=sigma, a_scale=s))
        Vs.append(probes(n, 8, 3000 + p))
    return {"name": f"cfg3_batch{nprob}", "problems": probs,
            "contour": Contour.circle(100.0, 90.0), "N": 32, "L": 8, "K": 2,
            "V": Vs}


def _string_pencil_value(n, k, a_scale):
    # Eigenvalues of the tridiagonal Toeplitz pencil (A, B) of the string:
    # eigenvectors sin(j*theta_k), theta_k = k*pi/(n+1).
    th = k * np.pi / (n + 1)
    return a_scale * 2.0 * n * (1 - np.cos(th)) / ((4 + 2 * np.cos(th)) / (6.0 * n))


def config4_stream(rate: float = 200.0, duration: float = 60.0,
                   warmup: float = 5.0, pool: int = 24, seed: int = 4,
                   nmin: int = 128, nmax: int = 2048):
    """Serving workload: Poisson arrivals at `rate` queries/s for
    warmup+duration seconds; 50/30/20 % rational/delay/sqrt problems with
    n ~ U{nmin..nmax}; N in {32, 64}, L in {8, 16}; a random contour around
    each problem's spectrum.  Problems come from a pool of `pool` registered
    operators (the A_i are uploaded once per operator)."""
    rng = np.random.default_rng(seed)
    ops = []
    for _ in range(pool):
        kind = rng.choice(3, p=[0.5, 0.3, 0.2])
        n = int(rng.integers(nmin, nmax + 1))
        if kind == 0:
            sigma = float(rng.uniform(0.5, 2.0))
            s = float(rng.uniform(0.5, 2.0))
            ops.append(("rational", n, {"sigma": sigma, "a_scale": s}))
        elif kind == 1:
            ops.append(("delay", n, {"seed": int(rng.integers(1 << 30))}))
        else:
            ops.append(("sqrt", n, {"seed": int(rng.integers(1 << 30))}))
    t, queries = 0.0, []
    total = warmup + duration
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t >= total:
            break
        op = int(rng.integers(pool))
        kind, n, par = ops[op]
        N = int(rng.choice([32, 64]))
        L = int(rng.choice([8, 16]))
        if kind == "rational":
            k = int(rng.integers(2, 7))
            lam = [_string_pencil_value(n, j, par["a_scale"]) for j in (k - 1, k, k + 1)]
            gap = min(lam[1] - lam[0], lam[2] - lam[1])
            con = Contour.circle(lam[1], 0.5 * gap)
            K = 2
        elif kind == "delay":
            r = 1.5 * np.sqrt(rng.uniform())
            ang = rng.uniform(0, 2 * np.pi)
            m = int(rng.integers(4, 13))
            con = Contour.circle(-1.0 + r * np.exp(1j * ang),
                                 np.sqrt(m / (np.pi * 0.068 * n)))
            K = 4
        else:
            c = 150.0 ** 2 + rng.uniform(-1500.0, 1500.0)
            con = Contour.ellipse(c, 1500.0, 1.0 / 3.0)
            K = 4
        queries.append({"t": t, "warm": t < warmup, "op": op, "N": N, "L": L,
                        "K": K, "contour": con,
                        "vseed": int(rng.integers(1 << 30))})
    return {"name": "cfg4_serving", "ops": ops, "queries": queries}


def build_operator(op):
    kind, n, par = op
    if kind == "rational":
        return loaded_string(n, sigma=par["sigma"], a_scale=par["a_scale"])
    if kind == "delay":
        return delay_problem(n, tau=1.0, seed=par["seed"])
    return sqrt_problem(n, seed=par["seed"])


CONFIGS = {0: config0, 1: config1, 2: config2, 3: config3}
