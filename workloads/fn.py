"""Scalar-function descriptors with the semantics of the paper's FN object
(Section 3.2.2, "Split form"): rational functions given by coefficient lists
(highest degree first), exp, log, principal sqrt and inverse sqrt, the
phi_k functions, an argument/result scaling f(z) = beta * g(alpha * z)
(FNSetScale) and combinations of two functions (FNCOMBINE).

A descriptor is a plain dict; nothing here evaluates a function.
"""

COMB_ADD, COMB_MUL, COMB_DIV, COMB_COMPOSE = 0, 1, 2, 3


def _scale(alpha, beta):
    return {"alpha": complex(alpha), "beta": complex(beta)}


def fn_rational(num, den=None, alpha=1.0, beta=1.0):
    """p(x)/q(x); coefficient lists highest degree first (so -x is [-1, 0])."""
    d = {"type": "rational", "num": [complex(c) for c in num],
         "den": [complex(c) for c in (den or [])]}
    d.update(_scale(alpha, beta))
    return d


def fn_exp(alpha=1.0, beta=1.0):
    d = {"type": "exp"}
    d.update(_scale(alpha, beta))
    return d


def fn_log(alpha=1.0, beta=1.0):
    d = {"type": "log"}
    d.update(_scale(alpha, beta))
    return d


def fn_sqrt(alpha=1.0, beta=1.0):
    d = {"type": "sqrt"}
    d.update(_scale(alpha, beta))
    return d


def fn_invsqrt(alpha=1.0, beta=1.0):
    d = {"type": "invsqrt"}
    d.update(_scale(alpha, beta))
    return d


def fn_phi(k, alpha=1.0, beta=1.0):
    d = {"type": "phi", "k": int(k)}
    d.update(_scale(alpha, beta))
    return d


def fn_combine(op, a, b, alpha=1.0, beta=1.0):
    """op in {COMB_ADD, COMB_MUL, COMB_DIV, COMB_COMPOSE}.

    ADD: a+b, MUL: a*b, DIV: a/b, COMPOSE: b(a(x)) (a is applied first).
    """
    d = {"type": "combine", "op": int(op), "a": a, "b": b}
    d.update(_scale(alpha, beta))
    return d
