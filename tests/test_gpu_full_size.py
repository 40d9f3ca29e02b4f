"""Parity at the full sizes of the benchmark workloads, through the C ABI.

* The square-root workload at n=4096 (N=64, L=32, K=2), both precisions,
  against oracle values stored by tests/golden/make_oracle_golden.py: every
  moment element at sampled rows, every moment's Frobenius norm and a
  weighted sum over all rows, and the complete set of eigenvalues inside the
  ellipse.
* The 256-problem rational batch as the benchmark runs it (one plan, HIP
  graph replay): every problem's eigenvalues inside the circle against the
  closed-form secular equation of the string, and a stratified sample of 16
  problems against the oracle's moments and eigenpairs.

Bars: moments |dS| <= 1e-10 max_i |S[i, c]| element by element (column
scale) and ||dS_p||_F <= 1e-10 ||S_p||_F; eigenvalues |dl| <= 1e-10 |l|,
same count; backward error eta <= 1e-10 (eq. (sressplit), infinity norms).

The eigenpairs compared are the converged ones inside the contour (eta at
most 1e-10, the paper's solvers' stopping test), on both sides.  The
numerical rank is not compared where a singular value of the moments lies
near the 1e-12 threshold: the moments' own error (normwise backward error
1e-14 per solve, times the conditioning) moves such a value across it, and
the extra direction then yields a spurious pair with a large backward error,
which the convergence test rejects.
"""
import os

import numpy as np
import pytest

import oracle
import workloads as wl
from closed_forms import string_secular_roots

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "cfg2_sqrt_n4096_oracle.npz")
TOL = 1e-10
BAND = 1e-6  # eigenvalues within this relative distance of the contour are not counted


@pytest.fixture(scope="module")
def nep():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1910_11712_amd as P
    P.binding.lib()
    return P


@pytest.fixture(scope="module")
def cfg2():
    return wl.config2()


def _inside_off_band(con, lam):
    mu = (np.asarray(lam) - con.c) / con.rho
    r = np.abs(mu) if con.kind == 0 else np.sqrt(mu.real ** 2 + (mu.imag / con.v) ** 2)
    return (r < 1.0) & (np.abs(r - 1.0) > BAND)


def _match(got, ref, tol):
    got = list(np.asarray(got))
    assert len(got) == len(ref), (np.sort_complex(np.asarray(got)), np.sort_complex(ref))
    worst = 0.0
    for r in ref:
        k = int(np.argmin([abs(g - r) for g in got]))
        e = abs(got[k] - r) / max(abs(r), 1e-300)
        worst = max(worst, e)
        assert e <= tol, (got[k], r, e)
        got.pop(k)
    return worst


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_config2_full_size_against_oracle(nep, cfg2, prec):
    g = np.load(GOLDEN, allow_pickle=False)
    p, con, N, L, K = cfg2["problem"], cfg2["contour"], cfg2["N"], cfg2["L"], cfg2["K"]
    assert (int(g["n"]), int(g["N"]), int(g["L"]), int(g["K"])) == (p.n, N, L, K)
    print(f"cfg2 n={p.n} N={N} L={L} K={K} prec={prec}", flush=True)
    op = nep.SplitOperator.from_problem(p)
    Vd = nep.device_probes(cfg2["V"])
    S, st = op.moments(con, Vd, N, L, K, prec=prec, max_refine=5 if prec == "mixed" else 1,
                       tol=0.0 if prec == "mixed" else 1e-14)
    print(st, flush=True)
    assert st["n_unconverged"] == 0 and st["singular_node"] < 0
    # per-node normwise backward error of the solves, measured in FP64 on the
    # device; the plain path passes it without a correction sweep, so its
    # moments are those of the unrefined FP64 solves the benchmark times
    assert 0.0 <= st["max_rel_residual"] <= 1e-14, st
    if prec == "fp64":
        assert st["refine_sweeps"] == 0, st
    Sg = nep.moments_to_numpy(S)
    rows = g["rows"]
    for q in range(2 * K):
        d = np.abs(Sg[q][rows] - g["S_rows"][q])
        e_elem = float((d / g["S_colmax"][q][None, :]).max())
        e_fro = abs(np.linalg.norm(Sg[q]) - g["S_fro"][q]) / g["S_fro"][q]
        u = wl.probes(p.n, 1, int(g["u_seed"]))[:, 0]
        e_u = float(np.abs(u.conj() @ Sg[q] - g["uS"][q]).max() / (np.linalg.norm(u) * g["S_fro"][q]))
        print(f"S_{q}: element {e_elem:.2e}  fro {e_fro:.2e}  u^H S {e_u:.2e}", flush=True)
        assert e_elem <= TOL and e_fro <= TOL and e_u <= TOL, (q, e_elem, e_fro, e_u)
    r = op.extract(con, S, N, L, K, prec=prec, max_eigs=K * L, eta_tol=TOL)
    assert r["m"] == int(g["m"])
    ref = g["lam"][_inside_off_band(con, g["lam"]) & (g["eta"] <= TOL)]
    got = r["lam"][_inside_off_band(con, r["lam"]) & r["inside"]]
    assert len(ref) >= 20
    worst = _match(got, ref, TOL)
    print(f"{len(ref)} eigenvalues inside, max |dl|/|l| = {worst:.2e}", flush=True)
    assert np.all(r["eta"][r["inside"]] <= TOL), r["eta"][r["inside"]]
    op.close()


def test_config3_full_batch_eigenvalues(nep):
    """All 256 problems of the batch, run as the benchmark runs them (graph
    replay): inside eigenvalues equal the secular-equation roots of each
    problem's (n, sigma, A scale); 16 problems spread over the size range
    also match the oracle's moments and eigenpairs."""
    cfg = wl.config3()
    con, N, L, K = cfg["contour"], cfg["N"], cfg["L"], cfg["K"]
    probs = cfg["problems"]
    ops = [nep.SplitOperator.from_problem(p) for p in probs]
    Vs = [nep.device_probes(V) for V in cfg["V"]]
    Ss = [torch.zeros((2 * K, L, p.n), dtype=torch.complex128, device="cuda") for p in probs]
    B = nep.binding
    print("cfg3 batch: 256 problems, graph", flush=True)
    b = B.nep_batch_create([op.h for op in ops], [con] * len(ops), B.opts_struct(N, L, K, "mixed"), Vs, Ss,
                           use_graph=True)
    # three replays, each waited for: nodes the fixed sweeps leave above the
    # tolerance are re-solved in FP64 after every replay, not only the first
    first = None
    for rep in range(3):
        stats = B.nep_batch_run(b, len(ops))
        assert all(s["n_unconverged"] == 0 and s["singular_node"] < 0 for s in stats), rep
        snap = [nep.moments_to_numpy(S) for S in Ss[::37]]
        if first is None:
            first = snap
        else:
            assert all(np.array_equal(a, c) for a, c in zip(first, snap)), rep
    print("FP64 re-solved nodes per replay:", sum(s["n_fallback"] for s in stats), flush=True)
    B.nep_batch_destroy(b)
    worst, count, spurious = 0.0, 0, 0
    for k, (p, op) in enumerate(zip(probs, ops)):
        r = op.extract(con, Ss[k], N, L, K, prec="mixed", max_eigs=K * L, eta_tol=TOL)
        roots = string_secular_roots(p.n, p.meta["sigma"], 0.0, 200.0, a_scale=p.meta["a_scale"])
        ref = roots[_inside_off_band(con, roots)]
        got = r["lam"][_inside_off_band(con, r["lam"]) & r["inside"]]
        spurious += int(r["unconverged"].sum())
        worst = max(worst, _match(got, ref, TOL))
        assert np.all(r["eta"][r["inside"]] <= TOL), (k, r["eta"][r["inside"]])
        assert np.all(np.abs(got.imag) <= TOL * np.abs(got)), k   # real eigenvalues
        count += len(ref)
    print(f"{count} inside eigenvalues over 256 problems, max |dl|/|l| vs secular roots {worst:.2e}; "
          f"{spurious} unconverged pairs inside rejected", flush=True)
    # stratified oracle sample: 16 problems at evenly spaced ranks of n
    order = np.argsort([p.n for p in probs], kind="stable")
    for k in order[np.linspace(0, len(order) - 1, 16).round().astype(int)]:
        p = probs[k]
        So = oracle.ciss_moments(p, con, N, K, cfg["V"][k])
        Sg = nep.moments_to_numpy(Ss[k])
        for q in range(2 * K):
            e = np.linalg.norm(Sg[q] - So[q]) / np.linalg.norm(So[q])
            assert e <= TOL, (k, p.n, q, e)
        ro = oracle.extract(p, con, So, K)
        r = ops[k].extract(con, Ss[k], N, L, K, prec="mixed", max_eigs=K * L, eta_tol=TOL)
        _match(r["lam"][_inside_off_band(con, r["lam"]) & r["inside"]],
               ro["lam"][_inside_off_band(con, ro["lam"]) & (ro["eta"] <= TOL)], TOL)
    for op in ops:
        op.close()
