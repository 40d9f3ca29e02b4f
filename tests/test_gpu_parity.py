"""Parity of the HIP path (through the C ABI) against the FP64 oracle.

Tolerances: moments ||S_gpu - S_oracle||_F / ||S_oracle||_F <= 1e-10 for every
p (both precisions); eigenvalues |dl|/|l| <= 1e-10 with eta <= 1e-10 for the
pairs inside the contour.  The mixed path refines every node to a normwise
backward error of 1e-15 by default (1e-14 where the residual stops halving),
so its moments carry the error of FP64 solves.

Where a problem is ill-conditioned at some node (the random dense cases
below), a solve with normwise backward error b has forward error up to
kappa(T(z_j)) b.  The oracle's LAPACK solves and the plain FP64 path reach
b ~ u = 1.1e-16, the mixed path stops at b <= 1e-14 ~ 100 u.  The bar for the
mixed path there is therefore max(1e-10, 100 e64), with e64 the plain FP64
path's own distance from the oracle on the same inputs (which measures
kappa u): what a backward error of 100 u allows, not a loosened constant.
"""
import numpy as np
import pytest

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


def _rel_fro(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _run_moments(P, prob, con, N, L, K, V, prec, **kw):
    op = P.SplitOperator.from_problem(prob)
    Vd = P.device_probes(V)
    S, st = op.moments(con, Vd, N, L, K, prec=prec, **kw)
    return op, S, P.moments_to_numpy(S), st


def _check_moments(Sg, So, tol=1e-10):
    for p in range(So.shape[0]):
        assert _rel_fro(Sg[p], So[p]) <= tol, (p, _rel_fro(Sg[p], So[p]))


def _check_mixed_vs_fp64(Sm, S64, So):
    """Mixed-path bar derived from the plain FP64 path's error (docstring)."""
    for p in range(So.shape[0]):
        e64, em = _rel_fro(S64[p], So[p]), _rel_fro(Sm[p], So[p])
        print(f"  S_{p}: fp64 {e64:.2e}  mixed {em:.2e}")
        assert e64 <= 1e-10, (p, e64)
        assert em <= max(1e-10, 100.0 * e64), (p, em, e64)


def _match_inside(got_lam, ref_lam, tol):
    got = list(np.asarray(got_lam))
    assert len(got) == len(ref_lam), (got_lam, ref_lam)
    for r in ref_lam:
        k = int(np.argmin([abs(g - r) for g in got]))
        assert abs(got[k] - r) <= tol * max(abs(r), 1e-2), (got[k], r)
        got.pop(k)


# ---------------------------------------------------------------------------

def test_fn_eval_matches_oracle(nep):
    rng = np.random.default_rng(1)
    z = rng.standard_normal(64) * 50 + 1j * rng.standard_normal(64) * 50 + 100
    fns = [wl.fn_rational([1.0, -2.0, 3.0], [1.0, 0.5j]), wl.fn_exp(alpha=-0.7 + 0.1j, beta=2.0),
           wl.fn_log(), wl.fn_sqrt(beta=1j), wl.fn_invsqrt(alpha=2.0),
           wl.fn_phi(0), wl.fn_phi(1), wl.fn_phi(3, alpha=0.01),
           wl.fn_combine(wl.COMB_COMPOSE, wl.fn_rational([1.0, -108.8 ** 2]), wl.fn_sqrt(), beta=1j),
           wl.fn_combine(wl.COMB_DIV, wl.fn_exp(alpha=0.01), wl.fn_rational([1.0, 3.0]))]
    mats = [np.eye(3)] * len(fns)
    op = nep.SplitOperator(mats, fns)
    got = op.fn_eval(z)
    for i, f in enumerate(fns):
        ref = np.array([oracle.fn_value(f, zz) for zz in z])
        assert np.max(np.abs(got[i] - ref) / np.maximum(np.abs(ref), 1e-300)) < 1e-13, i


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_config0_moments(nep, prec):
    cfg = wl.config0()
    p, con = cfg["problem"], cfg["contour"]
    So = oracle.ciss_moments(p, con, cfg["N"], cfg["K"], cfg["V"])
    op, S, Sg, st = _run_moments(nep, p, con, cfg["N"], cfg["L"], cfg["K"], cfg["V"], prec)
    print(prec, st)
    _check_moments(Sg, So)
    if prec == "mixed":
        # the complex-FP32 factorization alone must carry the refinement: no
        # FP64 fallback, few sweeps
        assert st["n_unconverged"] == 0 and st["n_fallback"] == 0
        # an FP32 factor contracts the error by kappa u32 per sweep; the
        # default 1e-15 tolerance takes at most one sweep more than 1e-14 did
        assert st["refine_sweeps"] <= 4
        # at most the tolerance, or 10x it where the residual stopped halving
        assert st["max_rel_residual"] <= 1e-14


@pytest.mark.parametrize("n", [1, 5, 63, 64, 65, 130, 200, 257, 520])
def test_ragged_sizes_complex_terms(nep, n):
    """Dense complex terms, sizes spanning several tiles and ragged tails."""
    rng = np.random.default_rng(n)
    A0 = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    A1 = np.eye(n)
    A2 = rng.standard_normal((n, n)) / np.sqrt(n)
    prob = Problem("rand", [A0, A1, A2],
                   [wl.fn_rational([1.0]), wl.fn_rational([-1.0, 0.0]), wl.fn_exp(alpha=-0.5)])
    con = Contour.circle(0.5 + 0.2j, 1.5 * np.sqrt(n) + 0.3)
    N, L, K = 16, 3, 2
    V = wl.probes(n, L, 5)
    So = oracle.ciss_moments(prob, con, N, K, V)
    _, _, S64, _ = _run_moments(nep, prob, con, N, L, K, V, "fp64")
    _, _, Sm, st = _run_moments(nep, prob, con, N, L, K, V, "mixed")
    print(n, st)
    _check_mixed_vs_fp64(Sm, S64, So)
    # an FP32 factor with kappa u32 ~ 1e-3 contracts the error about 1e3-fold a
    # sweep: 1e-7 -> 1e-14 takes three sweeps, and one may stall at a node
    # close to an eigenvalue before the next converges
    assert st["n_fallback"] == 0 and st["refine_sweeps"] <= 4, st
    assert st["max_rel_residual"] <= 1e-14, st


def test_config0_extract(nep):
    cfg = wl.config0()
    p, con = cfg["problem"], cfg["contour"]
    So = oracle.ciss_moments(p, con, cfg["N"], cfg["K"], cfg["V"])
    ro = oracle.extract(p, con, So, cfg["K"])
    op, S, Sg, st = _run_moments(nep, p, con, cfg["N"], cfg["L"], cfg["K"], cfg["V"], "mixed")
    r = op.extract(con, S, cfg["N"], cfg["L"], cfg["K"], max_eigs=16)
    ins = r["inside"]
    _match_inside(r["lam"][ins], ro["lam"][ro["inside"]], 1e-10)
    assert np.all(r["eta"][ins] <= 1e-10), r["eta"]
    # eigenvectors agree with the oracle's (same normalization)
    for lam, x in zip(r["lam"][ins], r["X"][:, ins].T):
        k = int(np.argmin(np.abs(ro["lam"] - lam)))
        assert np.linalg.norm(x - ro["X"][:, k]) < 1e-8
    assert r["m"] == ro["m"]


def test_config1_full_size_moments(nep):
    """Delay problem at its full size (n=1000, N=64, L=16, K=16), both paths."""
    cfg = wl.config1()
    p, con = cfg["problem"], cfg["contour"]
    So = oracle.ciss_moments(p, con, cfg["N"], cfg["K"], cfg["V"])
    for prec in ("mixed", "fp64"):
        # the plain path runs one residual check (max_refine=1) so that its
        # per-node backward error is measured too; it passes without a sweep
        _, _, Sg, st = _run_moments(nep, p, con, cfg["N"], cfg["L"], cfg["K"], cfg["V"], prec,
                                    max_refine=5 if prec == "mixed" else 1, tol=0.0 if prec == "mixed" else 1e-14)
        print(prec, st)
        _check_moments(Sg, So)
        # per-node normwise backward error of the solves (measured in FP64;
        # the plain path's check runs at 1e-14, the parity rule's level)
        assert 0.0 <= st["max_rel_residual"] <= 1e-14, st
        assert st["min_abs_pivot"] > 0.0 and st["ms_lu"] > 0.0, st
        if prec == "mixed":
            assert st["n_fallback"] == 0 and st["refine_sweeps"] <= 4, st
        else:
            assert st["refine_sweeps"] == 0, st


def test_config2_reduced_extract(nep):
    """Square-root problem (two sqrt terms, complex T) at n=1024: moments and
    the eigenpairs inside the ellipse against the oracle."""
    cfg = wl.config2(1024)
    p, con = cfg["problem"], cfg["contour"]
    So = oracle.ciss_moments(p, con, cfg["N"], cfg["K"], cfg["V"])
    ro = oracle.extract(p, con, So, cfg["K"])
    op, S, Sg, st = _run_moments(nep, p, con, cfg["N"], cfg["L"], cfg["K"], cfg["V"], "mixed")
    print(st)
    _check_moments(Sg, So)
    r = op.extract(con, S, cfg["N"], cfg["L"], cfg["K"], max_eigs=64)
    band = np.abs(np.abs((ro["lam"] - con.c) / con.rho) - 1) > 1e-6
    ref = ro["lam"][ro["inside"] & band]
    assert len(ref) >= 20
    _match_inside(r["lam"][r["inside"]], ref, 1e-10)
    assert np.all(r["eta"][r["inside"]] <= 1e-10)


def test_error_singular_node(nep):
    prob = Problem("sing", [np.diag([1.0, 0.0, 2.0])], [wl.fn_rational([1.0])])
    V = wl.probes(3, 2, 0)
    for prec in ("mixed", "fp64"):
        with pytest.raises(nep.NepError) as ei:
            _run_moments(nep, prob, Contour.circle(0.0, 1.0), 8, 2, 1, V, prec)
        assert ei.value.name == "NEP_ERR_SINGULAR"


def test_error_branch_cut(nep):
    f = wl.fn_combine(wl.COMB_COMPOSE, wl.fn_rational([-1.0]), wl.fn_sqrt())   # sqrt(-1): on the cut
    prob = Problem("cut", [np.eye(3), np.eye(3)], [wl.fn_rational([1.0]), f])
    with pytest.raises(nep.NepError) as ei:
        _run_moments(nep, prob, Contour.circle(0.0, 1.0), 8, 2, 1, wl.probes(3, 2, 0), "mixed")
    assert ei.value.name == "NEP_ERR_NOT_HOLOMORPHIC"


def test_error_rank_saturated(nep):
    d = np.array([0.1, -0.2j, 0.3 + 0.1j, 5.0])
    prob = Problem("diag", [np.diag(d).astype(complex), np.eye(4)],
                   [wl.fn_rational([1.0]), wl.fn_rational([-1.0, 0.0])])
    con = Contour.circle(0.0, 1.0)
    op, S, Sg, st = _run_moments(nep, prob, con, 32, 2, 1, wl.probes(4, 2, 0), "fp64")
    with pytest.raises(nep.NepError) as ei:
        op.extract(con, S, 32, 2, 1, max_eigs=8)
    assert ei.value.name == "NEP_ERR_RANK"


@pytest.mark.parametrize("use_graph", [0, 1])
def test_batch_equals_single_calls(nep, use_graph):
    """A ragged batch (one plan, one set of launches or one graph) gives
    bitwise the same moments as one call per problem."""
    import ctypes as C
    cfg = wl.config3(nprob=6, nmin=64, nmax=300)
    con, N, L, K = cfg["contour"], cfg["N"], cfg["L"], cfg["K"]
    ops, Vs, Ss, singles = [], [], [], []
    for p, V in zip(cfg["problems"], cfg["V"]):
        op, S1, Sg1, st = _run_moments(nep, p, con, N, L, K, V, "mixed")
        ops.append(op)
        singles.append(Sg1)
        Vs.append(nep.device_probes(V))
        Ss.append(torch.zeros((2 * K, L, p.n), dtype=torch.complex128, device="cuda"))
    B = nep.binding
    n = len(ops)
    harr = (C.c_void_p * n)(*[o.h.value for o in ops])
    garr = (B.nep_contour * n)(*[B.contour_struct(con) for _ in ops])
    o = B.opts_struct(N, L, K, "mixed")
    varr = (C.c_void_p * n)(*[v.data_ptr() for v in Vs])
    sarr = (C.c_void_p * n)(*[s.data_ptr() for s in Ss])
    bh = C.c_void_p()
    B.check(B.lib().nep_batch_create(n, harr, garr, C.byref(o), varr, sarr, use_graph, None, C.byref(bh)))
    st = (B.nep_ciss_stats * n)()
    for rep in range(2):   # replays see the same result
        for s in Ss:
            s.zero_()
        torch.cuda.synchronize()
        B.check(B.lib().nep_batch_run(bh, st))
        for k in range(n):
            Sg = nep.moments_to_numpy(Ss[k])
            assert np.array_equal(Sg, singles[k]), (rep, k, np.abs(Sg - singles[k]).max())
    B.check(B.lib().nep_batch_destroy(C.byref(bh)))


def test_small_panel_groups_same_bits(nep):
    """17 problems of at most 256 rows put 544 panels in every LU step, so the
    batch factors with the 256-thread panel groups, while a single call (32
    panels a step) uses the 512-thread groups: the moments agree bitwise."""
    import ctypes as C
    cfg = wl.config3(nprob=17, nmin=64, nmax=256)
    con, N, L, K = cfg["contour"], cfg["N"], cfg["L"], cfg["K"]
    ops, Vs, Ss, singles = [], [], [], []
    for p, V in zip(cfg["problems"], cfg["V"]):
        op, S1, Sg1, st = _run_moments(nep, p, con, N, L, K, V, "mixed")
        ops.append(op)
        singles.append(Sg1)
        Vs.append(nep.device_probes(V))
        Ss.append(torch.zeros((2 * K, L, p.n), dtype=torch.complex128, device="cuda"))
    assert len(ops) * N >= 512 and max(p.n for p in cfg["problems"]) <= 256
    B = nep.binding
    b = B.nep_batch_create([op.h for op in ops], [con] * len(ops), B.opts_struct(N, L, K, "mixed"), Vs, Ss,
                           use_graph=False)
    stats = B.nep_batch_run(b, len(ops))
    B.nep_batch_destroy(b)
    assert all(s["n_unconverged"] == 0 for s in stats)
    for k in range(len(ops)):
        Sg = nep.moments_to_numpy(Ss[k])
        assert np.array_equal(Sg, singles[k]), (k, np.abs(Sg - singles[k]).max())


def test_config3_full_batch_graph_sampled(nep):
    """The 256-problem ragged batch at full size, replayed from a HIP graph
    exactly as the benchmark runs it; every problem converges, and sampled
    problems (smallest, largest and a middle n) match the oracle's moments."""
    cfg = wl.config3()
    con, N, L, K = cfg["contour"], cfg["N"], cfg["L"], cfg["K"]
    probs = cfg["problems"]
    ops = [nep.SplitOperator.from_problem(p) for p in probs]
    Vs = [nep.device_probes(V) for V in cfg["V"]]
    Ss = [torch.zeros((2 * K, L, p.n), dtype=torch.complex128, device="cuda") for p in probs]
    B = nep.binding
    b = B.nep_batch_create([op.h for op in ops], [con] * len(ops), B.opts_struct(N, L, K, "mixed"), Vs, Ss,
                           use_graph=True)
    B.nep_batch_run(b)                 # first replay
    stats = B.nep_batch_run(b, len(ops))   # second replay, synchronous
    B.nep_batch_destroy(b)
    assert all(s["n_unconverged"] == 0 and s["singular_node"] < 0 for s in stats)
    ns = np.array([p.n for p in probs])
    for k in sorted({int(np.argmin(ns)), int(np.argmax(ns)), int(np.argsort(ns)[len(ns) // 2])}):
        So = oracle.ciss_moments(probs[k], con, N, K, cfg["V"][k])
        _check_moments(nep.moments_to_numpy(Ss[k]), So)


def test_config2_full_size_backward_error(nep):
    """The square-root problem at its full size n=4096 (mixed path): every
    eigenpair returned inside the ellipse has an FP64 backward error, computed
    by the oracle on the CPU, of at most 1e-10."""
    cfg = wl.config2()
    p, con = cfg["problem"], cfg["contour"]
    op, S, Sg, st = _run_moments(nep, p, con, cfg["N"], cfg["L"], cfg["K"], cfg["V"], "mixed")
    assert st["n_unconverged"] == 0
    r = op.extract(con, S, cfg["N"], cfg["L"], cfg["K"], max_eigs=64)
    ins = r["inside"]
    assert ins.sum() >= 20
    eta_cpu = oracle.backward_error(p, r["lam"][ins], r["X"][:, ins])
    assert np.all(eta_cpu <= 1e-10), eta_cpu
    assert np.all(r["eta"][ins] <= 1e-10)


@pytest.mark.parametrize("n", [1100, 2048])
def test_large_sizes_both_precisions(nep, n):
    """Sizes with four rows per thread in the panel and the solves (the
    serving workload draws n up to 2048): moments of both paths match the
    oracle."""
    rng = np.random.default_rng(n)
    A0 = 2.0 * rng.standard_normal((n, n)) / np.sqrt(n)
    A2 = rng.standard_normal((n, n)) / np.sqrt(n)
    prob = Problem("delay", [A0, np.eye(n), A2],
                   [wl.fn_rational([1.0]), wl.fn_rational([-1.0, 0.0]), wl.fn_exp(alpha=-1.0)])
    con = Contour.circle(-1.0 + 0.3j, 0.5)
    N, L, K = 8, 2, 1
    V = wl.probes(n, L, 7)
    So = oracle.ciss_moments(prob, con, N, K, V)
    _, _, S64, _ = _run_moments(nep, prob, con, N, L, K, V, "fp64")
    _, _, Sm, st = _run_moments(nep, prob, con, N, L, K, V, "mixed")
    print(n, st)
    _check_mixed_vs_fp64(Sm, S64, So)
    assert st["n_fallback"] == 0 and st["refine_sweeps"] <= 4, st


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_ragged_batch_large_sizes(nep, prec):
    """A ragged batch spanning one to four rows per thread (n = 300 .. 2000),
    run as one plan: every problem equals its single call bitwise, and one
    problem matches the oracle."""
    sizes = [2000, 300, 1500, 900]
    con, N, L, K = Contour.circle(-1.0 + 0.3j, 0.5), 8, 2, 1
    probs, Vs = [], []
    for i, n in enumerate(sizes):
        rng = np.random.default_rng(100 + i)
        A0 = 2.0 * rng.standard_normal((n, n)) / np.sqrt(n)
        A2 = rng.standard_normal((n, n)) / np.sqrt(n)
        probs.append(Problem("delay", [A0, np.eye(n), A2],
                             [wl.fn_rational([1.0]), wl.fn_rational([-1.0, 0.0]), wl.fn_exp(alpha=-1.0)]))
        Vs.append(wl.probes(n, L, 200 + i))
    ops, singles = [], []
    for p, V in zip(probs, Vs):
        op, _, Sg, _ = _run_moments(nep, p, con, N, L, K, V, prec)
        ops.append(op)
        singles.append(Sg)
    B = nep.binding
    Vd = [nep.device_probes(V) for V in Vs]
    Ss = [torch.zeros((2 * K, L, p.n), dtype=torch.complex128, device="cuda") for p in probs]
    b = B.nep_batch_create([op.h for op in ops], [con] * len(ops), B.opts_struct(N, L, K, prec), Vd, Ss,
                           use_graph=False)
    stats = B.nep_batch_run(b, len(ops))
    B.nep_batch_destroy(b)
    for k in range(len(ops)):
        Sg = nep.moments_to_numpy(Ss[k])
        assert np.array_equal(Sg, singles[k]), (k, sizes[k], np.abs(Sg - singles[k]).max(), stats[k])
    So = oracle.ciss_moments(probs[1], con, N, K, Vs[1])
    if prec == "fp64":
        _check_moments(nep.moments_to_numpy(Ss[1]), So)
    else:
        _, _, S64, _ = _run_moments(nep, probs[1], con, N, L, K, Vs[1], "fp64")
        _check_mixed_vs_fp64(nep.moments_to_numpy(Ss[1]), S64, So)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_ragged_batch_wide_panels(nep, prec):
    """A ragged batch whose matrices all have 2048 rows or more takes
    128-wide panels (and, in complex FP32, the blocked solve), including a
    size that is not a multiple of 64 and a last panel narrower than 64:
    every problem equals its single call bitwise, and the odd size matches the
    oracle."""
    sizes = [2600, 2048, 2111]
    con, N, L, K = Contour.circle(-1.0 + 0.3j, 0.5), 8, 2, 1
    probs, Vs = [], []
    for i, n in enumerate(sizes):
        rng = np.random.default_rng(300 + i)
        A0 = 2.0 * rng.standard_normal((n, n)) / np.sqrt(n)
        A2 = rng.standard_normal((n, n)) / np.sqrt(n)
        probs.append(Problem("delay", [A0, np.eye(n), A2],
                             [wl.fn_rational([1.0]), wl.fn_rational([-1.0, 0.0]), wl.fn_exp(alpha=-1.0)]))
        Vs.append(wl.probes(n, L, 400 + i))
    ops, singles = [], []
    for p, V in zip(probs, Vs):
        op, _, Sg, st = _run_moments(nep, p, con, N, L, K, V, prec)
        ops.append(op)
        singles.append(Sg)
        assert st["n_unconverged"] == 0, st
    B = nep.binding
    Vd = [nep.device_probes(V) for V in Vs]
    Ss = [torch.zeros((2 * K, L, p.n), dtype=torch.complex128, device="cuda") for p in probs]
    b = B.nep_batch_create([op.h for op in ops], [con] * len(ops), B.opts_struct(N, L, K, prec), Vd, Ss,
                           use_graph=False)
    stats = B.nep_batch_run(b, len(ops))
    B.nep_batch_destroy(b)
    for k in range(len(ops)):
        Sg = nep.moments_to_numpy(Ss[k])
        assert np.array_equal(Sg, singles[k]), (k, sizes[k], np.abs(Sg - singles[k]).max(), stats[k])
    So = oracle.ciss_moments(probs[2], con, N, K, Vs[2])
    if prec == "fp64":
        _check_moments(nep.moments_to_numpy(Ss[2]), So)
    else:
        _, _, S64, _ = _run_moments(nep, probs[2], con, N, L, K, Vs[2], "fp64")
        _check_mixed_vs_fp64(nep.moments_to_numpy(Ss[2]), S64, So)


def test_mixed_fallback_refined_on_ill_conditioned_nodes(nep):
    """Loaded string n=1912 (sigma 1.413, A scale 1.557) with the serving
    contour around its third eigenvalue: FP32-factor refinement stalls at
    some nodes (kappa(T(z)) ~ 1e6), those nodes are re-solved in FP64 and
    refined with the FP64 factor to the tolerance; the eigenvalue inside
    matches the oracle."""
    from workloads.problems import _string_pencil_value
    n, sig, s = 1912, 1.4132774252668214, 1.5572971183471138
    prob = wl.loaded_string(n, sigma=sig, a_scale=s)
    lam = [_string_pencil_value(n, j, s) for j in (2, 3, 4)]
    con = Contour.circle(lam[1], 0.5 * min(lam[1] - lam[0], lam[2] - lam[1]))
    N, L, K = 32, 8, 2
    V = wl.probes(n, L, 330947230)
    op, S, Sg, st = _run_moments(nep, prob, con, N, L, K, V, "mixed")
    print(st)
    assert st["n_fallback"] >= 1 and st["n_unconverged"] == 0, st
    assert 0.0 < st["max_rel_residual"] <= 1e-14, st
    So = oracle.ciss_moments(prob, con, N, K, V)
    # S_1 cancels by ~1e6 here and kappa ~ 1e6 magnifies any backward-stable
    # solver's error, so the moments are held to the plain FP64 path's own
    # distance from the oracle rather than to a fixed 1e-10
    _, _, S64, _ = _run_moments(nep, prob, con, N, L, K, V, "fp64")
    for p in range(2 * K):
        e_mixed, e_64 = _rel_fro(Sg[p], So[p]), _rel_fro(S64[p], So[p])
        print(p, e_mixed, e_64)
        assert e_mixed <= 10.0 * max(e_64, 1e-12), (p, e_mixed, e_64)
    ro = oracle.extract(prob, con, So, K)
    r = op.extract(con, S, N, L, K, prec="mixed", max_eigs=16)
    ref = np.sort_complex(ro["lam"][ro["inside"]])
    got = np.sort_complex(r["lam"][r["inside"]])
    assert len(ref) == len(got) == 1
    assert np.max(np.abs(got - ref) / np.abs(ref)) <= 1e-10
    assert np.all(r["eta"][r["inside"]] <= 1e-10)


def test_backward_error_matches_oracle(nep):
    """eq. (sressplit) with infinity norms: the device's eta (nep_backward_error
    and the eta nep_extract reports) against the oracle's backward_error on
    pairs far from eigenpairs, where eta is O(1e-3 .. 1) and rounding cannot
    hide a wrong term, norm or scale."""
    cfg = wl.config0()
    p, con = cfg["problem"], cfg["contour"]
    op, S, Sg, st = _run_moments(nep, p, con, cfg["N"], cfg["L"], cfg["K"], cfg["V"], "mixed")
    r = op.extract(con, S, cfg["N"], cfg["L"], cfg["K"], max_eigs=16)
    # the extracted pairs: eta agrees with the oracle's at roundoff level
    eta_o = oracle.backward_error(p, r["lam"], r["X"])
    assert np.all(np.abs(r["eta"] - eta_o) <= 1e-14 + 1e-6 * eta_o), (r["eta"], eta_o)
    # perturbed and random pairs: relative agreement
    rng = np.random.default_rng(5)
    m = 12
    lam = np.concatenate([r["lam"][:4] * (1 + 1e-3), 100 + 80 * rng.standard_normal(m - 4)
                          + 30j * rng.standard_normal(m - 4)])
    X = np.asfortranarray(np.concatenate(
        [r["X"][:, :4] + 1e-3 * (rng.standard_normal((p.n, 4)) + 1j * rng.standard_normal((p.n, 4))),
         rng.standard_normal((p.n, m - 4)) + 1j * rng.standard_normal((p.n, m - 4))], axis=1))
    Xd = torch.from_numpy(np.ascontiguousarray(X.T)).to("cuda")
    eta_g = op.backward_error(lam, Xd)
    eta_o = oracle.backward_error(p, lam, X)
    print(eta_g, eta_o)
    assert np.all(eta_o > 1e-6)
    assert np.max(np.abs(eta_g - eta_o) / eta_o) <= 1e-12, np.abs(eta_g - eta_o) / eta_o
    # complex A_i and a non-rational term (the square-root problem at n=256)
    q = wl.sqrt_problem(256, seed=9)
    op2 = nep.SplitOperator.from_problem(q)
    lam2 = 22600 + 3000 * rng.standard_normal(6) + 500j * rng.standard_normal(6)
    X2 = rng.standard_normal((256, 6)) + 1j * rng.standard_normal((256, 6))
    eta_g2 = op2.backward_error(lam2, torch.from_numpy(np.ascontiguousarray(X2.T)).to("cuda"))
    eta_o2 = oracle.backward_error(q, lam2, X2)
    assert np.max(np.abs(eta_g2 - eta_o2) / eta_o2) <= 1e-12, (eta_g2, eta_o2)


def test_mixed_fp32_overflow_falls_back_to_fp64(nep):
    """T(z) = e^{-100 z} (A - z I) in split form (f_1 = e^{-100 z},
    f_2 = -z e^{-100 z} by FN combine) on circle(-1, 0.1): its eigenvalues are
    A's, but at the nodes |e^{-100 z}| ranges over e^90 .. e^110, so the
    assembled entries overflow complex FP32 (max 3.4e38) while FP64 holds them.
    The FP32 factors and solves are non-finite; refinement must never count
    such a node converged.  With the FP64 re-solve every node falls back and
    the moments match the oracle; without it the call reports
    NEP_ERR_REFINE."""
    n = 64
    rng = np.random.default_rng(12)
    d = np.concatenate([[-1.02, -0.97 + 0.02j, -1.0 - 0.04j],
                        -0.5 + 2.0 * rng.uniform(-1, 1, n - 3) + 1j * rng.uniform(-1, 1, n - 3)])
    A = np.diag(d) + 0.01 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    ex = wl.fn_exp(alpha=-100.0)
    prob = Problem("scaled", [A, np.eye(n)],
                   [ex, wl.fn_combine(wl.COMB_MUL, wl.fn_rational([-1.0, 0.0]), wl.fn_exp(alpha=-100.0))])
    con = Contour.circle(-1.0, 0.1)
    N, L, K = 32, 4, 2
    V = wl.probes(n, L, 8)
    So = oracle.ciss_moments(prob, con, N, K, V)
    op, S, Sg, st = _run_moments(nep, prob, con, N, L, K, V, "mixed")
    print(st)
    assert st["n_fallback"] == N and st["n_unconverged"] == 0, st
    assert np.all(np.isfinite(Sg))
    _, _, S64, _ = _run_moments(nep, prob, con, N, L, K, V, "fp64")
    _check_mixed_vs_fp64(Sg, S64, So)
    with pytest.raises(nep.NepError) as ei:
        _run_moments(nep, prob, con, N, L, K, V, "mixed", fallback=False)
    assert ei.value.name == "NEP_ERR_REFINE"
