"""Serving path (continuous batching over several streams) through the C ABI.

A query's result must not depend on what else is in flight: every query run
in a mix equals the same query run alone (moments + extraction on its own
handle), bit for bit, and matches the oracle's eigenvalues inside the
contour."""
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


def _alone(P, op, con, V, N, L, K, prec, max_eigs):
    Vd = P.device_probes(V)
    S, st = op.moments(con, Vd, N, L, K, prec=prec)
    X = torch.zeros((max_eigs, op.n), dtype=torch.complex128, device="cuda")
    return op.extract(con, S, N, L, K, prec=prec, max_eigs=max_eigs, X=X)


def _mix_cases():
    """Rational problems of several sizes and two option groups, plus a
    delay problem: (problem, contour, N, L, K, V)."""
    cases = []
    for i, (n, sig, s) in enumerate([(200, 1.0, 1.0), (150, 1.5, 0.8), (260, 0.7, 1.3), (96, 1.0, 1.0)]):
        p = wl.loaded_string(n, sigma=sig, a_scale=s)
        N = 32 if i % 2 == 0 else 64
        cases.append((p, Contour.circle(100.0 * s, 90.0 * s), N, 8, 2, wl.probes(n, 8, 10 + i)))
    d = wl.delay_problem(120, tau=1.0, seed=7)
    cases.append((d, Contour.circle(-1.0, 0.4), 32, 8, 4, wl.probes(120, 8, 20)))
    return cases


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_server_mix_equals_alone(nep, prec):
    cases = _mix_cases()
    ops = [nep.SplitOperator.from_problem(c[0]) for c in cases]
    max_eigs = 32
    alone = [_alone(nep, op, c[1], c[5], c[2], c[3], c[4], prec, max_eigs) for op, c in zip(ops, cases)]
    srv = nep.Server(hbm_budget=1 << 30, max_inflight=16, nstreams=3)
    try:
        tickets = []
        for rep in range(2):  # every case twice, interleaved
            for op, c in zip(ops, cases):
                tickets.append(srv.submit(op, c[1], c[5], c[2], c[3], c[4], prec=prec, max_eigs=max_eigs,
                                          want_X=True))
        results = [srv.wait(t) for t in tickets]
    finally:
        srv.close()
    for k, r in enumerate(results):
        a = alone[k % len(cases)]
        assert r["status"] == 0, (k, r["status"])
        assert r["m"] == a["m"]
        assert np.array_equal(r["lam"], a["lam"]), k
        assert np.array_equal(r["eta"], a["eta"]), k
        assert np.array_equal(r["inside"], a["inside"]), k
        assert np.array_equal(r["X"], a["X"]), k
        assert r["t_submit"] <= r["t_start"] <= r["t_done"]
    # the first case is the rational n=200 problem: its inside eigenvalues
    # match the oracle
    p, con, N, L, K, V = cases[0]
    So = oracle.ciss_moments(p, con, N, K, V)
    ro = oracle.extract(p, con, So, K)
    ref = np.sort_complex(ro["lam"][ro["inside"]])
    got = np.sort_complex(results[0]["lam"][results[0]["inside"]])
    assert len(ref) == len(got) == 3
    assert np.max(np.abs(got - ref) / np.abs(ref)) <= 1e-10
    assert np.all(results[0]["eta"][results[0]["inside"]] <= 1e-10)


def test_server_query_errors_are_isolated(nep):
    """A query whose contour crosses a branch cut fails alone; the queries
    batched with it succeed."""
    good = wl.config0()
    f = wl.fn_combine(wl.COMB_COMPOSE, wl.fn_rational([-1.0]), wl.fn_sqrt())  # sqrt(-1): on the cut everywhere
    bad = Problem("cut", [np.eye(8), np.eye(8)], [wl.fn_rational([1.0]), f])
    op_g = nep.SplitOperator.from_problem(good["problem"])
    op_b = nep.SplitOperator.from_problem(bad)
    srv = nep.Server(hbm_budget=1 << 30, max_inflight=8, nstreams=1)
    try:
        t1 = srv.submit(op_g, good["contour"], good["V"], 32, 8, 2)
        t2 = srv.submit(op_b, Contour.circle(0.0, 1.0), wl.probes(8, 8, 0), 32, 8, 2)
        t3 = srv.submit(op_g, good["contour"], good["V"], 32, 8, 2)
        r1, r2, r3 = srv.wait(t1), srv.wait(t2), srv.wait(t3)
    finally:
        srv.close()
    assert r1["status"] == 0 and r3["status"] == 0
    assert nep.binding.ERRORS[r2["status"]] == "NEP_ERR_NOT_HOLOMORPHIC"
    assert np.array_equal(r1["lam"], r3["lam"])


def test_server_fallback_unaffected_by_failing_neighbour(nep):
    """A query whose nodes need the FP64 re-solve (loaded string n=1912 at a
    serving contour, kappa(T(z)) ~ 1e6) batched with a query whose contour
    crosses a branch cut: the cut query fails alone, and the other is
    re-solved exactly as when it runs alone (same bits)."""
    from workloads.problems import _string_pencil_value
    n, sig, s = 1912, 1.4132774252668214, 1.5572971183471138
    prob = wl.loaded_string(n, sigma=sig, a_scale=s)
    lam = [_string_pencil_value(n, j, s) for j in (2, 3, 4)]
    con = Contour.circle(lam[1], 0.5 * min(lam[1] - lam[0], lam[2] - lam[1]))
    N, L, K = 32, 8, 2
    V = wl.probes(n, L, 330947230)
    op = nep.SplitOperator.from_problem(prob)
    alone = _alone(nep, op, con, V, N, L, K, "mixed", 16)
    f = wl.fn_combine(wl.COMB_COMPOSE, wl.fn_rational([-1.0]), wl.fn_sqrt())  # sqrt(-1): on the cut everywhere
    op_b = nep.SplitOperator.from_problem(Problem("cut", [np.eye(8), np.eye(8)], [wl.fn_rational([1.0]), f]))
    srv = nep.Server(hbm_budget=8 << 30, max_inflight=8, nstreams=1)
    try:
        # the first query holds the only slot while the next two queue, so
        # those two are dispatched together as one batch (the first runs on
        # another handle of the same problem, so the third cannot run on
        # the first's resident factors instead)
        op_first = nep.SplitOperator.from_problem(prob)
        t_first = srv.submit(op_first, con, V, N, L, K, max_eigs=16, want_X=True)
        t_bad = srv.submit(op_b, Contour.circle(0.0, 1.0), wl.probes(8, 8, 0), N, L, K, max_eigs=16)
        t_good = srv.submit(op, con, V, N, L, K, max_eigs=16, want_X=True)
        r_first, r_bad, r_good = srv.wait(t_first), srv.wait(t_bad), srv.wait(t_good)
    finally:
        srv.close()
    assert nep.binding.ERRORS[r_bad["status"]] == "NEP_ERR_NOT_HOLOMORPHIC"
    assert r_bad["t_start"] == r_good["t_start"]  # one batch
    for r in (r_first, r_good):
        assert r["status"] == 0, nep.binding.ERRORS.get(r["status"])
        assert r["m"] == alone["m"]
        assert np.array_equal(r["lam"], alone["lam"])
        assert np.array_equal(r["eta"], alone["eta"])
        assert np.array_equal(r["X"], alone["X"])


def test_server_budget(nep):
    """A query larger than the whole budget is refused at submit; a budget
    that holds one query at a time still serves every query."""
    cfg = wl.config0()
    op = nep.SplitOperator.from_problem(cfg["problem"])
    srv = nep.Server(hbm_budget=4 << 20, max_inflight=4, nstreams=2)
    try:
        with pytest.raises(nep.NepError) as ei:
            srv.submit(op, cfg["contour"], cfg["V"], 32, 8, 2)
        assert ei.value.name == "NEP_ERR_BUSY"
    finally:
        srv.close()
    one = 40 << 20  # holds one n=200 query (about 33 MB) but not two
    srv = nep.Server(hbm_budget=one, max_inflight=4, nstreams=2)
    try:
        ts = [srv.submit(op, cfg["contour"], cfg["V"], 32, 8, 2) for _ in range(4)]
        rs = [srv.wait(t) for t in ts]
    finally:
        srv.close()
    for r in rs:
        assert r["status"] == 0
        assert np.array_equal(r["lam"], rs[0]["lam"])
    # served one after another: no two queries overlap in time
    spans = sorted((r["t_start"], r["t_done"]) for r in rs)
    for a, b in zip(spans, spans[1:]):
        assert b[0] >= a[1]


def test_server_follow_up_runs_on_resident_factors(nep):
    """A query with the operator, contour and options of a finished one runs
    on the factors that query left resident (no assembly or LU): reused is
    set and the result equals a fresh run of the same probes bit for bit.
    Other N, another handle of the same problem, or an evicted plan mean new
    factors.  A small budget holds one plan at a time: a larger query evicts
    the resident one."""
    p = wl.loaded_string(200, sigma=1.0, a_scale=1.0)
    con = Contour.circle(100.0, 90.0)
    N, L, K, me = 32, 8, 2, 16
    op = nep.SplitOperator.from_problem(p)
    V1, V2, V3 = (wl.probes(200, L, s) for s in (41, 42, 43))
    alone2 = _alone(nep, op, con, V2, N, L, K, "mixed", me)
    alone3 = _alone(nep, op, con, V3, N, L, K, "mixed", me)
    srv = nep.Server(hbm_budget=1 << 30, max_inflight=8, nstreams=2)
    try:
        r1 = srv.wait(srv.submit(op, con, V1, N, L, K, max_eigs=me, want_X=True))
        r2 = srv.wait(srv.submit(op, con, V2, N, L, K, max_eigs=me, want_X=True))
        r3 = srv.wait(srv.submit(op, con, V3, 64, L, K, max_eigs=me, want_X=True))
        op_b = nep.SplitOperator.from_problem(p)  # same data, another handle
        r4 = srv.wait(srv.submit(op_b, con, V3, N, L, K, max_eigs=me, want_X=True))
        # two follow-ups queued together: one pass on the resident plan runs
        # the first, the second waits for it (one member, one pass)
        ta = srv.submit(op, con, V2, N, L, K, max_eigs=me, want_X=True)
        tb = srv.submit(op, con, V3, N, L, K, max_eigs=me, want_X=True)
        ra, rb = srv.wait(ta), srv.wait(tb)
    finally:
        srv.close()
    assert [r["status"] for r in (r1, r2, r3, r4, ra, rb)] == [0] * 6
    assert not r1["reused"] and r2["reused"] and not r3["reused"] and not r4["reused"]
    assert ra["reused"] and rb["reused"]
    for r, a in ((r2, alone2), (ra, alone2), (r4, alone3), (rb, alone3)):
        assert r["m"] == a["m"]
        assert np.array_equal(r["lam"], a["lam"])
        assert np.array_equal(r["eta"], a["eta"])
        assert np.array_equal(r["X"], a["X"])
    print("first", r1["t_done"] - r1["t_start"], "on resident factors", r2["t_done"] - r2["t_start"])

    # eviction: a 140 MB budget holds the n=200 plan (about 30 MB) or the
    # n=600 one (about 130 MB), not both
    q = wl.loaded_string(600, sigma=1.0, a_scale=1.0)
    op_q = nep.SplitOperator.from_problem(q)
    srv = nep.Server(hbm_budget=140 << 20, max_inflight=4, nstreams=1)
    try:
        s1 = srv.wait(srv.submit(op, con, V1, N, L, K, max_eigs=me))
        s2 = srv.wait(srv.submit(op_q, con, wl.probes(600, L, 5), N, L, K, max_eigs=me))
        s3 = srv.wait(srv.submit(op, con, V2, N, L, K, max_eigs=me))
        s4 = srv.wait(srv.submit(op, con, V3, N, L, K, max_eigs=me))
    finally:
        srv.close()
    assert [r["status"] for r in (s1, s2, s3, s4)] == [0] * 4
    assert [r["reused"] for r in (s1, s2, s3, s4)] == [False, False, False, True]
    assert np.array_equal(s3["lam"], alone2["lam"]) and np.array_equal(s4["lam"], alone3["lam"])


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_server_probe_pool_augments_saturated_query(nep, prec):
    """Delay problem with 9 eigenvalues inside circle(-1, 0.6) and K = 2: 8 and
    16 probes saturate the moments' rank.  Submitted with a pool of 32 probe
    columns, the query solves further blocks of 8 on the same factors until 24
    resolve the rank, and returns what nep_eigs returns on a handle, bit for
    bit, also when a second submission runs on the resident factors and
    beside other queries.  Without a pool the query reports the saturation;
    queries whose rank does not saturate use their first L columns only."""
    B = nep.binding
    p = wl.delay_problem(120, tau=1.0, seed=7)
    con = Contour.circle(-1.0, 0.6)
    N, L, K, Lmax = 32, 8, 2, 32
    V = wl.probes(120, Lmax, 20)
    op = nep.SplitOperator.from_problem(p)
    X = torch.zeros((64, 120), dtype=torch.complex128, device="cuda")
    ref = B.nep_eigs(op.h, con, B.opts_struct(N, L, K, prec), nep.device_probes(V), Lmax, X, max_eigs=64)
    assert ref["L_used"] == 24
    others = [c for c in _mix_cases() if c[2] == N][:2]  # rational, same N, L, K: they share the batch
    oops = [nep.SplitOperator.from_problem(c[0]) for c in others]
    alone = [_alone(nep, o, c[1], c[5], c[2], c[3], c[4], prec, 32) for o, c in zip(oops, others)]
    srv = nep.Server(hbm_budget=1 << 30, max_inflight=16, nstreams=2)
    try:
        tickets = [srv.submit(op, con, V, N, L, K, prec=prec, max_eigs=64)]
        tickets += [srv.submit(o, c[1], np.hstack([c[5], wl.probes(c[0].n, L, 77)]), c[2], c[3], c[4],
                               prec=prec, max_eigs=32) for o, c in zip(oops, others)]
        res = [srv.wait(t) for t in tickets]
        # after completion, the same key runs on the resident factors
        res.append(srv.wait(srv.submit(op, con, V, N, L, K, prec=prec, max_eigs=64)))
        res.append(srv.wait(srv.submit(op, con, V[:, :L], N, L, K, prec=prec, max_eigs=64)))  # no pool
    finally:
        srv.close()
    for r in (res[0], res[3]):
        assert r["status"] == 0 and r["L_used"] == 24 and r["m"] == ref["m"], (r["status"], r["L_used"], r["m"])
        assert np.array_equal(r["lam"], ref["lam"])
        assert np.array_equal(r["eta"], ref["eta"])
        assert np.array_equal(r["inside"], ref["inside"])
    assert res[3]["reused"] and res[4]["reused"]
    assert B.ERRORS.get(res[4]["status"]) == "NEP_ERR_RANK" and res[4]["L_used"] == L
    for r, a in zip(res[1:3], alone):
        assert r["status"] == 0 and r["L_used"] == L
        assert np.array_equal(r["lam"], a["lam"]) and np.array_equal(r["eta"], a["eta"])
    for o in oops:
        o.close()
    op.close()
