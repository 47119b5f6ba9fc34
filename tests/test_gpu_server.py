"""GPU request server (dwf_submit / dwf_poll): continuous batching of solves,
each with its own quark mass, in the multi-right-hand-side kernels.

Every served solve meets the bar of a plain solve: ||b - D x|| / ||b|| <= 1e-10
with the oracle's FP64 operator (at the request's mass), and it equals the
solution that dwf_solve finds for that request alone.  The per-slot arithmetic
does not depend on the other slots, so the two agree to the last bit; the test
allows 1e-12 (relative).
"""
import ctypes
import time

import numpy as np
import pytest

import dwf_inputs as inp
import oracle
from _util import Problem, rel

pytestmark = pytest.mark.gpu

TOL_RES = 1e-10
TOL_FWD = 1e-8
SMALL = Problem.workload("shamir_4x4x4x4_ns8")
# a second field of the same shape and operator parameters (another gauge seed)
_w = inp.workload("shamir_4x4x4x4_ns8")
SMALL2 = Problem(_w["dims"], _w["ns"], _w["m0"], _w["mq"], _w["sigma"], _w["omega"], _w["eps"], 4711, 4712)
_rng = np.random.default_rng(191)
RAGGED = Problem((4, 6, 2, 8), 5, 1.6, 0.1, _rng.uniform(0.2, 1.4, 5), _rng.uniform(0.5, 1.5, 5), 0.5, 51, 52,
                 antiperiodic=True)
MASSES = [0.02, 0.05, 0.1, 0.3]


def rhs(P, k):
    return inp.gaussian_spinor(P.dims, P.ns, seed=7000 + k)


def ctx_mass(P, mq, **kw):
    import paper_1101_0423_amd as dwf
    return dwf.Context(P.U, P.dims, P.ns, P.m0, mq, P.sigma, P.omega, antiperiodic_t=P.antiperiodic, **kw)


def wait(ticket, shape, timeout_s=90):
    import paper_1101_0423_amd as dwf
    t0 = time.time()
    while True:
        rc, x, st = dwf.poll(ticket, shape, timeout_us=200000)
        if rc != dwf.DWF_PENDING:
            return rc, x, st
        assert time.time() - t0 < timeout_s, "request did not finish"


def true_res(P, mq, b, x):
    return oracle.true_residual(P.U, P.dims, P.ns, P.m0, mq, P.sigma, P.omega, b, x, bct=P.bct)


def test_mixed_masses_each_equals_alone():
    """Requests on three resident fields at once (two of the same shape, one
    ragged), several masses each: every result equals its solve alone."""
    import paper_1101_0423_amd as dwf
    print("[server] 4^4x8 (two fields) + ragged, masses", MASSES, flush=True)
    dwf.server_stats(reset=True)
    cs, cs2, cr = SMALL.context(), SMALL2.context(), RAGGED.context()
    try:
        jobs = []
        for k in range(8):
            mq = MASSES[k % len(MASSES)]
            b = rhs(SMALL, k)
            jobs.append((SMALL, mq, b, cs.submit(b, mq=mq)))
        for k in range(4):
            mq = MASSES[(k + 1) % len(MASSES)]
            b = rhs(SMALL2, 50 + k)
            jobs.append((SMALL2, mq, b, cs2.submit(b, mq=mq)))
        for k in range(2):
            b = rhs(RAGGED, 100 + k)
            jobs.append((RAGGED, RAGGED.mq, b, cr.submit(b)))
        shape = {id(SMALL): cs.spinor_shape(), id(SMALL2): cs2.spinor_shape(), id(RAGGED): cr.spinor_shape()}
        out = []
        for P, mq, b, t in jobs:
            rc, x, st = wait(t, shape[id(P)])
            assert rc == dwf.DWF_OK, st
            assert st["true_residual"] <= TOL_RES, st
            r = true_res(P, mq, b, x)
            assert r <= TOL_RES, r
            out.append((P, mq, b, x))
        s = dwf.server_stats()
        assert s["completed"] == len(jobs) and s["admitted"] == len(jobs)
        assert s["peak_batch"] >= 2
        assert 0 < s["p50_latency"] <= s["p99_latency"]
        assert s["busy_seconds"] > 0
    finally:
        cs.close()
        cs2.close()
        cr.close()
    # each request alone, through dwf_solve on a context with its mass
    for P, mq, b, x in out:
        c = ctx_mass(P, mq)
        try:
            xa, st, rc = c.solve(b)
            assert rc == dwf.DWF_OK
            d = rel(x, xa)
            print(f"[server] mq={mq} alone vs served: {d:.2e}", flush=True)
            assert d <= 1e-12, d
        finally:
            c.close()


def test_served_solution_matches_oracle():
    # also the ownership rules of the served form: dwf_submit copies b (the
    # caller's array is overwritten right after it returns), and dwf_poll
    # leaves x untouched while the request is pending
    import paper_1101_0423_amd as dwf
    mq = 0.05
    b = rhs(SMALL, 50)
    b_submitted = b.copy()
    c = SMALL.context()
    try:
        t = c.submit(b, mq=mq)
        b[...] = rhs(SMALL, 51)
        xs = np.full(c.spinor_shape(), 7.0)
        st0 = dwf.SolveStats()
        rc = dwf.lib().dwf_poll(ctypes.c_uint64(t), xs.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                ctypes.byref(st0), 0)
        print(f"[serve] first poll: {'pending' if rc == dwf.DWF_PENDING else 'final'}", flush=True)
        if rc == dwf.DWF_PENDING:
            assert np.all(xs == 7.0)
            rc, x, st = wait(t, c.spinor_shape())
        else:  # already done: that poll collected it
            x = xs
    finally:
        c.close()
    assert rc == dwf.DWF_OK
    b = b_submitted
    xo, info = oracle.solve(SMALL.U, SMALL.dims, SMALL.ns, SMALL.m0, mq, SMALL.sigma, SMALL.omega, b, tol=1e-12)
    assert info["converged"]
    err = rel(x, xo)
    assert err <= TOL_FWD, err


@pytest.mark.parametrize("prec", [0, 2], ids=["fp64", "fp16"])
def test_precision_lanes(prec):
    """Requests with another inner precision run in a lane of their own."""
    import paper_1101_0423_amd as dwf
    c = SMALL.context()
    try:
        bs = [rhs(SMALL, 200 + k) for k in range(3)]
        ts = [c.submit(b, mq=MASSES[k], inner_prec=prec) for k, b in enumerate(bs)]
        t32 = c.submit(bs[0], mq=MASSES[0])
        for k, (b, t) in enumerate(zip(bs, ts)):
            rc, x, st = wait(t, c.spinor_shape())
            assert rc == dwf.DWF_OK, st
            assert true_res(SMALL, MASSES[k], b, x) <= TOL_RES
        rc, x, st = wait(t32, c.spinor_shape())
        assert rc == dwf.DWF_OK
    finally:
        c.close()


def test_tiny_budget_waits_for_memory():
    """A budget that holds one lane of one slot: the second operator's requests
    wait until the first lane is idle and gives its memory back."""
    import paper_1101_0423_amd as dwf
    V5h = 4 ** 4 // 2 * SMALL.ns
    per_slot = (8 * V5h * 192 + 6 * V5h * 96) * 1.1 + 64 * 1024
    staging = 4 ** 4 * SMALL.ns * 24 * 8
    budget = int(1.6 * per_slot + staging)
    print(f"[server] budget {budget} B", flush=True)
    dwf.server_stats(reset=True)
    ca = ctx_mass(SMALL, 0.05, hbm_budget_bytes=budget)
    cb = ctx_mass(SMALL, 0.1, hbm_budget_bytes=budget)
    try:
        jobs = []
        for k in range(3):
            b = rhs(SMALL, 300 + k)
            jobs.append((0.05, b, ca.submit(b)))
            b = rhs(SMALL, 400 + k)
            jobs.append((0.1, b, cb.submit(b)))
        for mq, b, t in jobs:
            rc, x, st = wait(t, ca.spinor_shape())
            assert rc == dwf.DWF_OK, st
            assert true_res(SMALL, mq, b, x) <= TOL_RES
        s = dwf.server_stats()
        assert s["waits_for_memory"] >= 1, s
        assert s["peak_batch"] == 1, s
        assert s["completed"] == len(jobs)
    finally:
        ca.close()
        cb.close()


def test_destroy_with_requests_in_flight():
    """Closing a context ends its requests: each either finished or reports
    DWF_EINVAL; afterwards the tickets are unknown."""
    import paper_1101_0423_amd as dwf
    c = SMALL.context()
    shape = c.spinor_shape()
    ts = [c.submit(rhs(SMALL, 500 + k), mq=MASSES[k % 4]) for k in range(6)]
    c.close()
    for t in ts:
        try:
            rc, x, st = dwf.poll(t, shape, timeout_us=0)
            assert rc == dwf.DWF_OK
        except dwf.DwfError as e:
            assert e.code == dwf.DWF_EINVAL
        with pytest.raises(dwf.DwfError) as ei:
            dwf.poll(t, shape, timeout_us=0)
        assert ei.value.code == dwf.DWF_ENOTFOUND


def test_submit_rejects_bad_requests():
    import paper_1101_0423_amd as dwf
    c = SMALL.context()
    try:
        with pytest.raises(dwf.DwfError) as ei:
            c.submit(SMALL.b, tol=0.0)
        assert ei.value.code == dwf.DWF_EINVAL
        with pytest.raises(dwf.DwfError) as ei:
            c.submit(SMALL.b, inner_prec=7)
        assert ei.value.code == dwf.DWF_EINVAL
    finally:
        c.close()


def test_request_during_lane_release_is_served():
    """A budget that holds one lane: a request for operator A arrives just as
    A's idle lane gives its memory back to a waiting request for operator B.
    It must wait for a new lane and be served, not fail as if its context had
    been destroyed."""
    import paper_1101_0423_amd as dwf
    V5h = 4 ** 4 // 2 * SMALL.ns
    per_slot = (8 * V5h * 192 + 6 * V5h * 96) * 1.1 + 64 * 1024
    staging = 4 ** 4 * SMALL.ns * 24 * 8
    budget = int(1.6 * per_slot + staging)
    ca = ctx_mass(SMALL, 0.05, hbm_budget_bytes=budget)
    cb = ctx_mass(SMALL, 0.1, hbm_budget_bytes=budget)
    try:
        for k in range(4):
            ba, bb, ba2 = rhs(SMALL, 600 + k), rhs(SMALL, 610 + k), rhs(SMALL, 620 + k)
            ta = ca.submit(ba)
            tb = cb.submit(bb)                      # waits for A's lane to go
            rc, x, st = wait(ta, ca.spinor_shape())
            assert rc == dwf.DWF_OK, st
            ta2 = ca.submit(ba2)                    # A's lane is idle and releasing now
            for mq, b, t in ((0.1, bb, tb), (0.05, ba2, ta2)):
                rc, x, st = wait(t, ca.spinor_shape())
                assert rc == dwf.DWF_OK, st
                assert true_res(SMALL, mq, b, x) <= TOL_RES
    finally:
        ca.close()
        cb.close()
