"""GPU solves of C C^dag w = b on the odd sites (the system of the hybrid Monte
Carlo force, solved by CG on C C^dag): the same kernels as D x = b, with the
solution accumulating the search directions and an FP64 outer residual
b - C C^dag w.  Bar: ||b_o - C C^dag w|| / ||b_o|| <= 1e-10 with the oracle's
FP64 C and C^dag on the GPU's w, even sites of w exactly zero, and agreement
with the oracle's own solution (Algorithm 1, tol 1e-13) within the
conditioning of C C^dag (forward error <= 1e-10 x kappa_est, kappa_est from
the oracle's Lanczos-free bound ||w|| ||b||^-1 lambda_max; see the test).
"""
import numpy as np
import pytest

import dwf_inputs as inp
import oracle
from _util import Problem, on_parity, rel

pytestmark = pytest.mark.gpu

SMALL = Problem.workload("shamir_4x4x4x4_ns8")
_rng = np.random.default_rng(313)
RAGGED = Problem((4, 6, 2, 8), 5, 1.6, 0.1, _rng.uniform(0.2, 1.4, 5), _rng.uniform(0.5, 1.5, 5), 0.5, 61, 62,
                 antiperiodic=True)
ODWF8 = Problem((8, 8, 8, 8), 16, 1.8, 0.05, *(2 * [_rng.uniform(0.5, 1.5, 16)]), 0.5, 63, 64)


def ccdag(P, w):
    a = P.oargs()
    return oracle.schur_c(*a, oracle.schur_cdag(*a, w, bct=P.bct), bct=P.bct)


def residual(P, b, w):
    bo = on_parity(b, P.dims, 1)
    return np.linalg.norm(bo - ccdag(P, w)) / np.linalg.norm(bo)


_REF = {}


def reference(P, key):
    if key not in _REF:
        w, info = oracle.solve_ccdag(*P.oargs(), P.b, tol=1e-13, bct=P.bct)
        assert info["converged"]
        _REF[key] = w
    return _REF[key]


def forward_bound(P, w_ref):
    """Forward error allowed for a residual of 1e-10: 1e-10 ||A|| ||A^-1 b|| / ||b||
    <= 1e-10 kappa(A), with ||A|| from power iteration on A = C C^dag."""
    v = inp.gaussian_spinor(P.dims, P.ns, seed=5)
    v = on_parity(v, P.dims, 1)
    for _ in range(30):
        v = ccdag(P, v)
        lam = np.linalg.norm(v)
        v /= lam
    bo = on_parity(P.b, P.dims, 1)
    return 1e-10 * lam * np.linalg.norm(w_ref) / np.linalg.norm(bo)


@pytest.mark.parametrize("name,P", [("shamir4", SMALL), ("ragged", RAGGED), ("odwf8", ODWF8)])
@pytest.mark.parametrize("prec", [0, 1, 2], ids=["fp64", "fp32", "fp16"])
def test_force_solve(name, P, prec):
    import paper_1101_0423_amd as dwf
    print(f"[force] {name} prec={prec}", flush=True)
    c = P.context()
    try:
        w, st, rc = c.solve(P.b, inner_prec=prec, system=dwf.SYSTEM_CCDAG)
    finally:
        c.close()
    assert rc == dwf.DWF_OK, st
    assert np.all(on_parity(w, P.dims, 0) == 0)
    r = residual(P, P.b, w)
    assert r <= 1e-10, r
    assert st[0]["true_residual"] <= 1e-10
    assert abs(st[0]["true_residual"] - r) <= 1e-3 * r + 1e-13
    wref = reference(P, name)
    err = rel(w, wref)
    bound = forward_bound(P, wref)
    print(f"[force] {name} prec={prec}: residual {r:.2e}, forward error {err:.2e} (bound {bound:.2e}), "
          f"iters {st[0]['iters']}", flush=True)
    assert err <= max(bound, 1e-10), (err, bound)


def test_force_and_plain_share_a_batch():
    """Both systems in one batch of the server: each equals its solve alone."""
    import paper_1101_0423_amd as dwf
    c = SMALL.context()
    try:
        bs = [inp.gaussian_spinor(SMALL.dims, SMALL.ns, seed=800 + k) for k in range(4)]
        systems = [dwf.SYSTEM_CCDAG, dwf.SYSTEM_D, dwf.SYSTEM_CCDAG, dwf.SYSTEM_D]
        ts = [c.submit(b, system=sy) for b, sy in zip(bs, systems)]
        for b, sy, t in zip(bs, systems, ts):
            while True:
                rc, x, st = dwf.poll(t, c.spinor_shape(), timeout_us=200000)
                if rc != dwf.DWF_PENDING:
                    break
            assert rc == dwf.DWF_OK
            xa, sta, rca = c.solve(b, system=sy)
            assert rel(x, xa) <= 1e-12
            if sy == dwf.SYSTEM_CCDAG:
                assert residual(SMALL, b, x) <= 1e-10
            else:
                assert oracle.true_residual(*SMALL.oargs(), b, x) <= 1e-10
    finally:
        c.close()
