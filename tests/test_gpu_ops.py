"""GPU operator parity: every dwf_apply operator against the FP64 oracle.

Bars, norm-wise |got - exp| / |exp| and element-wise max|got - exp| / max|exp|:
FP64 1e-13 and 4e-13; FP32 1e-6 and 4e-6, with 12-real links (what the FP32
solver uses) and 18-real links alike; FP16 storage 1e-3 and 1.5e-3.  The FP16
bar comes from the format: binary16 keeps 11 significant bits, so a component
is stored to 2^-12 = 2.4e-4 of its site's largest component, and an operator
such as C C^dag rounds its input, its intermediates and its output and reads
binary16 links, each adding an error of that size.  Measured over these shapes
and the full 16^3x32x16 lattice: at most 3.8e-4 norm-wise and 5.4e-4
element-wise (printed by each case), so the bars leave a factor 2.6-2.8.
Shapes span several workgroups and a ragged last workgroup; the full
16^3x32x16 workload runs in the launch configuration the solver uses.
"""
import numpy as np
import pytest

import dwf_inputs as inp
import oracle
from _util import Problem, max_rel, on_parity, rel

pytestmark = pytest.mark.gpu

TOL = {0: 1e-13, 1: 1e-6, 2: 1e-3}              # norm-wise, by storage precision
TOL_EL = {0: 4e-13, 1: 4e-6, 2: 1.5e-3}          # element-wise
# storage precision | link storage (dwf_apply's prec argument)
PRECS = {"fp64": 0, "fp32-12real": 1 | 0x200, "fp32-18real": 1 | 0x100, "fp16": 2}


def problems():
    rng = np.random.default_rng(77)
    ns5_s, ns5_w = rng.uniform(0.2, 1.4, 5), rng.uniform(0.5, 1.5, 5)
    return {
        # 4^4 x 8 Shamir (the small configuration)
        "shamir4": Problem.workload("shamir_4x4x4x4_ns8"),
        # unequal extents, Ns = 5, sigma != omega, antiperiodic time: several
        # workgroups with a ragged tail (V4h = 192 sites, 51 per FP32 workgroup)
        "ragged": Problem((4, 6, 2, 8), 5, 1.6, 0.1, ns5_s, ns5_w, 0.5, 31, 32, antiperiodic=True),
        # Ns = 16 optimal-DWF weights on 8^3 x 4
        "odwf8": Problem((8, 8, 8, 4), 16, 1.8, 0.01, *(2 * [rng.uniform(0.5, 1.5, 16)]), 0.5, 33, 34),
        # Ns = 1 and Ns = 32 edges
        "ns1": Problem((4, 4, 2, 2), 1, 1.2, 0.3, [0.7], [1.3], 0.5, 35, 36),
        "ns32": Problem((4, 2, 2, 4), 32, 1.8, 0.05, np.zeros(32), np.ones(32), 0.5, 37, 38),
    }


PROBS = problems()


def oracle_op(P, op, psi):
    import paper_1101_0423_amd as dwf
    a = P.oargs()
    U, dims, ns, m0, mq, sg, om = a
    if op == dwf.OP_DW:
        return oracle.dw(U, dims, ns, m0, psi, bct=P.bct)
    if op == dwf.OP_HOP_EO:
        return oracle.hop(U, dims, ns, 0, psi, bct=P.bct)
    if op == dwf.OP_HOP_OE:
        return oracle.hop(U, dims, ns, 1, psi, bct=P.bct)
    if op in (dwf.OP_M5, dwf.OP_M5T):
        mp, mm = oracle.m5(ns, m0, mq, sg, om)
        if op == dwf.OP_M5T:
            mp, mm = mp.T, mm.T
        return oracle.apply_s(dims, ns, mp, mm, psi)
    if op == dwf.OP_C:
        return oracle.schur_c(*a, on_parity(psi, dims, 1), bct=P.bct)
    if op == dwf.OP_CDAG:
        return oracle.schur_cdag(*a, on_parity(psi, dims, 1), bct=P.bct)
    if op == dwf.OP_CCDAG:
        t = oracle.schur_cdag(*a, on_parity(psi, dims, 1), bct=P.bct)
        return oracle.schur_c(*a, t, bct=P.bct)
    if op == dwf.OP_D:
        return oracle.d5(*a, psi, bct=P.bct)
    if op == dwf.OP_DDAG:
        return oracle.d5dag(*a, psi, bct=P.bct)
    raise ValueError(op)


OPS = list(range(10))
OP_NAMES = ["DW", "HOP_EO", "HOP_OE", "M5", "M5T", "C", "CDAG", "CCDAG", "D", "DDAG"]


@pytest.fixture(scope="module")
def contexts():
    ctx = {}
    yield ctx
    for c in ctx.values():
        c.close()


def get_ctx(contexts, name):
    if name not in contexts:
        contexts[name] = PROBS[name].context()
    return contexts[name]


@pytest.mark.parametrize("name", list(PROBS))
@pytest.mark.parametrize("op", OPS, ids=OP_NAMES)
@pytest.mark.parametrize("prec", list(PRECS.values()), ids=list(PRECS))
def test_operator_parity(contexts, name, op, prec):
    P = PROBS[name]
    print(f"[ops] {name} {OP_NAMES[op]} prec={prec:#x}", flush=True)
    ctx = get_ctx(contexts, name)
    psi = P.b
    got = ctx.apply(op, psi, prec=prec)
    exp = oracle_op(P, op, psi)
    e_n, e_el = rel(got, exp), max_rel(got, exp)
    print(f"[ops]   error norm-wise {e_n:.3e}, element-wise {e_el:.3e}", flush=True)
    assert e_n <= TOL[prec & 0xff], (e_n, TOL[prec & 0xff])
    assert e_el <= TOL_EL[prec & 0xff], (e_el, TOL_EL[prec & 0xff])
    if prec == 0:
        # the parity a block operator does not touch is exactly zero
        import paper_1101_0423_amd as dwf
        zero_par = {dwf.OP_HOP_EO: 1, dwf.OP_HOP_OE: 0, dwf.OP_C: 0, dwf.OP_CDAG: 0, dwf.OP_CCDAG: 0}.get(op)
        if zero_par is not None:
            assert np.all(on_parity(got, P.dims, zero_par) == 0)


def test_multi_rhs_apply_equals_single(contexts):
    import paper_1101_0423_amd as dwf
    P = PROBS["ragged"]
    ctx = get_ctx(contexts, "ragged")
    bs = inp.gaussian_spinor(P.dims, P.ns, seed=99, nrhs=3)
    for op in (dwf.OP_C, dwf.OP_CDAG, dwf.OP_D):
        for prec in (0, PRECS["fp32-12real"], PRECS["fp32-18real"]):
            many = ctx.apply(op, bs, prec=prec)
            for k in range(3):
                one = ctx.apply(op, bs[k], prec=prec)
                assert np.array_equal(many[k], one)


def test_gamma5_hermiticity_on_gpu(contexts):
    import paper_1101_0423_amd as dwf
    P = PROBS["odwf8"]
    ctx = get_ctx(contexts, "odwf8")
    phi = inp.gaussian_spinor(P.dims, P.ns, seed=5)
    psi = inp.gaussian_spinor(P.dims, P.ns, seed=6)
    g5 = np.ones(24)
    g5[12:] = -1
    lhs = np.vdot(inp.host_to_complex(phi), inp.host_to_complex(g5 * ctx.apply(dwf.OP_DW, g5 * psi)))
    rhs = np.vdot(inp.host_to_complex(ctx.apply(dwf.OP_DW, phi)), inp.host_to_complex(psi))
    assert abs(lhs - rhs) <= 1e-12 * abs(rhs)
    # C and C^dag are adjoints on odd-supported vectors
    po, so = on_parity(phi, P.dims, 1), on_parity(psi, P.dims, 1)
    a = np.vdot(inp.host_to_complex(po), inp.host_to_complex(ctx.apply(dwf.OP_C, so)))
    b = np.vdot(inp.host_to_complex(ctx.apply(dwf.OP_CDAG, po)), inp.host_to_complex(so))
    assert abs(a - b) <= 1e-12 * abs(a)


def test_contexts_share_one_field():
    """Contexts on the same gauge field share its resident links (they do not
    depend on Ns, the masses or the time boundary): the second context keeps
    working after the first one is destroyed, with its own Ns and boundary."""
    import paper_1101_0423_amd as dwf
    P = PROBS["ragged"]
    a = dwf.Context(P.U, P.dims, 8, 1.8, 0.02, np.zeros(8), np.ones(8), antiperiodic_t=False)
    b = P.context()
    a.close()
    got = b.apply(dwf.OP_D, P.b, prec=0)
    b.close()
    exp = oracle_op(P, dwf.OP_D, P.b)
    assert rel(got, exp) <= TOL[0]


def test_full_size_operator_parity():
    """16^3x32, Ns = 16, the configuration of the primary solve: C, C^dag and D
    in FP64, FP32 (12-real links, the solver's, and 18-real) and FP16 storage
    against the oracle over the whole lattice."""
    import paper_1101_0423_amd as dwf
    P = Problem.workload("odwf_16x16x16x32_ns16")
    ctx = P.context()
    try:
        for op in (dwf.OP_C, dwf.OP_CDAG, dwf.OP_D):
            print(f"[ops] full-size {OP_NAMES[op]}", flush=True)
            exp = oracle_op(P, op, P.b)
            for name, prec in PRECS.items():
                got = ctx.apply(op, P.b, prec=prec)
                e_n, e_el = rel(got, exp), max_rel(got, exp)
                print(f"[ops]   {name}: norm-wise {e_n:.3e}, element-wise {e_el:.3e}", flush=True)
                assert e_n <= TOL[prec & 0xff], (op, name, e_n)
                assert e_el <= TOL_EL[prec & 0xff], (op, name, e_el)
    finally:
        ctx.close()


def _cplx(a, ns):
    """host spinor -> complex [t][z][y][x][s][spin][colour]"""
    z = inp.host_to_complex(a)
    return z.reshape(z.shape[:-1] + (4, 3))


def _real(z):
    return inp.complex_to_host(z.reshape(z.shape[:-2] + (12,)))


def _gammas():
    """Chiral basis: gamma_k = [[0, -i sigma_k], [i sigma_k, 0]] (mu = 0, 1, 2 for
    k = 1, 2, 3), gamma_4 = [[0, 1], [1, 0]] (mu = 3)."""
    sig = [np.array([[0, 1], [1, 0]], complex), np.array([[0, -1j], [1j, 0]]), np.array([[1, 0], [0, -1]], complex)]
    z = np.zeros((2, 2), complex)
    g = [np.block([[z, -1j * s], [1j * s, z]]) for s in sig]
    g.append(np.block([[z, np.eye(2)], [np.eye(2), z]]))
    return g


@pytest.mark.parametrize("prec", [0, PRECS["fp32-12real"], PRECS["fp32-18real"]], ids=["fp64", "fp32-12", "fp32-18"])
@pytest.mark.parametrize("bct", [1.0, -1.0], ids=["periodic", "antiperiodic"])
def test_unit_link_plane_waves_on_gpu(prec, bct):
    """With U = 1 the GPU's D_w (Eq. (2)) maps a plane wave e^{ipx} chi_s to
    [(4 - m0 - sum_mu cos p_mu) + i sum_mu gamma_mu sin p_mu] e^{ipx} chi_s on
    every slice: the closed form, written out here, not taken from the oracle.
    Antiperiodic time shifts p_t by pi / Lt."""
    import paper_1101_0423_amd as dwf
    dims, ns, m0 = (4, 6, 2, 8), 3, 1.3
    lx, ly, lz, lt = dims
    print(f"[ops] plane waves prec={prec} bct={bct}", flush=True)
    c = dwf.Context(inp.unit_gauge(dims), dims, ns, m0, 0.1, np.zeros(ns), np.ones(ns), antiperiodic_t=bct < 0)
    try:
        t, z, y, x = np.meshgrid(range(lt), range(lz), range(ly), range(lx), indexing="ij")
        g = _gammas()
        rng = np.random.default_rng(17)
        shift = 0.5 if bct < 0 else 0.0
        for n in [(1, 2, 1, 3), (0, 1, 0, 0), (3, 5, 1, 7)]:
            p = [2 * np.pi * n[0] / lx, 2 * np.pi * n[1] / ly, 2 * np.pi * n[2] / lz, 2 * np.pi * (n[3] + shift) / lt]
            phase = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))[..., None, None, None]
            chi = rng.normal(size=(ns, 4, 3)) + 1j * rng.normal(size=(ns, 4, 3))
            W = 4 - m0 - sum(np.cos(pm) for pm in p)
            M = W * np.eye(4) + 1j * sum(g[m] * np.sin(p[m]) for m in range(4))
            exp = phase * np.einsum("ij,sjc->sic", M, chi)
            got = _cplx(c.apply(dwf.OP_DW, _real(phase * chi), prec=prec), ns)
            err = np.linalg.norm(got - exp) / np.linalg.norm(exp)
            assert err <= TOL[prec & 0xff], (n, err)
    finally:
        c.close()


@pytest.mark.parametrize("prec", [0, PRECS["fp32-12real"], PRECS["fp32-18real"]], ids=["fp64", "fp32-12", "fp32-18"])
def test_gauge_covariance_on_gpu(prec):
    """D_w[U^g](g psi) = g D_w[U] psi and the same for the Schur operator C,
    U^g_mu(x) = g(x) U_mu(x) g(x + mu)^dag, on the GPU alone (two contexts,
    antiperiodic time, ragged workgroups)."""
    import paper_1101_0423_amd as dwf
    P = PROBS["ragged"]
    print(f"[ops] gauge covariance prec={prec}", flush=True)
    gt = inp.gauge_transform(P.dims, 0.7, seed=41)
    Uc = P.U[..., 0] + 1j * P.U[..., 1]
    Ug = np.empty_like(Uc)
    for mu in range(4):
        gshift = np.roll(gt, -1, axis=3 - mu)  # g(x + mu); array axes are [t][z][y][x]
        Ug[..., mu, :, :] = gt @ Uc[..., mu, :, :] @ np.conj(np.swapaxes(gshift, -1, -2))
    Ugr = np.stack([Ug.real, Ug.imag], axis=-1)

    def rot(a):
        return _real(np.einsum("tzyxab,tzyxsib->tzyxsia", gt, _cplx(a, P.ns)))

    c1 = P.context()
    c2 = dwf.Context(Ugr, *P.args, antiperiodic_t=True)
    try:
        psi = P.b
        for op in (dwf.OP_DW, dwf.OP_C):
            lhs = c2.apply(op, rot(psi), prec=prec)
            rhs = rot(c1.apply(op, psi, prec=prec))
            assert rel(lhs, rhs) <= 2 * TOL[prec & 0xff], (op, rel(lhs, rhs))
    finally:
        c1.close()
        c2.close()


# 24 x 24 z-planes (18 FP32 / 36 FP64 blocks of 16 / 8 sites) with 4 t-slices
# per XCD chunk: the launches walk the planes in tiles (the order used at
# 24^3 x 48), which every other operator test here leaves untouched
_rng_t = np.random.default_rng(81)
TILED = Problem((24, 24, 2, 32), 16, 1.8, 0.02, *(2 * [_rng_t.uniform(0.5, 1.5, 16)]), 0.5, 43, 44)
_TILED_EXP = {}


@pytest.mark.parametrize("prec", [0, PRECS["fp32-12real"], PRECS["fp32-18real"]], ids=["fp64", "fp32-12", "fp32-18"])
def test_tiled_block_order_parity(prec):
    """Operators on a lattice whose z-planes are walked in tiles of workgroups
    equal the oracle's: every block is visited exactly once in that order."""
    import paper_1101_0423_amd as dwf
    print(f"[ops] tiled block order prec={prec}", flush=True)
    ops = [dwf.OP_DW, dwf.OP_HOP_EO, dwf.OP_HOP_OE, dwf.OP_M5, dwf.OP_C, dwf.OP_D]
    c = TILED.context()
    try:
        for op in ops:
            if op not in _TILED_EXP:
                _TILED_EXP[op] = oracle_op(TILED, op, TILED.b)
            got = c.apply(op, TILED.b, prec=prec)
            exp = _TILED_EXP[op]
            assert rel(got, exp) <= TOL[prec & 0xff], (OP_NAMES[op], rel(got, exp))
            assert max_rel(got, exp) <= TOL_EL[prec & 0xff], OP_NAMES[op]
    finally:
        c.close()


def test_non_su3_field_uses_18_real_links():
    """A U(3) field (every link times e^{i phi}): 12-real storage would rebuild a
    different third row, so the library refuses it (12-real links, FP16
    storage), its FP32 default uses 18-real links and still meets the FP32
    bar, and a solve with the default parameters meets the solve bar."""
    import paper_1101_0423_amd as dwf
    P = PROBS["ragged"]
    z = (P.U[..., 0] + 1j * P.U[..., 1]) * np.exp(0.3j)
    U3 = np.stack([z.real, z.imag], axis=-1)
    assert dwf.gauge_su3_deviation(U3, P.dims) > dwf.SU3_TOL
    c = dwf.Context(U3, *P.args, antiperiodic_t=True)
    try:
        for prec in (PRECS["fp32-12real"], PRECS["fp16"]):
            with pytest.raises(dwf.DwfError) as ei:
                c.apply(dwf.OP_C, P.b, prec=prec)
            assert ei.value.code == dwf.DWF_EINVAL
        for kw in (dict(inner_prec=1, link_compress=1), dict(inner_prec=2)):
            with pytest.raises(dwf.DwfError) as ei:
                c.solve(P.b, **kw)
            assert ei.value.code == dwf.DWF_EINVAL
        a = (U3, P.dims, P.ns, P.m0, P.mq, P.sigma, P.omega)
        exp = oracle.schur_c(*a, on_parity(P.b, P.dims, 1), bct=P.bct)
        auto = c.apply(dwf.OP_C, P.b, prec=1)
        assert np.array_equal(auto, c.apply(dwf.OP_C, P.b, prec=PRECS["fp32-18real"]))
        assert rel(auto, exp) <= TOL[1], rel(auto, exp)
        x, st, rc = c.solve(P.b)
        assert rc == dwf.DWF_OK, st
        assert oracle.true_residual(*a, P.b, x, bct=P.bct) <= 1e-10
    finally:
        c.close()
