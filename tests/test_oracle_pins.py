"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against a fact that does not come from the
oracle's own formulas: a closed form, an algebraic identity between
independently computed pieces, a special case that reduces to a textbook
operator, or a brute-force dense solve by LAPACK.  A dropped term, a wrong
sign or index or a transposed operand anywhere in the oracle fails one of
them (see test_oracle_mutations.py, which plants such mistakes).
"""
import numpy as np
import pytest

import dwf_inputs as inp
import oracle

# ---------------------------------------------------------------------------
# helpers (test side: gamma_5 on a spinor, R5, inner products, gauge transform)
# ---------------------------------------------------------------------------


def cplx(a, ns):
    a = np.asarray(a)
    z = inp.host_to_complex(a)
    return z.reshape(a.shape[:-1] + (4, 3))


def real(z):
    return inp.complex_to_host(z.reshape(z.shape[:-2] + (12,)))


def vdot(a, b):
    za = inp.host_to_complex(a).ravel()
    zb = inp.host_to_complex(b).ravel()
    return np.vdot(za, zb)


def apply_spin(mat, a, ns):
    z = cplx(a, ns)
    return real(np.einsum("ij,...ja->...ia", mat, z))


def g5(a, ns):
    return apply_spin(oracle.gamma(4), a, ns)


def r5(a):
    return np.ascontiguousarray(a[..., ::-1, :])


def rnd(dims, ns, seed):
    return inp.gaussian_spinor(dims, ns, seed=seed)


def parity_mask(dims):
    lx, ly, lz, lt = dims
    t, z, y, x = np.meshgrid(range(lt), range(lz), range(ly), range(lx), indexing="ij")
    return (x + y + z + t) % 2


def on_parity(a, dims, p):
    m = (parity_mask(dims) == p)[..., None, None]
    return np.where(m, a, 0.0)


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


# ---------------------------------------------------------------------------
# gamma matrices
# ---------------------------------------------------------------------------


def test_gamma_clifford_and_chiral_basis():
    g = [oracle.gamma(m) for m in range(4)]
    for i in range(4):
        assert np.allclose(g[i], g[i].conj().T, atol=0)
        for j in range(4):
            assert np.allclose(g[i] @ g[j] + g[j] @ g[i], 2 * (i == j) * np.eye(4), atol=0)
    g5m = oracle.gamma(4)
    assert np.allclose(g5m, g[0] @ g[1] @ g[2] @ g[3], atol=0)
    # chiral basis: gamma_5 diagonal, upper two spins are the + chirality
    assert np.allclose(g5m, np.diag([1, 1, -1, -1]), atol=0)
    # the basis of the readings: gamma_k = [[0, -i sigma_k], [i sigma_k, 0]], gamma_4 = [[0,1],[1,0]]
    sig = [np.array([[0, 1], [1, 0]]), np.array([[0, -1j], [1j, 0]]), np.array([[1, 0], [0, -1]])]
    z = np.zeros((2, 2))
    for k in range(3):
        assert np.allclose(g[k], np.block([[z, -1j * sig[k]], [1j * sig[k], z]]), atol=0)
    assert np.allclose(g[3], np.block([[z, np.eye(2)], [np.eye(2), z]]), atol=0)


# ---------------------------------------------------------------------------
# Wilson-Dirac operator, Eq. (2)
# ---------------------------------------------------------------------------

DIMS_A = (4, 2, 6, 4)     # unequal extents catch a swapped axis order


@pytest.mark.parametrize("bct", [1.0, -1.0])
def test_dw_gamma5_hermiticity(bct):
    dims, ns, m0 = DIMS_A, 2, 1.3
    U = inp.gauge_field(dims, 0.5, seed=11)
    phi, psi = rnd(dims, ns, 1), rnd(dims, ns, 2)
    lhs = vdot(phi, g5(oracle.dw(U, dims, ns, m0, g5(psi, ns), bct=bct), ns))
    rhs = vdot(oracle.dw(U, dims, ns, m0, phi, bct=bct), psi)
    assert abs(lhs - rhs) <= 1e-12 * abs(rhs)


def test_dw_gauge_covariance():
    """D_w[U^g](g psi) = g D_w[U] psi with U^g_mu(x) = g(x) U_mu(x) g(x+mu)^dag."""
    dims, ns, m0 = DIMS_A, 2, 1.1
    lx, ly, lz, lt = dims
    U = inp.gauge_field(dims, 0.5, seed=12)
    g = inp.gauge_transform(dims, 0.7, seed=13)
    Uc = U[..., 0] + 1j * U[..., 1]
    Ug = np.empty_like(Uc)
    for mu in range(4):
        axis = 3 - mu     # array axes are [t][z][y][x]
        gshift = np.roll(g, -1, axis=axis)      # g(x + mu)
        Ug[..., mu, :, :] = g @ Uc[..., mu, :, :] @ np.conj(np.swapaxes(gshift, -1, -2))
    Ugr = np.stack([Ug.real, Ug.imag], axis=-1)
    psi = rnd(dims, ns, 3)
    gpsi = real(np.einsum("tzyxab,tzyxsib->tzyxsia", g, cplx(psi, ns)))
    lhs = oracle.dw(Ugr, dims, ns, m0, gpsi)
    rhs = real(np.einsum("tzyxab,tzyxsib->tzyxsia", g, cplx(oracle.dw(U, dims, ns, m0, psi), ns)))
    assert rel(lhs, rhs) < 1e-13


@pytest.mark.parametrize("bct", [1.0, -1.0])
def test_dw_free_field_momentum_space(bct):
    """With U = 1 a plane wave e^{ipx} chi maps to
    [(4 - m0 - sum cos p) + i sum gamma_mu sin p_mu] e^{ipx} chi;
    the eigenvalues are W(p) +- i sqrt(sum sin^2 p), each six-fold."""
    dims, ns, m0 = (4, 6, 2, 8), 1, 1.8
    lx, ly, lz, lt = dims
    U = inp.unit_gauge(dims)
    t, z, y, x = np.meshgrid(range(lt), range(lz), range(ly), range(lx), indexing="ij")
    g = [oracle.gamma(m) for m in range(4)]
    shift = 0.5 if bct < 0 else 0.0
    rng = np.random.default_rng(5)
    for _ in range(6):
        n = [int(rng.integers(0, L)) for L in dims]
        p = [2 * np.pi * n[0] / lx, 2 * np.pi * n[1] / ly, 2 * np.pi * n[2] / lz,
             2 * np.pi * (n[3] + shift) / lt]
        phase = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
        W = 4 - m0 - sum(np.cos(pm) for pm in p)
        Mexp = W * np.eye(4) + 1j * sum(g[m] * np.sin(p[m]) for m in range(4))
        M = np.zeros((12, 12), complex)
        for k in range(12):
            chi = np.zeros((4, 3), complex)
            chi[k // 3, k % 3] = 1
            psi = phase[..., None, None, None] * chi   # [t,z,y,x,s=1,4,3]
            out = cplx(oracle.dw(U, dims, ns, m0, real(psi), bct=bct), ns)
            coeff = out / phase[..., None, None, None]
            assert np.allclose(coeff, coeff[0, 0, 0, 0], atol=1e-13)   # stays a plane wave
            M[:, k] = coeff[0, 0, 0, 0, 0].reshape(12)
        assert np.allclose(M, np.kron(Mexp, np.eye(3)), atol=1e-13)
        ev = np.linalg.eigvals(M)
        s = np.sqrt(sum(np.sin(pm) ** 2 for pm in p))
        assert np.allclose(ev.real, W, atol=1e-12)
        assert np.allclose(np.sort(ev.imag), [-s] * 6 + [s] * 6, atol=1e-12)


def test_hop_blocks_are_the_parity_split_of_dw():
    dims, ns, m0 = DIMS_A, 3, 1.4
    U = inp.gauge_field(dims, 0.5, seed=14)
    psi = rnd(dims, ns, 4)
    heo, hoe = oracle.hop(U, dims, ns, 0, psi), oracle.hop(U, dims, ns, 1, psi)
    assert rel(heo + hoe, oracle.dw(U, dims, ns, m0, psi) - (4 - m0) * psi) < 1e-14
    assert np.all(on_parity(heo, dims, 1) == 0) and np.all(on_parity(hoe, dims, 0) == 0)
    # D^EO reads only odd sites, D^OE only even sites
    assert np.array_equal(oracle.hop(U, dims, ns, 0, on_parity(psi, dims, 1)), heo)
    assert np.array_equal(oracle.hop(U, dims, ns, 1, on_parity(psi, dims, 0)), hoe)


# ---------------------------------------------------------------------------
# fifth dimension, Eqs. (3)-(4), (7)-(9)
# ---------------------------------------------------------------------------


@pytest.mark.parametrize("ns", [1, 2, 5, 8])
def test_det_one_plus_cl(ns):
    """det(1 + c L_+) = 1 + (-1)^Ns kappa prod(c): fixes the corner's place, sign and value."""
    m0, mq = 1.6, 0.37
    kappa = mq / (2 * m0)
    c = np.random.default_rng(ns).uniform(0.3, 1.7, ns)
    lp, lm = oracle.lmat(ns, m0, mq)
    for lmat in (lp, lm):
        d = np.linalg.det(np.eye(ns) + np.diag(c) @ lmat)
        assert abs(d - (1 + (-1) ** ns * kappa * np.prod(c))) < 1e-13


def test_L_chirality_and_direction():
    """L = P_+ L_+ + P_- L_-: the + chirality (spins 0,1) moves s -> s+1 and picks up
    -kappa when wrapping from Ns-1 to 0; the - chirality moves s -> s-1."""
    dims, ns, m0, mq = (2, 2, 2, 2), 4, 1.5, 0.3
    kappa = mq / (2 * m0)
    for spin, sgn in ((0, +1), (1, +1), (2, -1), (3, -1)):
        for s in range(ns):
            psi = np.zeros((2, 2, 2, 2, ns, 24))
            psi[1, 0, 1, 0, s, 2 * (3 * spin + 1) + 1] = 1.0     # imaginary part, colour 1
            out = oracle.L(dims, ns, m0, mq, psi)
            expect = np.zeros_like(psi)
            tgt = (s + sgn) % ns
            wraps = (sgn > 0 and s == ns - 1) or (sgn < 0 and s == 0)
            expect[1, 0, 1, 0, tgt, 2 * (3 * spin + 1) + 1] = -kappa if wraps else 1.0
            assert np.array_equal(out, expect), (spin, s)


def weights(kind, ns, seed=7):
    rng = np.random.default_rng(seed)
    if kind == "shamir":
        return np.zeros(ns), np.ones(ns)
    if kind == "borici":
        return np.ones(ns), np.ones(ns)
    if kind == "odwf":
        w = rng.uniform(0.5, 1.5, ns)
        return w.copy(), w.copy()
    return rng.uniform(0.2, 1.4, ns), rng.uniform(0.5, 1.5, ns)   # general sigma != omega


@pytest.mark.parametrize("kind", ["shamir", "borici", "odwf", "general"])
@pytest.mark.parametrize("ns", [1, 4, 8, 16])
def test_m5_two_forms_and_s1(kind, ns):
    m0, mq = 1.8, 0.05
    sigma, omega = weights(kind, ns)
    a_p, a_m = oracle.m5(ns, m0, mq, sigma, omega, form=1)
    b_p, b_m = oracle.m5(ns, m0, mq, sigma, omega, form=2)
    assert np.max(abs(a_p - b_p)) < 1e-13 * np.max(abs(b_p))
    assert np.max(abs(a_m - b_m)) < 1e-13 * np.max(abs(b_m))
    # S1 = sqrt(w)^-1 Y X^-1 equals M5 sqrt(w)^-1 (Eq. (9)), with LAPACK's inverse
    Xp, Xm, Yp, Ym = oracle.xy(ns, m0, mq, sigma, omega)
    sw = np.diag(np.sqrt(omega))
    for X, Y, M in ((Xp, Yp, b_p), (Xm, Ym, b_m)):
        s1 = np.linalg.inv(sw) @ Y @ np.linalg.inv(X)
        assert np.max(abs(s1 - M @ np.linalg.inv(sw))) < 1e-13 * np.max(abs(s1))


def test_ns1_reduces_to_wilson():
    """Ns = 1: L = -kappa, so D = (omega - sigma kappa) D_w + (1 + kappa)."""
    dims, m0, mq = DIMS_A, 1.7, 0.4
    kappa = mq / (2 * m0)
    U = inp.gauge_field(dims, 0.5, seed=15)
    psi = rnd(dims, 1, 5)
    sigma, omega = np.array([0.8]), np.array([1.3])
    d = oracle.d5(U, dims, 1, m0, mq, sigma, omega, psi)
    expect = (omega[0] - sigma[0] * kappa) * oracle.dw(U, dims, 1, m0, psi) + (1 + kappa) * psi
    assert rel(d, expect) < 1e-14


@pytest.mark.parametrize("kind", ["shamir", "symmetric"])
def test_shamir_g5r5_hermiticity(kind):
    """sigma = 0 with reflection-symmetric omega: D^dag = g5 R5 D g5 R5."""
    dims, ns, m0, mq = DIMS_A, 6, 1.8, 0.1
    U = inp.gauge_field(dims, 0.5, seed=16)
    if kind == "shamir":
        sigma, omega = np.zeros(ns), np.ones(ns)
    else:
        w = np.random.default_rng(3).uniform(0.5, 1.5, ns)
        sigma, omega = np.zeros(ns), 0.5 * (w + w[::-1])
    phi, psi = rnd(dims, ns, 6), rnd(dims, ns, 7)
    t = r5(g5(psi, ns))
    lhs = vdot(phi, r5(g5(oracle.d5(U, dims, ns, m0, mq, sigma, omega, t), ns)))
    rhs = vdot(oracle.d5(U, dims, ns, m0, mq, sigma, omega, phi), psi)
    assert abs(lhs - rhs) < 1e-12 * abs(rhs)


@pytest.mark.parametrize("kind", ["shamir", "general"])
def test_d5dag_and_cdag_are_adjoints(kind):
    dims, ns, m0, mq = DIMS_A, 4, 1.8, 0.07
    U = inp.gauge_field(dims, 0.5, seed=17)
    sigma, omega = weights(kind, ns)
    phi, psi = rnd(dims, ns, 8), rnd(dims, ns, 9)
    a = vdot(phi, oracle.d5(U, dims, ns, m0, mq, sigma, omega, psi))
    b = vdot(oracle.d5dag(U, dims, ns, m0, mq, sigma, omega, phi), psi)
    assert abs(a - b) < 1e-12 * abs(a)
    phio, psio = on_parity(phi, dims, 1), on_parity(psi, dims, 1)
    a = vdot(phio, oracle.schur_c(U, dims, ns, m0, mq, sigma, omega, psio))
    b = vdot(oracle.schur_cdag(U, dims, ns, m0, mq, sigma, omega, phio), psio)
    assert abs(a - b) < 1e-12 * abs(a)


# ---------------------------------------------------------------------------
# even-odd structure, Eqs. (6), (7), (10), (11)
# ---------------------------------------------------------------------------


@pytest.mark.parametrize("kind", ["shamir", "odwf", "general"])
def test_eo_blocks_x_and_dy(kind):
    """Eq. (6)-(7): on an even-supported vector, (D psi)_e = X psi_e and (D psi)_o = D^OE Y psi_e."""
    dims, ns, m0, mq = DIMS_A, 4, 1.8, 0.03
    U = inp.gauge_field(dims, 0.5, seed=18)
    sigma, omega = weights(kind, ns)
    Xp, Xm, Yp, Ym = oracle.xy(ns, m0, mq, sigma, omega)
    psi = on_parity(rnd(dims, ns, 10), dims, 0)
    d = oracle.d5(U, dims, ns, m0, mq, sigma, omega, psi)
    assert rel(on_parity(d, dims, 0), oracle.apply_s(dims, ns, Xp, Xm, psi)) < 1e-14
    expect_o = oracle.hop(U, dims, ns, 1, oracle.apply_s(dims, ns, Yp, Ym, psi))
    assert rel(on_parity(d, dims, 1), expect_o) < 1e-14


@pytest.mark.parametrize("kind", ["shamir", "odwf", "general"])
def test_eq10_factorisation(kind):
    """D = S1^-1 [[1, M5 D^EO], [M5 D^OE, 1]] S2^-1 with S1 = M5 sqrt(w)^-1, S2 = Y^-1 sqrt(w)."""
    dims, ns, m0, mq = DIMS_A, 5, 1.8, 0.05
    U = inp.gauge_field(dims, 0.5, seed=19)
    sigma, omega = weights(kind, ns)
    M5p, M5m = oracle.m5(ns, m0, mq, sigma, omega)
    Xp, Xm, Yp, Ym = oracle.xy(ns, m0, mq, sigma, omega)
    sw = np.diag(np.sqrt(omega))
    s1i = [np.linalg.inv(M @ np.linalg.inv(sw)) for M in (M5p, M5m)]
    s2i = [np.linalg.inv(np.linalg.inv(Y) @ sw) for Y in (Yp, Ym)]
    psi = rnd(dims, ns, 11)
    v = oracle.apply_s(dims, ns, *s2i, psi)
    mid = v + oracle.apply_s(dims, ns, M5p, M5m, oracle.hop(U, dims, ns, 0, v) + oracle.hop(U, dims, ns, 1, v))
    lhs = oracle.apply_s(dims, ns, *s1i, mid)
    assert rel(lhs, oracle.d5(U, dims, ns, m0, mq, sigma, omega, psi)) < 1e-13


def test_schur_complement_definition():
    """C = 1 - M5 D^OE M5 D^EO on odd sites, Eq. (11), from separately applied pieces."""
    dims, ns, m0, mq = DIMS_A, 4, 1.8, 0.05
    U = inp.gauge_field(dims, 0.5, seed=20)
    sigma, omega = weights("general", ns)
    M5p, M5m = oracle.m5(ns, m0, mq, sigma, omega, form=1)
    psi = on_parity(rnd(dims, ns, 12), dims, 1)
    t = oracle.apply_s(dims, ns, M5p, M5m, oracle.hop(U, dims, ns, 0, psi))
    t = oracle.apply_s(dims, ns, M5p, M5m, oracle.hop(U, dims, ns, 1, t))
    assert rel(oracle.schur_c(U, dims, ns, m0, mq, sigma, omega, psi), psi - t) < 1e-14


# ---------------------------------------------------------------------------
# the true residual, the initial-guess path of the solve, truncated CG
# ---------------------------------------------------------------------------


def _dense_problem(kind, seed=31):
    dims, ns, m0, mq = (2, 2, 2, 2), 4, 1.8, 0.05
    U = inp.gauge_field(dims, 0.3, seed=seed)
    sigma, omega = weights(kind, ns)
    a = (U, dims, ns, m0, mq, sigma, omega)
    shape = (2, 2, 2, 2, ns, 24)
    D = dense_matrix(lambda v: oracle.d5(*a, v), shape)
    b = rnd(dims, ns, seed + 1)
    xd = np.linalg.solve(D, inp.host_to_complex(b).ravel())
    xs = inp.complex_to_host(xd.reshape(shape[:-1] + (12,)))
    return a, shape, b, xs


@pytest.mark.parametrize("kind", ["shamir", "general"])
def test_truncated_cg_iterates_minimise_the_error(kind):
    """After k iterations from zero, CG on C C^dag w = b'' tracking y = C^dag w
    (Craig's method) holds the y of the Krylov space
    span{C^dag (C C^dag)^j b'', j < k} closest to y* = C^-1 b'': checked by
    projecting y* (from a dense LAPACK solve) onto that space.  The oracle's
    solve capped at k iterations is then the reconstruction of that y, which is
    compared through its Schur part y_o = (S2^-1 x)_o."""
    a, shape, b, xs = _dense_problem(kind, seed=43)
    U, dims, ns = a[0], a[1], a[2]
    Xp, Xm, Yp, Ym = oracle.xy(*a[2:])
    sw = np.diag(np.sqrt(a[6]))
    s2i = [np.linalg.inv(sw) @ Y for Y in (Yp, Ym)]          # S2^-1 = sqrt(w)^-1 Y

    def schur_part(x):
        return inp.host_to_complex(on_parity(oracle.apply_s(dims, ns, *s2i, x), dims, 1)).ravel()

    C = dense_matrix(lambda v: oracle.schur_c(*a, on_parity(v, dims, 1)), shape)
    odd = np.repeat(parity_mask(dims).ravel() == 1, ns * 12)
    Co = C[np.ix_(odd, odd)]
    ystar = schur_part(xs)[odd]
    bpp = Co @ ystar                                        # b'' = C y*
    kry, v = [], bpp.copy()
    for k in range(1, 6):
        kry.append(Co.conj().T @ v)
        v = Co @ kry[-1]
        Q, _ = np.linalg.qr(np.array(kry).T)
        yk = Q @ (Q.conj().T @ ystar)                       # orthogonal projection of y*
        x, info = oracle.solve(*a, b, tol=1e-300, maxiter=k)
        assert info["iters"] == k and not info["converged"]
        got = schur_part(x)[odd]
        assert np.linalg.norm(got - yk) <= 1e-11 * np.linalg.norm(yk), k


@pytest.mark.parametrize("kind", ["shamir", "general"])
def test_true_residual_closed_forms(kind):
    """|b - D x| / |b| on points where its value is known without the oracle's
    formula: x = 0 gives exactly 1; x = t x* with x* the LAPACK solution of
    D x = b gives |1 - t| (b - D t x* = (1 - t) b); x* itself gives rounding;
    b = 0 and x = 0 give 0."""
    a, shape, b, xs = _dense_problem(kind)
    assert oracle.true_residual(*a, b, np.zeros_like(b)) == 1.0
    for t in (0.5, 0.9, 1.25, -2.0):
        r = oracle.true_residual(*a, b, t * xs)
        assert abs(r - abs(1 - t)) <= 1e-13 * max(1.0, abs(1 - t)), (t, r)
    assert oracle.true_residual(*a, b, xs) < 1e-13
    assert oracle.true_residual(*a, np.zeros_like(b), np.zeros_like(b)) == 0.0
    # a residual confined to one site and slice: b = D x + e gives |e| / |b|
    e = np.zeros_like(b)
    e[1, 0, 1, 1, 2, 5] = 0.25
    r = oracle.true_residual(*a, b + e, xs)
    assert abs(r - 0.25 / np.linalg.norm(b + e)) <= 1e-12 * r


@pytest.mark.parametrize("kind", ["shamir", "general"])
def test_solve_initial_guess_path(kind):
    """The solve's initial guess enters through y_o = (S2^-1 x)_o: the LAPACK
    solution as the guess is already converged (no CG iteration, returned as
    is up to rounding), and a guess that differs from it only on even sites
    still needs none (the even half is rebuilt from y_o by Eq. (10))."""
    a, shape, b, xs = _dense_problem(kind, seed=37)
    x, info = oracle.solve(*a, b, tol=1e-10, x0=xs)
    assert info["converged"] and info["iters"] == 0, info
    assert rel(x, xs) < 1e-12
    # S2 y changes both parities; the guess is read only through (S2^-1 x0)_o,
    # so add to x* something whose image under S2^-1 vanishes on odd sites
    Xp, Xm, Yp, Ym = oracle.xy(a[2], a[3], a[4], a[5], a[6])
    sw = np.diag(np.sqrt(a[6]))
    s2 = [np.linalg.inv(Y) @ sw for Y in (Yp, Ym)]
    junk = on_parity(rnd(a[1], a[2], 41), a[1], 0)
    x0 = xs + oracle.apply_s(a[1], a[2], *s2, junk)
    x, info = oracle.solve(*a, b, tol=1e-10, x0=x0)
    assert info["converged"] and info["iters"] == 0, info
    assert rel(x, xs) < 1e-12
    # a guess away from x* takes iterations and still converges
    x, info = oracle.solve(*a, b, tol=1e-12, x0=0.5 * xs)
    assert info["converged"] and info["iters"] > 0
    assert rel(x, xs) < 1e-10


# ---------------------------------------------------------------------------
# brute force: dense LAPACK solve on a 2^4 x Ns = 4 lattice
# ---------------------------------------------------------------------------


def dense_matrix(fn, shape):
    n = int(np.prod(shape))
    cols = []
    for k in range(0, n, 2):       # unit real part of complex component k/2
        e = np.zeros(n)
        e[k] = 1.0
        cols.append(fn(e.reshape(shape)).ravel())
    Mr = np.array(cols).T          # rows: interleaved (re, im) of the image
    return Mr[0::2] + 1j * Mr[1::2]


@pytest.mark.parametrize("kind", ["shamir", "odwf", "general"])
def test_schur_solve_equals_dense_full_solve(kind):
    dims, ns, m0, mq = (2, 2, 2, 2), 4, 1.8, 0.02
    U = inp.gauge_field(dims, 0.3, seed=21)
    sigma, omega = weights(kind, ns)
    shape = (2, 2, 2, 2, ns, 24)
    D = dense_matrix(lambda v: oracle.d5(U, dims, ns, m0, mq, sigma, omega, v), shape)
    b = rnd(dims, ns, 13)
    xd = np.linalg.solve(D, inp.host_to_complex(b).ravel())
    x, info = oracle.solve(U, dims, ns, m0, mq, sigma, omega, b, tol=1e-14)
    assert info["converged"]
    assert np.linalg.norm(inp.host_to_complex(x).ravel() - xd) / np.linalg.norm(xd) < 1e-11
    assert oracle.true_residual(U, dims, ns, m0, mq, sigma, omega, b, x) < 1e-12
    # the dense matrix is the operator of Eq. (1) itself: (omega_s D_w + 1) delta + (sigma_s D_w - 1) L
    Dw = dense_matrix(lambda v: oracle.dw(U, dims, ns, m0, v), shape)
    Lm = dense_matrix(lambda v: oracle.L(dims, ns, m0, mq, v), shape)
    V5 = D.shape[0]
    Om = np.diag(np.tile(np.repeat(omega, 12), 16))
    Sg = np.diag(np.tile(np.repeat(sigma, 12), 16))
    eq1 = Dw @ Om + np.eye(V5) + (Dw @ Sg - np.eye(V5)) @ Lm
    assert np.max(abs(eq1 - D)) < 1e-13


def test_cg_matches_dense_solve_and_full_cgne():
    """Config-0 shaped operator on 4^4 x 8 (Shamir, eps = 0.3, mq = 0.02):
    the Schur-route CG and CG on the unpreconditioned operator reach the same x."""
    w = inp.workload("shamir_4x4x4x4_ns8")
    dims, ns = w["dims"], w["ns"]
    U = inp.gauge_field(dims, w["eps"], seed=w["seed_gauge"])
    b = rnd(dims, ns, w["seed_rhs"])
    args = (U, dims, ns, w["m0"], w["mq"], w["sigma"], w["omega"])
    x1, i1 = oracle.solve(*args, b, tol=1e-12)
    x2, i2 = oracle.cgne_full(*args, b, tol=1e-12)
    assert i1["converged"] and i2["converged"]
    assert i1["iters"] < i2["iters"]
    assert oracle.true_residual(*args, b, x1) < 1e-11
    assert rel(x1, x2) < 1e-9


@pytest.mark.parametrize("kind", ["shamir", "general"])
def test_ccdag_solve_equals_dense_solve(kind):
    """The force solve C C^dag w = b (odd sites) by Algorithm 1 equals a LAPACK
    solve of the dense C C^dag restricted to odd sites, which is Hermitian and
    positive definite; even sites of w are zero."""
    dims, ns, m0, mq = (2, 2, 2, 2), 4, 1.8, 0.1
    U = inp.gauge_field(dims, 0.3, seed=23)
    sigma, omega = weights(kind, ns)
    shape = (2, 2, 2, 2, ns, 24)
    a = (U, dims, ns, m0, mq, sigma, omega)
    A = dense_matrix(lambda v: oracle.schur_c(*a, oracle.schur_cdag(*a, v)), shape)
    par = parity_mask(dims).ravel()                       # per 4D site, [t][z][y][x] order
    odd = np.repeat(par == 1, ns * 12)                    # per complex component
    Ao = A[np.ix_(odd, odd)]
    assert np.max(abs(Ao - Ao.conj().T)) < 1e-12 * np.max(abs(Ao))
    assert np.min(np.linalg.eigvalsh(Ao)) > 0
    b = rnd(dims, ns, 29)
    wd = np.linalg.solve(Ao, inp.host_to_complex(b).ravel()[odd])
    w, info = oracle.solve_ccdag(*a, b, tol=1e-14)
    assert info["converged"]
    wc = inp.host_to_complex(w).ravel()
    assert np.all(wc[~odd] == 0)
    assert np.linalg.norm(wc[odd] - wd) / np.linalg.norm(wd) < 1e-11


# ---------------------------------------------------------------------------
# 4D propagator from the 5D solve (Sec. 2.2): S eta = R D^-1 W eta
# ---------------------------------------------------------------------------


def _chiral_proj():
    g5m = np.diag([1.0, 1.0, -1.0, -1.0]).astype(complex)      # the chiral basis (reading 1)
    return 0.5 * (np.eye(4) + g5m), 0.5 * (np.eye(4) - g5m), g5m


def _prop_dense(a, dims):
    """S as a dense 4D matrix (12 V4 x 12 V4 complex), column by column from
    oracle.propagator on unit sources."""
    import concurrent.futures
    lx, ly, lz, lt = dims
    n = lx * ly * lz * lt * 12
    src = np.zeros((n, lt, lz, ly, lx, 24))
    for k in range(n):
        src.reshape(n, -1)[k, 2 * k] = 1.0

    def run(k):  # the oracle's C code runs without the GIL: columns in parallel
        out, info = oracle.propagator(*a, src[k], tol=1e-14)
        assert info["converged"]
        return inp.host_to_complex(out).reshape(-1)

    with concurrent.futures.ThreadPoolExecutor(8) as ex:
        cols = list(ex.map(run, range(n)))
    return np.array(cols).T                                    # column k = S e_k


def _prop_numpy(a, dims):
    """The same matrix built independently: LAPACK inverse of the dense 5D
    operator (Eq. (1), pinned above), with R and W written out here."""
    U, _, ns, m0, mq, sigma, omega = a
    lx, ly, lz, lt = dims
    V = lx * ly * lz * lt
    shape = (lt, lz, ly, lx, ns, 24)
    D = dense_matrix(lambda v: oracle.d5(*a, v), shape)
    Dw = dense_matrix(lambda v: oracle.dw(U, dims, ns, m0, v), shape)
    Pp, Pm, _ = _chiral_proj()
    n4, n5 = 12 * V, 12 * V * ns
    C = np.zeros((n5, n4), complex)                            # c = P_+ eta on s = 1, P_- eta on s = Ns
    Rm = np.zeros((n4, n5), complex)                           # R psi = P_+ psi_Ns + P_- psi_1
    for x in range(V):
        for i in range(4):
            for j in range(4):
                for col in range(3):
                    r4 = 12 * x + 3 * i + col
                    c4 = 12 * x + 3 * j + col
                    C[12 * (x * ns + 0) + 3 * i + col, c4] += Pp[i, j]
                    C[12 * (x * ns + ns - 1) + 3 * i + col, c4] += Pm[i, j]
                    Rm[r4, 12 * (x * ns + ns - 1) + 3 * j + col] += Pp[i, j]
                    Rm[r4, 12 * (x * ns + 0) + 3 * j + col] += Pm[i, j]
    Sg = np.diag(np.tile(np.repeat(sigma, 12), V))
    W = C - Sg @ Dw @ C                                        # (1 - sigma_s D_w) on the two walls
    return Rm @ np.linalg.solve(D, W)


@pytest.mark.parametrize("kind", ["odwf", "general"])
def test_propagator_mass_enters_additively(kind):
    """S(mq)^-1 = S(0)^-1 + kappa (kappa = mq / (2 m0)): the corner of L, the
    only place mq enters (Eq. (4)), is kappa W R, so the Woodbury identity
    gives R D(mq)^-1 W = (1 + kappa S(0))^-1 S(0), and two masses differ by
    exactly the difference of their kappas.  Checked on dense matrices, and
    the oracle's S against the same matrix built from a LAPACK inverse of the
    dense 5D operator with R and W written out here."""
    dims, ns, m0 = (2, 2, 2, 2), 4, 1.8
    U = inp.gauge_field(dims, 0.3, seed=47)
    sigma, omega = weights(kind, ns)
    S = {mq: _prop_dense((U, dims, ns, m0, mq, sigma, omega), dims) for mq in (0.05, 0.3)}
    Si = {mq: np.linalg.inv(S[mq]) for mq in S}
    d = Si[0.3] - Si[0.05]
    dk = (0.3 - 0.05) / (2 * m0)
    assert np.max(abs(d - dk * np.eye(d.shape[0]))) < 1e-9 * np.max(abs(Si[0.05]))
    Sn = _prop_numpy((U, dims, ns, m0, 0.05, sigma, omega), dims)
    assert np.max(abs(S[0.05] - Sn)) < 1e-11 * np.max(abs(Sn))


def test_propagator_gamma5_hermitian_for_shamir():
    """With sigma = 0 and reflection-symmetric omega, D^dag = g5 R5 D g5 R5
    (pinned above) and R g5 R5 = g5 W^dag, so S^dag = g5 S g5."""
    dims, ns, m0, mq = (2, 2, 2, 2), 4, 1.8, 0.1
    U = inp.gauge_field(dims, 0.3, seed=53)
    w = np.random.default_rng(3).uniform(0.5, 1.5, ns)
    a = (U, dims, ns, m0, mq, np.zeros(ns), 0.5 * (w + w[::-1]))
    S = _prop_dense(a, dims)
    _, _, g5m = _chiral_proj()
    G5 = np.kron(np.eye(S.shape[0] // 12), np.kron(g5m, np.eye(3)))
    assert np.max(abs(S.conj().T - G5 @ S @ G5)) < 1e-11 * np.max(abs(S))


@pytest.mark.parametrize("kind", ["shamir", "odwf"])
def test_propagator_free_field_momentum_space(kind):
    """Unit links: a plane-wave source e^{ipx} chi gives e^{ipx} S(p) chi with
    S(p) = R D(p)^-1 W(p) built from the 4Ns x 4Ns momentum block
    D(p) = D_w(p)(omega + sigma L) + (1 - L), D_w(p) = (4 - m0 - sum cos p)
    + i sum gamma sin p (the closed form pinned for D_w above), written out
    here with the chiral gamma matrices."""
    dims, ns, m0, mq = (4, 2, 2, 6), 5, 1.7, 0.08
    lx, ly, lz, lt = dims
    sigma, omega = weights(kind, ns)
    U = inp.unit_gauge(dims)
    kappa = mq / (2 * m0)
    g = [oracle.gamma(m) for m in range(4)]
    Pp, Pm, _ = _chiral_proj()
    Lp = np.diag(np.ones(ns - 1), -1)
    Lp[0, ns - 1] = -kappa
    Lm = Lp.T
    t, z, y, x = np.meshgrid(range(lt), range(lz), range(ly), range(lx), indexing="ij")
    rng = np.random.default_rng(9)
    for n in [(1, 0, 1, 2), (0, 1, 0, 5), (3, 1, 1, 0)]:
        p = [2 * np.pi * n[k] / dims[k] for k in range(4)]
        Dwp = (4 - m0 - sum(np.cos(pm) for pm in p)) * np.eye(4) + 1j * sum(g[m] * np.sin(p[m]) for m in range(4))
        Lmat = np.kron(Lp, Pp) + np.kron(Lm, Pm)                # [s, spin] x [s', spin']
        Om, Sg = np.kron(np.diag(omega), np.eye(4)), np.kron(np.diag(sigma), np.eye(4))
        Dp = np.kron(np.eye(ns), Dwp) @ (Om + Sg @ Lmat) + np.eye(4 * ns) - Lmat
        Wp = np.zeros((4 * ns, 4), complex)
        Wp[0:4] = (np.eye(4) - sigma[0] * Dwp) @ Pp
        Wp[4 * (ns - 1):] = (np.eye(4) - sigma[ns - 1] * Dwp) @ Pm
        Rp = np.zeros((4, 4 * ns), complex)
        Rp[:, 4 * (ns - 1):] = Pp
        Rp[:, 0:4] += Pm
        Sp = Rp @ np.linalg.solve(Dp, Wp)
        chi = rng.normal(size=(4, 3)) + 1j * rng.normal(size=(4, 3))
        phase = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))[..., None, None]
        eta = inp.complex_to_host((phase * chi).reshape(lt, lz, ly, lx, 12))
        out, info = oracle.propagator(U, dims, ns, m0, mq, sigma, omega, eta, tol=1e-14)
        assert info["converged"]
        got = inp.host_to_complex(out).reshape(lt, lz, ly, lx, 4, 3)
        exp = phase * (Sp @ chi)
        assert np.max(abs(got - exp)) < 1e-11 * np.max(abs(exp)), n


# ---------------------------------------------------------------------------
# optimal domain-wall weights (Sec. 2.1): the transfer product and its minimax
# ---------------------------------------------------------------------------


def test_odwf_walls_see_the_transfer_product():
    """With sigma = omega the 4D propagator at mq = 0 satisfies
    S(0)^-1 = (1 + V)/(1 - V), V = g5 (1 - Pi(H))/(1 + Pi(H)),
    Pi(H) = prod_s (1 - omega_s H)/(1 + omega_s H), H = g5 D_w: the weights
    reach the 4D operator only through Pi on the spectrum of H (dense
    matrices; H diagonalised by LAPACK)."""
    dims, ns, m0 = (2, 2, 2, 2), 4, 1.8
    U = inp.gauge_field(dims, 0.3, seed=59)
    w = np.random.default_rng(1).uniform(0.5, 1.5, ns)
    S0 = _prop_dense((U, dims, ns, m0, 0.0, w, w), dims)
    Dw = dense_matrix(lambda v: oracle.dw(U, dims, 1, m0, v), (2, 2, 2, 2, 1, 24))
    n = Dw.shape[0]
    G5 = np.kron(np.eye(n // 12), np.kron(np.diag([1.0, 1.0, -1.0, -1.0]), np.eye(3)))
    lam, Q = np.linalg.eigh(G5 @ Dw)
    Pi = np.prod([(1 - o * lam) / (1 + o * lam) for o in w], axis=0)
    V = G5 @ (Q @ np.diag((1 - Pi) / (1 + Pi)) @ Q.conj().T)
    A = (np.eye(n) + V) @ np.linalg.inv(np.eye(n) - V)
    Si = np.linalg.inv(S0)
    assert np.max(abs(Si - A)) < 1e-10 * np.max(abs(A))


def _zol_extrema(omega, a, b, n=400001):
    """Signs and magnitudes of the local extrema of Pi on a dense log grid,
    with both ends."""
    from oracle import zolotarev
    t = np.exp(np.linspace(np.log(a), np.log(b), n))
    E = zolotarev.transfer_product(omega, t)
    idx = [0] + [i for i in range(1, n - 1) if abs(E[i]) >= abs(E[i - 1]) and abs(E[i]) >= abs(E[i + 1])
                 and abs(E[i]) > 0] + [n - 1]
    return E[idx], np.max(np.abs(E))


@pytest.mark.parametrize("ns", [1, 2, 5, 8, 16])
def test_optimal_weights_minimax(ns):
    """The oracle's optimal weights (a Remez exchange on the minimax of
    |Pi| over [a, b]) against what fixes them without the exchange: for Ns = 1
    the closed form omega = 1/sqrt(ab) (|Pi| equal at both ends); for every Ns
    the Chebyshev alternation that characterises the unique minimax solution
    (Ns + 1 extrema of equal size and alternating sign, found on a dense grid
    independent of the exchange's own search); the symmetry of the problem
    under lam -> ab / lam (the zeros map onto themselves); no nearby weights do
    better; and the classical closed form of Zolotarev's third problem,
    zeros b dn((2j - 1) K / (2 Ns), k), k = sqrt(1 - (a/b)^2), evaluated with
    scipy's elliptic functions."""
    import scipy.special as sps

    from oracle import zolotarev
    a, b = 0.04, 5.5
    w = zolotarev.optimal_omega(ns, a, b)
    if ns == 1:
        assert abs(w[0] - 1 / np.sqrt(a * b)) < 1e-13 * w[0]
    ext, emax = _zol_extrema(w, a, b)
    assert len(ext) == ns + 1
    assert np.all(np.sign(ext[1:]) == -np.sign(ext[:-1]))
    assert np.max(np.abs(np.abs(ext) - emax)) < 1e-8 * emax
    p = np.sort(1 / w)
    assert np.max(np.abs(np.sort(a * b / p) - p) / p) < 1e-12
    rng = np.random.default_rng(ns)
    for _ in range(5):
        wp = w * np.exp(1e-3 * rng.standard_normal(ns))
        assert _zol_extrema(wp, a, b)[1] > emax
    k = np.sqrt(1 - (a / b) ** 2)
    u = (2 * np.arange(1, ns + 1) - 1) * sps.ellipk(k * k) / (2 * ns)
    dn = sps.ellipj(u, k * k)[2]
    assert np.max(np.abs(np.sort(b * dn) - p) / p) < 1e-11
