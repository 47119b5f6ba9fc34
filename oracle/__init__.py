"""ctypes binding of the plain FP64 CPU oracle (``oracle/dwf_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only users.  The HIP library never imports it.

All arrays are numpy float64 in the canonical host layouts:
spinor ``[Lt][Lz][Ly][Lx][Ns][24]``, gauge ``[Lt][Lz][Ly][Lx][4][3][3][2]``,
s-space matrices ``[Ns][Ns]``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dwf_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# the pins' mutation test loads deliberately broken copies of the oracle
_LIB_OVERRIDE = os.environ.get("DWF_ORACLE_LIB")

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def build(force=False):
    """Compile the oracle with gcc (plain -O2, OpenMP, IEEE arithmetic)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                           "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if _LIB_OVERRIDE:
            L = ctypes.CDLL(_LIB_OVERRIDE)
        else:
            if not os.path.exists(_LIB):
                build()
            L = ctypes.CDLL(_LIB)
        L.orc_gamma.argtypes = [ctypes.c_int, _dp]
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_dw.argtypes = [_dp, _ip, ctypes.c_int, ctypes.c_double, ctypes.c_double, _dp, _dp]
        L.orc_hop.argtypes = [_dp, _ip, ctypes.c_int, ctypes.c_double, ctypes.c_int, _dp, _dp]
        L.orc_lmat.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, _dp, _dp]
        L.orc_xy.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, _dp, _dp, _dp, _dp, _dp, _dp]
        for f in (L.orc_m5_form1, L.orc_m5_form2):
            f.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, _dp, _dp, _dp, _dp]
            f.restype = ctypes.c_int
        L.orc_invert.argtypes = [ctypes.c_int, _dp, _dp]
        L.orc_invert.restype = ctypes.c_int
        L.orc_apply_s.argtypes = [_ip, ctypes.c_int, _dp, _dp, _dp, _dp]
        L.orc_L.argtypes = [_ip, ctypes.c_int, ctypes.c_double, ctypes.c_double, _dp, _dp]
        opargs = [_dp, _ip, ctypes.c_int, ctypes.c_double, ctypes.c_double, _dp, _dp,
                  ctypes.c_double, _dp, _dp]
        for f in (L.orc_d5, L.orc_d5dag, L.orc_schur_c, L.orc_schur_cdag):
            f.argtypes = opargs
        L.orc_solve.argtypes = opargs + [ctypes.c_double, ctypes.c_int, _ip, _dp]
        L.orc_solve.restype = ctypes.c_int
        L.orc_solve_ccdag.argtypes = opargs + [ctypes.c_double, ctypes.c_int, _ip, _dp]
        L.orc_solve_ccdag.restype = ctypes.c_int
        L.orc_cgne_full.argtypes = opargs + [ctypes.c_double, ctypes.c_int, _ip, _dp]
        L.orc_cgne_full.restype = ctypes.c_int
        L.orc_true_residual.argtypes = opargs
        L.orc_true_residual.restype = ctypes.c_double
        L.orc_propagator.argtypes = opargs + [ctypes.c_double, ctypes.c_int, _ip, _dp]
        L.orc_propagator.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _dims(dims):
    return (ctypes.c_int * 4)(*dims)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads():
    return lib().orc_num_threads()


def gamma(mu):
    """gamma_mu (mu = 0..3 for x, y, z, t) or gamma_5 (mu = 4): complex 4x4."""
    out = np.zeros(32)
    lib().orc_gamma(mu, _p(out))
    return out[0::2].reshape(4, 4) + 1j * out[1::2].reshape(4, 4)


def dw(U, dims, ns, m0, psi, bct=1.0):
    U, psi = _f64(U), _f64(psi)
    out = np.zeros_like(psi)
    lib().orc_dw(_p(U), _dims(dims), ns, m0, bct, _p(psi), _p(out))
    return out


def hop(U, dims, ns, out_parity, psi, bct=1.0):
    """out_parity 0: D_w^EO (odd -> even), 1: D_w^OE (even -> odd)."""
    U, psi = _f64(U), _f64(psi)
    out = np.zeros_like(psi)
    lib().orc_hop(_p(U), _dims(dims), ns, bct, out_parity, _p(psi), _p(out))
    return out


def lmat(ns, m0, mq):
    lp, lm = np.zeros((ns, ns)), np.zeros((ns, ns))
    lib().orc_lmat(ns, m0, mq, _p(lp), _p(lm))
    return lp, lm


def xy(ns, m0, mq, sigma, omega):
    mats = [np.zeros((ns, ns)) for _ in range(4)]
    lib().orc_xy(ns, m0, mq, _p(_f64(sigma)), _p(_f64(omega)), *[_p(m) for m in mats])
    return mats  # Xp, Xm, Yp, Ym


def m5(ns, m0, mq, sigma, omega, form=2):
    mp, mm = np.zeros((ns, ns)), np.zeros((ns, ns))
    f = lib().orc_m5_form1 if form == 1 else lib().orc_m5_form2
    rc = f(ns, m0, mq, _p(_f64(sigma)), _p(_f64(omega)), _p(mp), _p(mm))
    if rc:
        raise ValueError("singular fifth-dimension matrix")
    return mp, mm


def invert(a):
    a = _f64(a)
    out = np.zeros_like(a)
    if lib().orc_invert(a.shape[0], _p(a), _p(out)):
        raise ValueError("singular")
    return out


def apply_s(dims, ns, mp, mm, psi):
    psi = _f64(psi)
    out = np.zeros_like(psi)
    lib().orc_apply_s(_dims(dims), ns, _p(_f64(mp)), _p(_f64(mm)), _p(psi), _p(out))
    return out


def L(dims, ns, m0, mq, psi):
    psi = _f64(psi)
    out = np.zeros_like(psi)
    lib().orc_L(_dims(dims), ns, m0, mq, _p(psi), _p(out))
    return out


def _op(fn, U, dims, ns, m0, mq, sigma, omega, psi, bct):
    U, psi = _f64(U), _f64(psi)
    out = np.zeros_like(psi)
    fn(_p(U), _dims(dims), ns, m0, mq, _p(_f64(sigma)), _p(_f64(omega)), bct, _p(psi), _p(out))
    return out


def d5(U, dims, ns, m0, mq, sigma, omega, psi, bct=1.0):
    return _op(lib().orc_d5, U, dims, ns, m0, mq, sigma, omega, psi, bct)


def d5dag(U, dims, ns, m0, mq, sigma, omega, psi, bct=1.0):
    return _op(lib().orc_d5dag, U, dims, ns, m0, mq, sigma, omega, psi, bct)


def schur_c(U, dims, ns, m0, mq, sigma, omega, psi, bct=1.0):
    return _op(lib().orc_schur_c, U, dims, ns, m0, mq, sigma, omega, psi, bct)


def schur_cdag(U, dims, ns, m0, mq, sigma, omega, psi, bct=1.0):
    return _op(lib().orc_schur_cdag, U, dims, ns, m0, mq, sigma, omega, psi, bct)


def solve(U, dims, ns, m0, mq, sigma, omega, b, tol=1e-12, maxiter=100000, x0=None, bct=1.0):
    """Schur-route solve of D x = b.  Returns (x, info dict)."""
    U, b = _f64(U), _f64(b)
    x = np.zeros_like(b) if x0 is None else _f64(x0).copy()
    it = ctypes.c_int(0)
    res = ctypes.c_double(0)
    rc = lib().orc_solve(_p(U), _dims(dims), ns, m0, mq, _p(_f64(sigma)), _p(_f64(omega)), bct,
                         _p(b), _p(x), tol, maxiter, ctypes.byref(it), ctypes.byref(res))
    if rc < 0:
        raise ValueError("singular fifth-dimension matrix")
    return x, dict(converged=(rc == 0), iters=it.value, schur_res=res.value)


def solve_ccdag(U, dims, ns, m0, mq, sigma, omega, b, tol=1e-12, maxiter=100000, w0=None, bct=1.0):
    """C C^dag w = b on the odd sites by Algorithm 1 (even sites of b ignored,
    of w zero).  Returns (w, info dict)."""
    U, b = _f64(U), _f64(b)
    w = np.zeros_like(b) if w0 is None else _f64(w0).copy()
    it = ctypes.c_int(0)
    res = ctypes.c_double(0)
    rc = lib().orc_solve_ccdag(_p(U), _dims(dims), ns, m0, mq, _p(_f64(sigma)), _p(_f64(omega)), bct,
                               _p(b), _p(w), tol, maxiter, ctypes.byref(it), ctypes.byref(res))
    if rc < 0:
        raise ValueError("singular fifth-dimension matrix")
    return w, dict(converged=(rc == 0), iters=it.value, relres=res.value)


def cgne_full(U, dims, ns, m0, mq, sigma, omega, b, tol=1e-12, maxiter=100000, bct=1.0):
    U, b = _f64(U), _f64(b)
    x = np.zeros_like(b)
    it = ctypes.c_int(0)
    res = ctypes.c_double(0)
    rc = lib().orc_cgne_full(_p(U), _dims(dims), ns, m0, mq, _p(_f64(sigma)), _p(_f64(omega)), bct,
                             _p(b), _p(x), tol, maxiter, ctypes.byref(it), ctypes.byref(res))
    return x, dict(converged=(rc == 0), iters=it.value, relres=res.value)


def true_residual(U, dims, ns, m0, mq, sigma, omega, b, x, bct=1.0):
    U, b, x = _f64(U), _f64(b), _f64(x)
    return lib().orc_true_residual(_p(U), _dims(dims), ns, m0, mq, _p(_f64(sigma)), _p(_f64(omega)),
                                   bct, _p(b), _p(x))


def propagator(U, dims, ns, m0, mq, sigma, omega, eta, tol=1e-12, maxiter=100000, bct=1.0):
    """4D quark propagator S eta = R D^-1 W eta (see orc_propagator) for a 4D
    source eta [..][Lt][Lz][Ly][Lx][24] (one source, or several stacked in a
    leading axis).  Returns (S eta, info dict of the last solve)."""
    U, eta = _f64(U), _f64(eta)
    lx, ly, lz, lt = dims
    one = (lt, lz, ly, lx, 24)
    many = eta.reshape((-1,) + one)
    out = np.zeros_like(many)
    info = {}
    for k in range(many.shape[0]):
        it = ctypes.c_int(0)
        res = ctypes.c_double(0)
        src = np.ascontiguousarray(many[k])
        dst = np.zeros(one)
        rc = lib().orc_propagator(_p(U), _dims(dims), ns, m0, mq, _p(_f64(sigma)), _p(_f64(omega)), bct,
                                  _p(src), _p(dst), tol, maxiter, ctypes.byref(it), ctypes.byref(res))
        if rc < 0:
            raise ValueError("singular fifth-dimension matrix")
        out[k] = dst
        info = dict(converged=(rc == 0), iters=it.value, schur_res=res.value)
    return out.reshape(eta.shape), info
