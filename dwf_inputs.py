"""Seeded synthetic inputs for the domain-wall fermion solver.

This module is shared by the tests, the oracle checks and the benchmark.  It
only draws random numbers and lays them out in the canonical host layouts; it
contains none of the solver's arithmetic.

Host layouts (the boundary of the library):

* gauge field: float64 array ``[Lt][Lz][Ly][Lx][mu][a][b][re,im]`` where
  ``U_mu(x)`` is the SU(3) link from ``x`` to ``x + mu^`` and ``mu = 0..3`` is
  x, y, z, t;
* 5D spinor: float64 array ``[Lt][Lz][Ly][Lx][s][24]`` with the 24 reals of a
  site ordered ``c = 2*(3*spin + colour) + reim`` (spin slowest), i.e. the
  paper's host index of Eq. (12): ``c + 24 s + 24 Ns x + ...``.

Gauge links follow the recipe of the synthetic workloads: complex Gaussian
``G``, Hermitian traceless ``H = (G + G^dag)/2 - tr(H)/3``, ``U = exp(i eps H)``
by eigen-decomposition, then re-unitarised (Gram-Schmidt on rows 0 and 1,
row 2 = conj(row0 x row1)) so that every link is SU(3) to rounding.
"""
from __future__ import annotations

import numpy as np

SEED_GAUGE = 1000
SEED_RHS = 2000
SEED_STREAM = 3000


def _rng(seed):
    return np.random.default_rng(seed)


def _reunitarise(u):
    """Gram-Schmidt rows 0,1 of a batch of 3x3 complex matrices; row 2 = conj(row0 x row1)."""
    r0 = u[..., 0, :]
    r0 = r0 / np.linalg.norm(r0, axis=-1, keepdims=True)
    r1 = u[..., 1, :]
    r1 = r1 - np.sum(np.conj(r0) * r1, axis=-1, keepdims=True) * r0
    r1 = r1 / np.linalg.norm(r1, axis=-1, keepdims=True)
    r2 = np.conj(np.cross(r0, r1))
    return np.stack([r0, r1, r2], axis=-2)


def random_su3(n, eps, rng):
    """n SU(3) matrices U = exp(i eps H), H traceless Hermitian with Gaussian entries."""
    g = rng.standard_normal((n, 3, 3)) + 1j * rng.standard_normal((n, 3, 3))
    h = 0.5 * (g + np.conj(np.swapaxes(g, -1, -2)))
    tr = np.trace(h, axis1=-2, axis2=-1).real / 3.0
    h = h - tr[:, None, None] * np.eye(3)[None]
    lam, v = np.linalg.eigh(h)
    u = np.einsum("nab,nb,ncb->nac", v, np.exp(1j * eps * lam), np.conj(v))
    return _reunitarise(u)


def complex_to_host(z):
    """complex128 [..., k] -> float64 [..., 2k] with (re, im) interleaved."""
    out = np.empty(z.shape[:-1] + (2 * z.shape[-1],), dtype=np.float64)
    out[..., 0::2] = z.real
    out[..., 1::2] = z.imag
    return out


def host_to_complex(a):
    a = np.asarray(a, dtype=np.float64)
    return a[..., 0::2] + 1j * a[..., 1::2]


def gauge_field(dims, eps, seed=SEED_GAUGE):
    """Seeded SU(3) gauge field, host layout [Lt][Lz][Ly][Lx][4][3][3][2] (float64)."""
    lx, ly, lz, lt = dims
    rng = _rng(seed)
    n = lx * ly * lz * lt * 4
    u = random_su3(n, eps, rng).reshape(lt, lz, ly, lx, 4, 3, 3)
    out = np.empty(u.shape + (2,), dtype=np.float64)
    out[..., 0] = u.real
    out[..., 1] = u.imag
    return out


def unit_gauge(dims):
    lx, ly, lz, lt = dims
    out = np.zeros((lt, lz, ly, lx, 4, 3, 3, 2), dtype=np.float64)
    for a in range(3):
        out[..., a, a, 0] = 1.0
    return out


def gauge_transform(dims, eps, seed):
    """Seeded SU(3) matrix per 4D site, complex128 [Lt][Lz][Ly][Lx][3][3]."""
    lx, ly, lz, lt = dims
    rng = _rng(seed)
    return random_su3(lx * ly * lz * lt, eps, rng).reshape(lt, lz, ly, lx, 3, 3)


def gaussian_spinor(dims, ns, seed=SEED_RHS, nrhs=None):
    """Complex Gaussian 5D spinor(s): re and im independent N(0,1).

    Returns float64 [Lt][Lz][Ly][Lx][Ns][24], or [nrhs][...] when nrhs is given.
    """
    lx, ly, lz, lt = dims
    rng = _rng(seed)
    shape = (lt, lz, ly, lx, ns, 24)
    if nrhs is not None:
        shape = (nrhs,) + shape
    return rng.standard_normal(shape)


def point_sources(dims, ns, seed=SEED_RHS):
    """12 point sources at one seeded 5D site, one per (spin, colour) component.

    Returns (float64 [12][Lt][Lz][Ly][Lx][Ns][24], (x, y, z, t, s)).
    """
    lx, ly, lz, lt = dims
    rng = _rng(seed)
    x, y, z, t = (int(rng.integers(0, n)) for n in (lx, ly, lz, lt))
    s = int(rng.integers(0, ns))
    out = np.zeros((12, lt, lz, ly, lx, ns, 24), dtype=np.float64)
    for k in range(12):
        out[k, t, z, y, x, s, 2 * k] = 1.0
    return out, (x, y, z, t, s)


def point_source(dims, ns, k, seed=SEED_RHS):
    """Source k (spin-colour component k) of point_sources, built alone."""
    lx, ly, lz, lt = dims
    rng = _rng(seed)
    x, y, z, t = (int(rng.integers(0, n)) for n in (lx, ly, lz, lt))
    s = int(rng.integers(0, ns))
    out = np.zeros((lt, lz, ly, lx, ns, 24), dtype=np.float64)
    out[t, z, y, x, s, 2 * k] = 1.0
    return out


def uniform_weights(ns, lo, hi, seed):
    """Per-slice weights drawn uniformly from [lo, hi]."""
    return _rng(seed).uniform(lo, hi, size=ns)


# ---------------------------------------------------------------------------
# The workloads (operator parameters and seeds), as plain data.
# ---------------------------------------------------------------------------

def workload(name):
    """Operator parameters for a named workload.

    Returns a dict with dims (Lx, Ly, Lz, Lt), Ns, m0, mq, sigma, omega, eps.
    """
    if name == "shamir_4x4x4x4_ns8":
        ns = 8
        return dict(dims=(4, 4, 4, 4), ns=ns, m0=1.8, mq=0.02,
                    sigma=np.zeros(ns), omega=np.ones(ns), eps=0.3,
                    seed_gauge=SEED_GAUGE + 0, seed_rhs=SEED_RHS + 0)
    if name in ("odwf_16x16x16x32_ns16", "odwf_16x16x16x32_ns16_fp16"):
        ns = 16
        w = uniform_weights(ns, 0.5, 1.5, seed=SEED_GAUGE + 101)
        return dict(dims=(16, 16, 16, 32), ns=ns, m0=1.8, mq=0.01,
                    sigma=w.copy(), omega=w.copy(), eps=0.5,
                    seed_gauge=SEED_GAUGE + 1, seed_rhs=SEED_RHS + 1)
    if name == "odwf_8x8x8x16_ns16_12rhs":
        # a lattice small enough that one solve leaves most of the GPU idle
        ns = 16
        w = uniform_weights(ns, 0.5, 1.5, seed=SEED_GAUGE + 105)
        return dict(dims=(8, 8, 8, 16), ns=ns, m0=1.8, mq=0.01,
                    sigma=w.copy(), omega=w.copy(), eps=0.5,
                    seed_gauge=SEED_GAUGE + 5, seed_rhs=SEED_RHS + 5)
    if name == "shamir_24x24x24x48_ns16_12pt":
        ns = 16
        return dict(dims=(24, 24, 24, 48), ns=ns, m0=1.8, mq=0.005,
                    sigma=np.zeros(ns), omega=np.ones(ns), eps=0.5,
                    seed_gauge=SEED_GAUGE + 3, seed_rhs=SEED_RHS + 3)
    raise KeyError(name)


# ---------------------------------------------------------------------------
# The served workload: a Poisson stream of independent solves on four
# resident gauge fields.
# ---------------------------------------------------------------------------

SERVE_FIELDS = (((8, 8, 8, 16), SEED_GAUGE + 41), ((12, 12, 12, 24), SEED_GAUGE + 42),
                ((16, 16, 16, 32), SEED_GAUGE + 43), ((16, 16, 16, 32), SEED_GAUGE + 44))
SERVE_NS = (8, 16, 32)
SERVE_MQ = (0.01, 0.03, 0.1)
SERVE_RHS_PER_OPERATOR = 2


def serve_operator(field, ns):
    """Operator of one (field, Ns) pair of the served workload: m0 = 1.8,
    sigma = omega ~ U[0.5, 1.5] (seeded by Ns), links with eps = 0.5."""
    dims, seed = SERVE_FIELDS[field]
    w = uniform_weights(ns, 0.5, 1.5, seed=SEED_GAUGE + 200 + ns)
    return dict(dims=dims, ns=ns, m0=1.8, sigma=w.copy(), omega=w.copy(), eps=0.5, seed_gauge=seed)


def serve_rhs_seed(field, ns, k):
    return SEED_RHS + 400 + 100 * field + ns + 1000 * k


def serve_stream(n, seed=SEED_STREAM):
    """n requests: field, Ns and mq uniform over their sets, one of
    SERVE_RHS_PER_OPERATOR right-hand sides, and the gap to the previous
    arrival as a unit-mean exponential (scaled by 1/rate by the caller)."""
    rng = _rng(seed)
    out = []
    for _ in range(n):
        out.append(dict(field=int(rng.integers(0, len(SERVE_FIELDS))),
                        ns=SERVE_NS[int(rng.integers(0, len(SERVE_NS)))],
                        mq=SERVE_MQ[int(rng.integers(0, len(SERVE_MQ)))],
                        rhs=int(rng.integers(0, SERVE_RHS_PER_OPERATOR)),
                        gap=float(rng.exponential(1.0))))
    return out
