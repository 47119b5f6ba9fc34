"""Shared test helpers: seeded problem set-up and error measures."""
import numpy as np

import dwf_inputs as inp


def rel(a, b):
    """norm-wise relative difference |a - b| / |b|."""
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def max_rel(a, b):
    """element-wise: max |a - b| / max |b|."""
    mb = np.max(np.abs(b))
    return np.max(np.abs(a - b)) / (mb if mb > 0 else 1.0)


def parity_mask(dims):
    lx, ly, lz, lt = dims
    t, z, y, x = np.meshgrid(range(lt), range(lz), range(ly), range(lx), indexing="ij")
    return (x + y + z + t) % 2


def on_parity(a, dims, p):
    m = (parity_mask(dims) == p)[..., None, None]
    return np.where(m, a, 0.0)


class Problem:
    """An operator (gauge field + fifth-dimension parameters) and a right-hand side."""

    def __init__(self, dims, ns, m0, mq, sigma, omega, eps, seed_gauge, seed_rhs, antiperiodic=False):
        self.dims, self.ns, self.m0, self.mq = tuple(dims), ns, m0, mq
        self.sigma, self.omega = np.asarray(sigma, float), np.asarray(omega, float)
        self.bct = -1.0 if antiperiodic else 1.0
        self.antiperiodic = antiperiodic
        self.U = inp.gauge_field(self.dims, eps, seed=seed_gauge)
        self.b = inp.gaussian_spinor(self.dims, ns, seed=seed_rhs)

    @classmethod
    def workload(cls, name):
        w = inp.workload(name)
        return cls(w["dims"], w["ns"], w["m0"], w["mq"], w["sigma"], w["omega"], w["eps"],
                   w["seed_gauge"], w["seed_rhs"])

    @property
    def args(self):
        return (self.dims, self.ns, self.m0, self.mq, self.sigma, self.omega)

    def oargs(self):
        return (self.U, self.dims, self.ns, self.m0, self.mq, self.sigma, self.omega)

    def context(self, **kw):
        import paper_1101_0423_amd as dwf
        return dwf.Context(self.U, *self.args, antiperiodic_t=self.antiperiodic, **kw)
