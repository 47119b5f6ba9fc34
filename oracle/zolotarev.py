"""Optimal fifth-dimension weights of optimal domain-wall fermions (the
omega_s of Sec. 2.1, fixed there for optimal chiral symmetry) -- the oracle's
version, computed from the minimax definition by a Remez exchange.

TEST INFRASTRUCTURE ONLY (tests and the benchmark's CPU leg use it; the HIP
library does not).

With sigma = omega the 4D operator obtained from the 5D one through its walls
depends on the weights only through the transfer product
    Pi(lam) = prod_s (1 - omega_s lam) / (1 + omega_s lam),   lam in spec(H),
H = gamma_5 D_w (the oracle's pins check S(0)^-1 = (1 + V)/(1 - V) with
V = gamma_5 (1 - Pi(H)) / (1 + Pi(H))), and it is chirally exact where Pi = 0.
Optimal weights minimise max |Pi| over the interval [lam_min, lam_max] that
holds |spec(H)|.  With p_s = 1 / omega_s and t = ln(lam),
(1 - omega_s lam) / (1 + omega_s lam) = -tanh((t - ln p_s) / 2), so the task is
the minimax of |prod_s tanh((t - q_s) / 2)| over t in [ln lam_min, ln lam_max]
with free zeros q_s = ln p_s.  Its solution equioscillates: |E| reaches its
maximum at both ends and once between consecutive zeros, N_s + 1 points with
alternating signs.  The exchange below finds that point: it locates the
extrema for the current zeros and moves the zeros by Newton's method so that
the logarithms of the extremal magnitudes become equal.
"""
import numpy as np


def _logabs_e(t, q):
    return np.sum(np.log(np.abs(np.tanh((np.asarray(t)[..., None] - q) / 2.0))), axis=-1)


def _extrema(q, a, b, grid=257):
    """Interior maximum of |E| between each pair of consecutive zeros (by a
    grid and golden-section refinement), with the two ends."""
    pts = [a]
    for lo, hi in zip(q[:-1], q[1:]):
        ts = np.linspace(lo, hi, grid)[1:-1]
        k = int(np.argmax(_logabs_e(ts, q)))
        x0, x1 = ts[max(k - 1, 0)], ts[min(k + 1, len(ts) - 1)]
        g = (np.sqrt(5.0) - 1) / 2
        for _ in range(70):
            c, d = x1 - g * (x1 - x0), x0 + g * (x1 - x0)
            if _logabs_e(c, q) > _logabs_e(d, q):
                x1 = d
            else:
                x0 = c
        pts.append(0.5 * (x0 + x1))
    pts.append(b)
    return np.array(pts)


def optimal_zeros(ns, lam_min, lam_max, tol=1e-14, maxit=200):
    """The zeros p_s (descending) of the optimal transfer product on
    [lam_min, lam_max]; omega_s = 1 / p_s."""
    a, b = np.log(lam_min), np.log(lam_max)
    # start: zeros spread evenly in t (the minimax solution for ns = 1 is the midpoint)
    q = a + (b - a) * (np.arange(ns) + 0.5) / ns
    for _ in range(maxit):
        e = _extrema(q, a, b)
        f = _logabs_e(e, q)
        g = f[1:] - f[0]                       # all extremal magnitudes equal: g = 0
        if np.max(np.abs(g)) < tol:
            break
        # d log|tanh((e - q_j)/2)| / d q_j = -1 / sinh(e - q_j); the interior
        # extrema move with q but are stationary points, the ends are fixed
        J = -1.0 / np.sinh(e[:, None] - q[None, :])
        step = np.linalg.solve(J[1:] - J[0], -g)
        # keep the zeros ordered inside (a, b)
        lim = 0.45 * np.min(np.diff(np.concatenate([[a], q, [b]])))
        s = np.max(np.abs(step))
        if s > lim:
            step *= lim / s
        q = q + step
    return np.sort(np.exp(q))[::-1]


def optimal_omega(ns, lam_min, lam_max):
    """omega_s = 1 / p_s, largest first (omega_1 ~ 1 / lam_min falls to
    omega_Ns ~ 1 / lam_max; the 4D operator does not depend on the order)."""
    return np.sort(1.0 / optimal_zeros(ns, lam_min, lam_max))[::-1]


def transfer_product(omega, lam):
    lam = np.asarray(lam, dtype=float)
    out = np.ones_like(lam)
    for w in omega:
        out = out * (1 - w * lam) / (1 + w * lam)
    return out
