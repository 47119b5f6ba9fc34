"""The oracle's pins catch plausible mistakes (CPU).

Each case copies oracle/dwf_oracle.c, plants one mistake by replacing a
fragment of the source (a wrong sign, a missing dagger or corner, a swapped
index or vector), builds the copy, and runs the pin suite against it: at
least one pin must fail.  The committed oracle itself carries no hooks; the
copies live in a temporary directory.
"""
import concurrent.futures
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "dwf_oracle.c")

# (name, fragment, replacement)
MUTANTS = [
    ("hop projector sign (1 - gamma) <-> (1 + gamma)",
     "acc += G[mu][i][j] * (vb[j][a] - vf[j][a]);", "acc += G[mu][i][j] * (vf[j][a] - vb[j][a]);"),
    ("backward link not daggered",
     "b += conj(Ub[3 * bb + a]) * pb[3 * sp + bb];", "b += Ub[3 * a + bb] * pb[3 * sp + bb];"),
    ("backward hop uses U_mu(x) instead of U_mu(x - mu)",
     "const cplx *Ub = U + (nb * 4 + mu) * 9;", "const cplx *Ub = U + (n * 4 + mu) * 9;"),
    ("hopping term sign", "o[3 * i + a] += -0.5 * acc;", "o[3 * i + a] += 0.5 * acc;"),
    ("Wilson diagonal d - m0 with d = 5", "o[i] += (4.0 - m0) * p[i];", "o[i] += (5.0 - m0) * p[i];"),
    ("corner of L_+ with the wrong sign", "Lp[0 * Ns + (Ns - 1)] += -kappa;", "Lp[0 * Ns + (Ns - 1)] += kappa;"),
    ("corner of L_+ dropped", "Lp[0 * Ns + (Ns - 1)] += -kappa;", "Lp[0 * Ns + (Ns - 1)] += 0.0 * kappa;"),
    ("L_+ and L_- exchanged", "for (int s = 1; s < Ns; s++) Lp[s * Ns + (s - 1)] = 1.0;",
     "for (int s = 1; s < Ns; s++) Lp[(s - 1) * Ns + s] = 1.0;"),
    ("X with (1 + L) for (1 - L)", "X[s * Ns + t] = (4.0 - m0) * omega[s] * onepcl + id - Lc[s * Ns + t];",
     "X[s * Ns + t] = (4.0 - m0) * omega[s] * onepcl + id + Lc[s * Ns + t];"),
    ("c = sigma omega instead of sigma / omega", "double c = sigma[s] / omega[s];", "double c = sigma[s] * omega[s];"),
    ("D: omega - sigma L", "t[i] = omega[s] * p[i] + sigma[s] * Lpsi[i];", "t[i] = omega[s] * p[i] - sigma[s] * Lpsi[i];"),
    ("D: 1 + L", "for (long i = 0; i < N; i++) o[i] += p[i] - Lpsi[i];",
     "for (long i = 0; i < N; i++) o[i] += p[i] + Lpsi[i];"),
    ("M5 similarity transform with sqrt(omega) swapped",
     "M[s * Ns + t] = T[s * Ns + t] * sqrt(omega[t]) / sqrt(omega[s]);",
     "M[s * Ns + t] = T[s * Ns + t] * sqrt(omega[s]) / sqrt(omega[t]);"),
    ("chiral projectors exchanged", "Pp[i][j] = 0.5 * ((i == j) + G[4][i][j]);   /* P_+ = (1 + gamma_5)/2 */",
     "Pp[i][j] = 0.5 * ((i == j) - G[4][i][j]);   /* P_+ = (1 + gamma_5)/2 */"),
    ("Schur complement 1 + M5 D M5 D", "out[k] = odd ? in[k] - S->t2[k] : 0;\n    }\n}\n\n/* C^dag",
     "out[k] = odd ? in[k] + S->t2[k] : 0;\n    }\n}\n\n/* C^dag"),
    ("CGNE accumulates p instead of u", "for (long i = 0; i < N; i++) { y[i] += alpha * u[i]; r[i] -= alpha * q[i]; }",
     "for (long i = 0; i < N; i++) { y[i] += alpha * p[i]; r[i] -= alpha * q[i]; }"),
    ("force-solve CG accumulates r instead of p",
     "for (long i = 0; i < N; i++) { ww[i] += alpha * p[i]; r[i] -= alpha * ap[i]; }",
     "for (long i = 0; i < N; i++) { ww[i] += alpha * r[i]; r[i] -= alpha * ap[i]; }"),
    ("true residual without the square root", "return n > 0 ? sqrt(r / n) : sqrt(r);",
     "return n > 0 ? (r / n) : sqrt(r);"),
    ("true residual relative to |D x| instead of |b|", "double r = norm2(N, dx), n = norm2(N, bb);",
     "double r = norm2(N, dx), n = norm2(N, bb) + r;"),
    ("initial guess read through S2 instead of S2^-1", "apply_s(&S.l, Ns, S2ip, S2im, xx, y);",
     "apply_s(&S.l, Ns, S2p, S2m, xx, y);"),
    ("CGNE direction update without beta (steepest descent)",
     "for (long i = 0; i < N; i++) p[i] = r[i] + beta * p[i];\n        rr = rr_new;\n        k++;\n    }\n    *iters = k;\n    *relres = bb",
     "for (long i = 0; i < N; i++) p[i] = r[i] + 0.0 * beta * p[i];\n        rr = rr_new;\n        k++;\n    }\n    *iters = k;\n    *relres = bb"),
    ("propagator projects the walls exchanged (P_+ psi_1 + P_- psi_Ns)",
     "acc += Pp[i][j] * x[(n * Ns + Ns - 1) * 12 + 3 * j + a] + Pm[i][j] * x[(n * Ns + 0) * 12 + 3 * j + a];",
     "acc += Pp[i][j] * x[(n * Ns + 0) * 12 + 3 * j + a] + Pm[i][j] * x[(n * Ns + Ns - 1) * 12 + 3 * j + a];"),
    ("propagator source without the (1 - sigma D_w) factor", "b[i] = c[i] - sigma[s] * dc[i];", "b[i] = c[i];"),
    ("propagator source with the chiralities of the walls exchanged",
     "c[(n * Ns + 0) * 12 + 3 * i + a] += ap;\n                c[(n * Ns + Ns - 1) * 12 + 3 * i + a] += am;",
     "c[(n * Ns + 0) * 12 + 3 * i + a] += am;\n                c[(n * Ns + Ns - 1) * 12 + 3 * i + a] += ap;"),
]


def _run(case, tmp):
    name, frag, repl = case
    src = open(SRC).read()
    assert src.count(frag) == 1, f"fragment not unique or missing: {name}"
    d = os.path.join(tmp, "m%d" % MUTANTS.index(case))
    os.makedirs(d, exist_ok=True)
    c, so = os.path.join(d, "o.c"), os.path.join(d, "o.so")
    open(c, "w").write(src.replace(frag, repl))
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", so, c, "-lm"])
    env = dict(os.environ, DWF_ORACLE_LIB=so, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        "-x", "-q", "-p", "no:cacheprovider", "--timeout", "120"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    return name, r.returncode, r.stdout[-400:]


def test_every_mutant_fails_a_pin(tmp_path):
    workers = min(8, os.cpu_count() or 1)
    with concurrent.futures.ThreadPoolExecutor(workers) as ex:
        results = list(ex.map(lambda m: _run(m, str(tmp_path)), MUTANTS))
    survivors = [(n, out) for n, rc, out in results if rc == 0]
    assert not survivors, survivors
    for n, rc, out in results:
        assert rc == 1, (n, rc, out)  # pins failed (not a crash of the run)


def test_unmutated_copy_passes(tmp_path):
    """The same build route without a mutation passes every pin."""
    src = open(SRC).read()
    c, so = str(tmp_path / "o.c"), str(tmp_path / "o.so")
    open(c, "w").write(src)
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", so, c, "-lm"])
    env = dict(os.environ, DWF_ORACLE_LIB=so, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_oracle_pins.py"), "-q",
                        "-p", "no:cacheprovider", "--timeout", "300"], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=900)
    assert r.returncode == 0, r.stdout[-2000:]
