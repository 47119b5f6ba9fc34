"""Write sampled entries of the oracle's solution of D x = b for a named workload.

Calls only the CPU oracle (``oracle/``) and the seeded input generators.  The
JSON written here is the stored expected value that the GPU solve tests compare
against at full size, where running the oracle inside a test would take too
long.  Usage:

    python tests/golden/make_oracle_samples.py odwf_16x16x16x32_ns16
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import dwf_inputs as inp  # noqa: E402
import oracle  # noqa: E402

NSAMPLE = 4096
SAMPLE_SEED = 4242


def main(name, tol=1e-12, rhs_index=None):
    w = inp.workload(name)
    dims, ns = w["dims"], w["ns"]
    U = inp.gauge_field(dims, w["eps"], seed=w["seed_gauge"])
    if rhs_index is None:
        b = inp.gaussian_spinor(dims, ns, seed=w["seed_rhs"])
    else:
        srcs, _ = inp.point_sources(dims, ns, seed=w["seed_rhs"])
        b = np.ascontiguousarray(srcs[rhs_index])
    t0 = time.time()
    args = (U, dims, ns, w["m0"], w["mq"], w["sigma"], w["omega"])
    x, info = oracle.solve(*args, b, tol=tol)
    elapsed = time.time() - t0
    res = oracle.true_residual(*args, b, x)
    flat = x.ravel()
    idx = np.sort(np.random.default_rng(SAMPLE_SEED).choice(flat.size, NSAMPLE, replace=False))
    out = dict(workload=name, rhs_index=rhs_index, tol=tol, oracle_iters=info["iters"],
               oracle_schur_res=info["schur_res"], true_residual=res,
               norm_x=float(np.linalg.norm(flat)), norm_b=float(np.linalg.norm(b)),
               sample_seed=SAMPLE_SEED, indices=idx.tolist(), values=flat[idx].tolist(),
               oracle_seconds=elapsed, oracle_threads=oracle.num_threads())
    suffix = "" if rhs_index is None else f"_rhs{rhs_index}"
    path = os.path.join(HERE, f"{name}{suffix}_oracle_samples.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(path, info, res, elapsed)


if __name__ == "__main__":
    main(sys.argv[1], rhs_index=int(sys.argv[2]) if len(sys.argv) > 2 else None)
