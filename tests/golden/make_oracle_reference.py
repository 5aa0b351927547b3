"""Write the oracle's K phi at full size for the GPU parity tests and the benchmark.

Calls only oracle/ (and the seeded inputs).  Usage:
    python tests/golden/make_oracle_reference.py star256
writes tests/golden/<name>_Kphi_uexact.npy: K phi for phi = u_exact at the control points
(float64, shape (n, 3), control-point order of the oracle), and a JSON sidecar with the
control-point count, the CG iteration count and the wall time.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import kfbi_inputs as KI  # noqa: E402
from oracle.kfbi import Oracle  # noqa: E402


def main(name, N=None):
    cfg = KI.WORKLOADS[name]
    if N is not None:
        cfg = cfg.with_N(int(N))
    tag = name if N is None else f"{name}_N{N}"
    t0 = time.time()
    O = Oracle(cfg, workers=os.cpu_count())
    t1 = time.time()
    X = O.points
    phi = KI.exact_u(cfg.solution, X[:, 0], X[:, 1], X[:, 2])
    K = O.eval(phi)
    t2 = time.time()
    np.save(os.path.join(HERE, f"{tag}_Kphi_uexact.npy"), K)
    meta = {"workload": name, "N": cfg.N, "n_points": int(O.n), "n_crossings": int(O.T),
            "cg_iters": int(O.last_cg_iters), "setup_s": t1 - t0, "eval_s": t2 - t1,
            "cg_rtol": O.cg_rtol, "input": "phi = exact velocity at the control points"}
    with open(os.path.join(HERE, f"{tag}_Kphi_uexact.json"), "w") as f:
        json.dump(meta, f, indent=1)
    print(meta)


if __name__ == "__main__":
    main(*sys.argv[1:])
