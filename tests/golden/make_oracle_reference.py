"""Write the oracle's K phi (and, on request, K^T w) at full size for the GPU parity tests and
the benchmark.

Calls only oracle/ (and the seeded inputs).  Usage:
    python tests/golden/make_oracle_reference.py star256 [--form average|interior]
        writes tests/golden/star256_Kphi_uexact.npy: K phi for phi = u_exact at the control
        points (float64, shape (n, 3), control-point order of the oracle), and a JSON sidecar
        with the control-point count, the CG iteration count and the wall time.
    python tests/golden/make_oracle_reference.py star512n --sample 4096 --adjoint
        writes tests/golden/star512n_sample.npz with a seeded sample of control points
        (idx, seed 7) and, at those rows only, K phi for phi = u_exact (Kphi) and K^T w for
        w = random_density(n) (KTw), plus the JSON sidecar.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import kfbi_inputs as KI  # noqa: E402
from oracle.kfbi import Oracle  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("name")
    ap.add_argument("--N", type=int, default=None)
    ap.add_argument("--sample", type=int, default=0, help="store only this many seeded rows")
    ap.add_argument("--adjoint", action="store_true", help="also K^T w for w = random_density(n)")
    ap.add_argument("--form", default="average", choices=["average", "interior"], help="trace form of K")
    a = ap.parse_args()
    cfg = KI.WORKLOADS[a.name]
    if a.N is not None:
        cfg = cfg.with_N(a.N)
    tag = a.name if a.N is None else f"{a.name}_N{a.N}"
    t0 = time.time()
    O = Oracle(cfg, workers=os.cpu_count(), form=a.form)
    t1 = time.time()
    print(f"setup {t1 - t0:.1f} s, n = {O.n}, crossings = {O.T}", flush=True)
    X = O.points
    phi = KI.exact_u(cfg.solution, X[:, 0], X[:, 1], X[:, 2])
    K = O.eval(phi)
    t2 = time.time()
    meta = {"workload": a.name, "N": cfg.N, "n_points": int(O.n), "n_crossings": int(O.T),
            "cg_iters": int(O.last_cg_iters), "setup_s": t1 - t0, "eval_s": t2 - t1,
            "cg_rtol": O.cg_rtol, "form": a.form, "input": "phi = exact velocity at the control points"}
    print(meta, flush=True)
    if a.sample:
        idx = np.sort(np.random.default_rng(7).choice(O.n, size=min(a.sample, O.n), replace=False))
        out = {"idx": idx, "Kphi": K[idx]}
        if a.adjoint:
            KT = O.eval_adjoint(KI.random_density(O.n))
            meta["adjoint_cg_iters"] = int(O.last_cg_iters)
            meta["adjoint_s"] = time.time() - t2
            meta["adjoint_input"] = "w = random_density(n), seed 2"
            out["KTw"] = KT[idx]
        meta["sample"] = "rows idx = sorted default_rng(7).choice(n, size, replace=False)"
        np.savez(os.path.join(HERE, f"{tag}_sample.npz"), **out)
        path = os.path.join(HERE, f"{tag}_sample.json")
    else:
        if a.adjoint:
            raise SystemExit("--adjoint needs --sample")
        np.save(os.path.join(HERE, f"{tag}_Kphi_uexact.npy"), K)
        path = os.path.join(HERE, f"{tag}_Kphi_uexact.json")
    with open(path, "w") as f:
        json.dump(meta, f, indent=1)
    print(meta)


if __name__ == "__main__":
    main()
