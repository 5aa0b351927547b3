"""Write the oracle's K phi (and, on request, K^T w) at full size for the GPU parity tests and
the benchmark.

Calls only oracle/ (and the seeded inputs of kfbi_inputs).  One oracle setup serves both trace
forms (the interface solve is common to them) and every input density.  Usage:

    python tests/golden/make_oracle_reference.py star256 [--N 128] [--sample 4096] [--adjoint]

writes tests/golden/<tag>.npz (tag = the workload name, or <name>_N<N> with --N) holding, for
each trace form F in (average, interior) and density D in (uexact = exact velocity at the control
points, random = random_density(n), seed 2):

    Kphi_<D>_<F>   K phi, float64 (n, 3) in the oracle's control-point order (or the sampled rows)
    KTw_random_<F> K^T w for w = random_density(n)            (with --adjoint)
    idx            the sampled rows, sorted default_rng(7).choice(n, size, replace=False)
                   (with --sample; otherwise every row)

and a JSON sidecar <tag>.json with the sizes, the CG iteration counts and the wall times.
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

FORMS = ("average", "interior")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("name")
    ap.add_argument("--N", type=int, default=None)
    ap.add_argument("--sample", type=int, default=0, help="store only this many seeded rows")
    ap.add_argument("--adjoint", action="store_true", help="also K^T w for w = random_density(n)")
    ap.add_argument("--inputs", default="uexact,random", help="densities: uexact, random")
    a = ap.parse_args()
    cfg = KI.WORKLOADS[a.name]
    if a.N is not None:
        cfg = cfg.with_N(a.N)
    tag = a.name if a.N is None else f"{a.name}_N{a.N}"
    t0 = time.time()
    O = Oracle(cfg, workers=os.cpu_count(), form="average")  # holds the maps of both forms
    t1 = time.time()
    print(f"setup {t1 - t0:.1f} s, n = {O.n}, crossings = {O.T}", flush=True)
    X = O.points
    idx = (np.sort(np.random.default_rng(7).choice(O.n, size=min(a.sample, O.n), replace=False))
           if a.sample else np.arange(O.n))
    meta = {"workload": a.name, "N": cfg.N, "n_points": int(O.n), "n_crossings": int(O.T),
            "setup_s": t1 - t0, "cg_rtol": O.cg_rtol, "forms": list(FORMS), "workers": os.cpu_count(),
            "rows": ("sorted default_rng(7).choice(n, %d, replace=False)" % len(idx)) if a.sample else "all",
            "inputs": {k: v for k, v in (("uexact", "phi = exact velocity at the control points"),
                                         ("random", "phi = random_density(n), seed 2"))
                       if k in a.inputs.split(",")}}
    out = {"idx": idx}
    for inp in a.inputs.split(","):
        phi = (KI.exact_u(cfg.solution, X[:, 0], X[:, 1], X[:, 2]) if inp == "uexact"
               else KI.random_density(O.n))
        ts = time.time()
        both = O.eval_both(phi)
        meta[f"eval_{inp}_s"] = time.time() - ts
        meta[f"cg_iters_{inp}"] = int(O.last_cg_iters)
        for fm in FORMS:
            out[f"Kphi_{inp}_{fm}"] = both[fm][idx]
        print(f"K phi ({inp}) {meta[f'eval_{inp}_s']:.1f} s, cg {O.last_cg_iters}", flush=True)
    if a.adjoint:
        ts = time.time()
        both = O.eval_adjoint_both(KI.random_density(O.n))
        meta["adjoint_s"] = time.time() - ts
        meta["adjoint_cg_iters"] = int(O.last_cg_iters)
        meta["adjoint_input"] = "w = random_density(n), seed 2"
        for fm in FORMS:
            out[f"KTw_random_{fm}"] = both[fm][idx]
        print(f"K^T w {meta['adjoint_s']:.1f} s", flush=True)
    np.savez(os.path.join(HERE, f"{tag}.npz"), **out)
    with open(os.path.join(HERE, f"{tag}.json"), "w") as f:
        json.dump(meta, f, indent=1)
    print(meta)


if __name__ == "__main__":
    main()
