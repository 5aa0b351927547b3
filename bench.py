"""Benchmark: kfbi_eval (one boundary-integral operator evaluation) at 256^3 on one GPU.

Workload: Stokes, mu = 1, box [-1,1]^3, star r = 0.5 + 0.1 sin(3 theta) cos(4 phi), N = 256
(M = 16.8 M cells, ~55 k control points), density phi = exact velocity at the control
points (synthetic, seeded/analytic; no dataset).  A step is one full K phi (jumps,
corrections, corrected MAC solve, interpolation) with inputs resident in HBM.

Prints one JSON line: value = evaluations/s of the mixed form (float32 transforms and inner
CG, float64 corrections/residuals/dots/refinement), with the float64 form, the relative
error of both against the float64 oracle's stored result, the transform-pass roofline and
the oracle's CPU rate beside it.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "BIE operator evals/s at 256^3 (mixed vs FP64, rel err ≤1e-6) + HBM GB/s"
HBM_PEAK = 8000.0  # GB/s, MI355X


def cpu_baseline(cfg, n_cg):
    """The oracle as it stands, on the host cores, on a bounded sample: two Schur-complement
    applications (each three sine-transform Poisson solves plus the MAC gradient and
    divergence) at the full 256^3 size; one K phi costs about (n_cg + 2) of them (RHS and
    velocity back-substitution add the equivalent of two), the surface stages are <1%."""
    from oracle.mac import MAC
    workers = os.cpu_count()
    mac = MAC(cfg.N, cfg.lo, cfg.hi, cfg.pde, cfg.mu, cfg.lam, workers=workers)
    p = np.random.default_rng(0).standard_normal((cfg.N,) * 3)
    mac.schur(p)  # warm-up
    t0 = time.perf_counter()
    reps = 2
    for _ in range(reps):
        mac.schur(p)
    t = (time.perf_counter() - t0) / reps
    evals_per_s = 1.0 / (t * (n_cg + 2))
    return {"value": evals_per_s, "unit": "evals/s", "cores": workers, "kind": "oracle",
            "sample": f"{reps} oracle Schur-complement applications at {cfg.N}^3 ({t:.2f} s each), "
                      f"scaled by the oracle's CG count + 2 = {n_cg + 2}"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="star256")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--mixed-rtol", type=float, default=1e-9)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(see the sharding design); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import kfbi_inputs as KI
    import paper_2303_04992_amd as K

    cfg = KI.WORKLOADS[args.workload]
    ref_path = os.path.join(ROOT, "tests", "golden", f"{args.workload}_Kphi_uexact.npy")
    ref = np.load(ref_path) if os.path.exists(ref_path) else None
    meta_path = ref_path.replace(".npy", ".json")
    oracle_cg = json.load(open(meta_path))["cg_iters"] if os.path.exists(meta_path) else 30

    results = {}
    for name, prec, rtol in (("fp64", K.FP64, 1e-12), ("mixed", K.MIXED_FP32, args.mixed_rtol)):
        print(f"[bench] {name}: setup", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        op = K.Operator(cfg, prec, cg_rtol=rtol, inner_rtol=1e-5)
        setup_s = time.perf_counter() - t0
        xyz, _ = op.points()
        phi = torch.as_tensor(KI.exact_u(cfg.solution, xyz[:, 0], xyz[:, 1], xyz[:, 2]),
                              dtype=torch.float64, device="cuda")
        for _ in range(args.warmup):
            op.eval(phi)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = []
        for _ in range(args.steps):
            out = op.eval(phi)
            infos.append(op.last_info)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        rel = None
        if ref is not None and ref.shape == tuple(out.shape):
            o = out.cpu().numpy()
            rel = float(np.linalg.norm(o - ref) / np.linalg.norm(ref))
        # roofline of the dominant kernel (the transform pass), HIP events on the op's stream
        kms, kbytes = op.time_pass(kind=1, axis=1, reps=20)
        results[name] = {"ms_per_eval": dt * 1e3, "evals_per_s": 1.0 / dt, "rel_err_vs_oracle": rel,
                         "cg_iters": infos[-1]["cg_iters"], "refine_rounds": infos[-1]["refine_rounds"],
                         "setup_s": setup_s, "pass_ms": kms, "pass_bytes": kbytes,
                         "ms_stage": infos[-1]["ms_stage"][:3]}
        print(f"[bench] {name}: {results[name]}", file=sys.stderr, flush=True)
        del op
        torch.cuda.empty_cache()

    mx = results["mixed"]
    achieved = mx["pass_bytes"] / (mx["pass_ms"] * 1e-3) / 1e9
    line = {
        "metric": METRIC,
        "value": mx["evals_per_s"],
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mx["ms_per_eval"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic (analytic manufactured density on a level-set star)",
        "config": {"workload": f"{args.workload}: Stokes mu=1, star r=0.5+0.1 sin3t cos4p in [-1,1]^3, "
                               f"N={cfg.N}, phi=u_exact at control points",
                   "N": cfg.N, "mixed_refine_rtol": args.mixed_rtol},
        "fp64": {"evals_per_s": results["fp64"]["evals_per_s"], "ms_per_eval": results["fp64"]["ms_per_eval"],
                 "rel_err_vs_oracle": results["fp64"]["rel_err_vs_oracle"], "cg_iters": results["fp64"]["cg_iters"]},
        "mixed": {"rel_err_vs_oracle": mx["rel_err_vs_oracle"], "cg_iters": mx["cg_iters"],
                  "refine_rounds": mx["refine_rounds"]},
        "speedup_mixed_over_fp64": mx["evals_per_s"] / results["fp64"]["evals_per_s"],
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK, "traffic": None,
                     "kernel": "k_pass<float,256,DST2> (y axis)"},
    }
    if not args.no_cpu:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(cfg, oracle_cg)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
