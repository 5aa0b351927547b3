"""Benchmark: kfbi_eval (one boundary-integral operator evaluation) at 256^3 on one GPU.

Workload: Stokes, mu = 1, box [-1,1]^3, star r = 0.5 + 0.1 sin(3 theta) cos(4 phi), N = 256
(M = 16.8 M cells, ~55 k control points), density phi = exact velocity at the control
points (synthetic, analytic; no dataset).  A step is one full K phi (jumps, corrections,
corrected MAC solve, interpolation) with inputs resident in HBM.

Prints one JSON line.  value = evaluations/s of the mixed form (float32 transforms and
inner CG inside float64 residual refinement; corrections, residuals, dot products and
interpolation in float64) run to a refinement tolerance that keeps the relative error
against the float64 oracle below 1e-6; beside it the float64 form at full accuracy and at
an equal-or-better accuracy, the relative errors against the oracle's stored result, the
roofline of the dominant transform-pass kernel (HIP events around its launches in the last
quarter of the timed evaluations) and the oracle's own rate on the host cores.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import kfbi_inputs as KI  # noqa: E402  (problem data only; no device work)

METRIC = "BIE operator evals/s at 256^3 (mixed vs FP64, rel err ≤1e-6) + HBM GB/s"
HBM_PEAK = 8000.0  # GB/s, MI355X
DCT2, DST2, DCT3, DST3, DST1 = 0, 1, 2, 3, 4
K_XMID, K_ZFWD, K_ZINV, K_YFWD, K_YINV = 5, 6, 7, 8, 9
KIND_NAMES = {DCT2: "k_pass DCT2", DST2: "k_pass DST2", DCT3: "k_pass DCT3", DST3: "k_pass DST3",
              DST1: "k_pass DST1", K_XMID: "k_xmid", K_ZFWD: "k_zfwd_cg", K_ZINV: "k_zinv_cg",
              K_YFWD: "k_ypair_fwd", K_YINV: "k_ypair_inv"}


def _host_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _schur_seconds(mac, N, budget_s):
    """Mean seconds of one oracle Schur-complement application (three sine-transform Poisson
    solves plus the MAC gradient and divergence), over as many as fit in budget_s (2 to 40)."""
    p = np.random.default_rng(0).standard_normal((N,) * 3)
    t0 = time.perf_counter()
    mac.schur(p)  # warm-up, also sizes the sample
    reps = int(min(40, max(2, budget_s / max(time.perf_counter() - t0, 1e-3))))
    t0 = time.perf_counter()
    for _ in range(reps):
        mac.schur(p)
    return (time.perf_counter() - t0) / reps, reps


def cpu_baseline(cfg, n_cg, calib_N=128):
    """The oracle as it stands, on the host cores, on a bounded sample of the workload.

    At the full size one K phi costs about (n_cg + 2) Schur-complement applications (the
    right-hand side and the velocity back-substitution add the equivalent of two); those are
    timed on a sample of about 10 s.  The remaining work of a complete evaluation (surface
    stages, sparse corrections and interpolation, Python overhead) is calibrated on the same
    workload at calib_N^3: complete oracle evaluations (median of 3 after a warm-up, setup not
    timed) against the same extrapolation at that size; the ratio is applied at full size."""
    from oracle.kfbi import Oracle
    from oracle.mac import MAC
    workers = os.cpu_count()
    c = cfg.with_N(calib_N)
    O = Oracle(c, workers=workers, form="average")
    X = O.points
    phi = KI.exact_u(c.solution, X[:, 0], X[:, 1], X[:, 2])
    O.eval(phi)
    full = []
    for _ in range(3):
        t0 = time.perf_counter()
        O.eval(phi)
        full.append(time.perf_counter() - t0)
    t_full = float(np.median(full))
    n_cg_c = O.last_cg_iters
    ts_c, _ = _schur_seconds(O.mac, calib_N, 3.0)
    factor = t_full / ((n_cg_c + 2) * ts_c)
    del O
    mac = MAC(cfg.N, cfg.lo, cfg.hi, cfg.pde, cfg.mu, cfg.lam, workers=workers)
    t, reps = _schur_seconds(mac, cfg.N, 10.0)
    extrap = t * (n_cg + 2)
    return {"value": 1.0 / (extrap * factor), "unit": "evals/s", "cores": workers, "kind": "oracle",
            "host": _host_model(),
            "sample": f"{reps} oracle Schur-complement applications at {cfg.N}^3 ({t:.3f} s each, scipy.fft "
                      f"workers={workers}) x (oracle CG count {n_cg} + 2) = {extrap:.2f} s, times the "
                      f"calibration factor {factor:.2f} = complete oracle K phi at {calib_N}^3 (median of 3: "
                      f"{t_full:.2f} s) / the same extrapolation at {calib_N}^3",
            "extrapolated_value": 1.0 / extrap, "calibration": {"N": calib_N, "full_eval_s": t_full,
                                                                "extrapolated_s": (n_cg_c + 2) * ts_c,
                                                                "factor": factor}}


def errs(out, ref):
    """Relative l2 and relative max error of out against the oracle's ref."""
    if ref is None or ref.shape != tuple(out.shape):
        return None
    o = out.cpu().numpy() if hasattr(out, "cpu") else out
    return {"l2": float(np.linalg.norm(o - ref) / np.linalg.norm(ref)),
            "max": float(np.abs(o - ref).max() / np.abs(ref).max())}


def run_form(K, KI, cfg, prec, rtol, inner, steps, warmup, refs, prof=None, trace="average"):
    """Time `steps` evaluations of K phi (phi = u_exact at the control points) after `warmup`;
    errors against the oracle for phi = u_exact and for the random density (refs: dict of
    oracle results by input name, or None)."""
    import torch
    t0 = time.perf_counter()
    op = K.Operator(cfg, prec, cg_rtol=rtol, inner_rtol=inner, trace=trace)
    setup_s = time.perf_counter() - t0
    xyz, _ = op.points()
    phi = torch.as_tensor(KI.exact_u(cfg.solution, xyz[:, 0], xyz[:, 1], xyz[:, 2]), dtype=torch.float64,
                          device="cuda")
    for _ in range(warmup):
        op.eval(phi)
    # the dominant kernel's launches are timed with HIP events in the last quarter of the timed
    # steps (each event pair adds a few microseconds between launches)
    prof_from = steps - max(1, steps // 4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        if prof is not None and i == prof_from:
            op.profile_pass(prof[0], prof[1], True)
        out = op.eval(phi)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    info = op.last_info
    res = {"ms_per_eval": dt * 1e3, "evals_per_s": 1.0 / dt, "cg_iters": info["cg_iters"],
           "refine_rounds": info["refine_rounds"], "setup_s": setup_s, "cg_rtol": rtol,
           "model_bytes": info["model_bytes"], "device_ms": info["ms_total"],
           "ms_stage": {k: round(v, 4) for k, v in info["ms_stage"].items()}}
    if prof is not None:
        n, ms, by = op.profile_pass(prof[0], prof[1], False)
        res["prof"] = {"launches": n, "avg_ms": ms / max(n, 1), "bytes": by}
        # every kernel of the CG iteration, live inside a few more evaluations (outside the timed loop)
        res["kernels"] = {}
        for kind, axis in ((K_ZFWD, -1), (K_YFWD, -1), (DST2, 1), (K_XMID, -1), (K_YINV, -1), (DST3, 1),
                           (K_ZINV, -1)):
            op.profile_pass(kind, axis, True)
            for _ in range(3):
                op.eval(phi)
            n, ms, by = op.profile_pass(kind, axis, False)
            if n == 0:
                continue
            name = KIND_NAMES[kind] + ("" if axis < 0 else f" axis {axis}")
            avg = ms / n
            res["kernels"][name] = {"avg_us": round(avg * 1e3, 2), "gb_s": round(by / (avg * 1e-3) / 1e9, 1)}
    if refs:
        res["err_uexact"] = errs(out, refs.get("uexact"))
        res["err_random"] = errs(op.eval(torch.as_tensor(KI.random_density(op.n), device="cuda")), refs.get("random"))
    del op
    torch.cuda.empty_cache()
    return res


def run_batch(K, KI, cfg, rtol, inner, nrhs, steps, refs):
    """kfbi_eval_batch: nrhs densities (u_exact and random ones) per call, mixed form; time per
    call and per right-hand side, and the errors of the u_exact right-hand side."""
    import torch
    op = K.Operator(cfg, K.MIXED_FP32, cg_rtol=rtol, inner_rtol=inner)
    xyz, _ = op.points()
    ue = KI.exact_u(cfg.solution, xyz[:, 0], xyz[:, 1], xyz[:, 2])
    phis = torch.as_tensor(np.stack([ue] + [KI.random_density(op.n, seed=10 + i) for i in range(nrhs - 1)]),
                           device="cuda")
    out = op.eval_batch(phis)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out = op.eval_batch(phis)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    info = op.last_info
    res = {"nrhs": nrhs, "ms_per_call": dt * 1e3, "ms_per_rhs": dt * 1e3 / nrhs, "evals_per_s": nrhs / dt,
           "cg_iters_sum": info["cg_iters"], "model_bytes": info["model_bytes"],
           "gb_s": info["model_bytes"] / (info["ms_total"] * 1e-3) / 1e9,
           "err_uexact_rhs0": errs(out[0], refs.get("uexact")) if refs else None}
    del op, phis, out
    torch.cuda.empty_cache()
    return res


def transforms_compare(K, KI, say, sizes=(128, 256, 512), reps=20):
    """The DCT-II along x of one float32 field: the radix pass (k_pass) beside the split-bfloat16
    matrix-core pass (k_gemm_x), mean launch time from HIP events (kfbi_time_pass), HBM rate of
    the two field passes and the matrix-core rate (3 bfloat16 products of 2 N^4 flops each)."""
    rows = []
    for N in sizes:
        op = K.Operator(KI.WORKLOADS["sphere32"].with_N(N), K.MIXED_FP32)
        for kind, name in ((0, "radix k_pass DCT2 x"), (10, "matrix-core k_gemm_x DCT2 x")):
            ms, by = op.time_pass(kind, 0, reps)
            row = {"N": N, "kernel": name, "avg_us": round(ms * 1e3, 2), "gb_s": round(by / (ms * 1e-3) / 1e9, 1),
                   "hbm_frac": round(by / (ms * 1e-3) / 1e9 / HBM_PEAK, 3)}
            if kind == 10:
                tf = 6.0 * N ** 4 / (ms * 1e-3) / 1e12
                row.update({"bf16_tflop_s": round(tf, 1), "mfma_frac": round(tf / 2500.0, 3)})
            say(json.dumps(row))
            rows.append(row)
        del op
    return rows


def copy_bandwidth(nbytes=1 << 30, reps=10):
    """Read+write bandwidth (GB/s) of a plain device-to-device copy of nbytes (larger than the
    256 MB last-level cache), timed with events on torch's current stream, where the copy runs."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9


def all_configs(K, KI, say):
    """Timings of every configuration (not part of the one-line result): K phi and K^T w in
    float64 and mixed form, and the Dirichlet BVP (volume trace, GMRES, unified solve)."""
    import torch
    rows = []
    for name, N, bvp in (("sphere32", 32, True), ("star128", 128, True), ("ellip128", 128, True),
                         ("star256", 256, True), ("star512n", 512, True)):
        cfg = KI.WORKLOADS[name].with_N(N)
        for prec, pname, rt in ((K.FP64, "fp64", 1e-12), (K.MIXED_FP32, "mixed", 1e-9)):
            t0 = time.perf_counter()
            op = K.Operator(cfg, prec, cg_rtol=rt, gmres_rtol=1e-8)
            setup = time.perf_counter() - t0
            xyz, _ = op.points()
            g = torch.as_tensor(KI.exact_u(cfg.solution, xyz[:, 0], xyz[:, 1], xyz[:, 2]), device="cuda")
            op.eval(g)
            reps = 5 if N >= 512 else 20
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                op.eval(g)
            torch.cuda.synchronize()
            te = (time.perf_counter() - t0) / reps
            t0 = time.perf_counter()
            for _ in range(reps):
                op.eval_adjoint(g)
            torch.cuda.synchronize()
            ta = (time.perf_counter() - t0) / reps
            row = {"config": name, "N": N, "form": pname, "setup_s": round(setup, 2), "eval_ms": round(te * 1e3, 2),
                   "adjoint_ms": round(ta * 1e3, 2)}
            if bvp:
                f = lambda x, y, z, c=cfg: KI.body_force(c.solution, x, y, z, c.mu, c.lam)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                op.solve_bvp(g, f)
                torch.cuda.synchronize()
                row.update({"bvp_s": round(time.perf_counter() - t0, 3), "gmres_iters": op.last_info["gmres_iters"]})
            say(json.dumps(row))
            rows.append(row)
            del op
            torch.cuda.empty_cache()
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="star256")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--calib-copy", action="store_true", help="run plain copies first (counter calibration)")
    # 8e-6 / 8e-6 (11 CG iterations at 256^3, one refinement round) keeps the errors against the
    # oracle (l2 and max, phi = u_exact and a random density, both trace forms) at or below 5.5e-7
    # from 64^3 to 256^3; 1e-5 / 1e-5 (10 iterations) leaves 1.2e-6 on the random density, and
    # 3e-6 to 6e-6 take 12 iterations for u_exact with the same errors
    ap.add_argument("--refine-rtol", type=float, default=8e-6, help="mixed: float64 residual tolerance")
    ap.add_argument("--inner-rtol", type=float, default=8e-6, help="mixed: float32 inner CG tolerance")
    ap.add_argument("--all-configs", action="store_true", help="time every configuration instead (one line each)")
    ap.add_argument("--transforms", action="store_true",
                    help="time the radix and the matrix-core DCT-II along x at 128^3, 256^3, 512^3 instead")
    ap.add_argument("--mixed-only", action="store_true",
                    help="time the headline mixed form only (for profiler runs; prints its result dict)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only (there is no multi-GPU path; the sharding design is "
              "described with the method); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import paper_2303_04992_amd as K

    if args.all_configs:
        all_configs(K, KI, lambda m: print(m, flush=True))
        return
    if args.transforms:
        transforms_compare(K, KI, lambda m: print(m, flush=True))
        return
    cfg = KI.WORKLOADS[args.workload]
    # the oracle's K phi at this size (tests/golden/make_oracle_reference.py), both trace forms,
    # phi = u_exact and the random density
    ref_path = os.path.join(ROOT, "tests", "golden", f"{args.workload}.npz")
    meta_path = ref_path.replace(".npz", ".json")
    meta = json.load(open(meta_path)) if os.path.exists(meta_path) else {}
    oracle_cg = meta.get("cg_iters_uexact", 30)
    refs = {"average": {}, "interior": {}}
    if os.path.exists(ref_path) and meta.get("N") == cfg.N and meta.get("rows") == "all":
        z = np.load(ref_path)
        for fm in refs:
            for inp in ("uexact", "random"):
                if f"Kphi_{inp}_{fm}" in z:
                    refs[fm][inp] = z[f"Kphi_{inp}_{fm}"]

    dominant = (K_XMID, -1)  # the fused x kernel: the largest share of the evaluation's kernel time
    say = lambda m: print(m, file=sys.stderr, flush=True)
    if args.calib_copy:
        # plain device-to-device copies of a known size (one float32 field, 64 MiB), to scale
        # hardware byte counters against
        import torch
        src = torch.ones(cfg.N ** 3, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        say(f"[bench] calibration copies: 3 x {src.numel() * 4} bytes")
    say("[bench] mixed")
    mx = run_form(K, KI, cfg, K.MIXED_FP32, args.refine_rtol, args.inner_rtol, args.steps, args.warmup,
                  refs["average"], prof=dominant)
    say(f"[bench] mixed: {mx}")
    if args.mixed_only:
        print(json.dumps({k: v for k, v in mx.items() if k != "kernels"}), flush=True)
        return
    say("[bench] mixed, interior trace form")
    mxi = run_form(K, KI, cfg, K.MIXED_FP32, args.refine_rtol, args.inner_rtol, max(3, args.steps // 4), 1,
                   refs["interior"], trace="interior")
    say(f"[bench] mixed interior: {mxi}")
    say("[bench] fp64 (full accuracy)")
    f64 = run_form(K, KI, cfg, K.FP64, 1e-12, 0.0, max(3, args.steps // 4), 1, refs["average"])
    say(f"[bench] fp64: {f64}")
    # float64 at equal accuracy: the loosest CG tolerance of the sweep whose errors (l2 and max,
    # u_exact and random density) are all at most the mixed form's
    def worst(r):
        e = [r.get("err_uexact"), r.get("err_random")]
        return max(v for x in e if x for v in x.values()) if any(e) else None
    target = worst(mx)
    f64e = None
    for rt in (1e-4, 3e-5, 1e-5, 6e-6, 3e-6, 1e-6, 3e-7, 1e-7, 1e-8):
        r = run_form(K, KI, cfg, K.FP64, rt, 0.0, max(3, args.steps // 2), 1, refs["average"])
        say(f"[bench] fp64 cg_rtol {rt:g}: {r['ms_per_eval']:.2f} ms, worst error {worst(r)}")
        if target is None or (worst(r) is not None and worst(r) <= target):
            f64e = r
            break
    if f64e is None:
        f64e = f64

    say("[bench] batch of 4 right-hand sides (kfbi_eval_batch)")
    bat = run_batch(K, KI, cfg, args.refine_rtol, args.inner_rtol, 4, max(3, args.steps // 4), refs["average"])
    say(f"[bench] batch: {bat}")

    pr = mx["prof"]
    achieved = pr["bytes"] / (pr["avg_ms"] * 1e-3) / 1e9
    copy_gbs = copy_bandwidth()
    say(f"[bench] device copy: {copy_gbs:.0f} GB/s")
    # measured HBM traffic of the dominant kernel (rocprofv3 FETCH_SIZE/WRITE_SIZE, copy-calibrated),
    # valid only while the transform sources are the ones that were profiled
    traffic = None
    tpath = os.path.join(ROOT, "profiles", "kfbi_eval_star256_traffic.json")
    if os.path.exists(tpath) and args.workload == "star256":
        import hashlib
        h = hashlib.sha256()
        for f in ("trig.h", "kernels.hip"):  # the kernel sources the counters were taken on
            h.update(open(os.path.join(ROOT, "paper_2303_04992_amd", "csrc", f), "rb").read())
        tj = json.load(open(tpath))
        if tj.get("source_sha") == h.hexdigest()[:16] and tj.get("kernel") == f"k_xmid<float,{cfg.N}>":
            traffic = tj["traffic_bytes_per_launch"]
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
        "config": {"workload": f"{args.workload}: Stokes mu=1, star r=0.5+0.1 sin3t cos4p in [-1,1]^3, N={cfg.N}, "
                               "phi=u_exact at the control points",
                   "N": cfg.N, "trace": "average", "refine_rtol": args.refine_rtol, "inner_rtol": args.inner_rtol},
        "rel_err_vs_oracle": (mx.get("err_uexact") or {}).get("l2"),
        "errors_vs_oracle": {
            "average": {"u_exact": mx.get("err_uexact"), "random": mx.get("err_random")},
            "interior": {"u_exact": mxi.get("err_uexact"), "random": mxi.get("err_random"),
                         "ms_per_eval": mxi["ms_per_eval"], "cg_iters": mxi["cg_iters"]}},
        "mixed": {k: mx[k] for k in ("cg_iters", "refine_rounds", "setup_s", "device_ms", "ms_stage")},
        "eval_bandwidth": {"model_bytes": mx["model_bytes"],
                           "gb_s": mx["model_bytes"] / (mx["device_ms"] * 1e-3) / 1e9,
                           "frac": mx["model_bytes"] / (mx["device_ms"] * 1e-3) / 1e9 / HBM_PEAK},
        "fp64": {k: f64.get(k) for k in ("evals_per_s", "ms_per_eval", "err_uexact", "err_random", "cg_iters",
                                         "cg_rtol")},
        "fp64_equal_accuracy": {k: f64e.get(k) for k in ("evals_per_s", "ms_per_eval", "err_uexact", "err_random",
                                                          "cg_iters", "cg_rtol")},
        "batch": bat,
        "speedup_mixed_over_fp64": mx["evals_per_s"] / f64["evals_per_s"],
        "speedup_mixed_over_fp64_equal_accuracy": mx["evals_per_s"] / f64e["evals_per_s"],
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK, "traffic": traffic,
                     "kernel": f"{KIND_NAMES[dominant[0]]}<float,{cfg.N}>",
                     "launches_timed": pr["launches"], "avg_us": pr["avg_ms"] * 1e3, "bytes_per_launch": pr["bytes"],
                     "copy_gb_s": copy_gbs, "frac_of_copy": achieved / copy_gbs},
        "cg_iteration_kernels": mx.get("kernels"),
    }
    if not args.no_cpu:
        say("[bench] cpu baseline (oracle)")
        line["cpu_baseline"] = cpu_baseline(cfg, oracle_cg)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
