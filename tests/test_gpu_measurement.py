"""GPU tests of the measurement helpers that bench.py relies on: kfbi_time_pass launches every
kernel kind (the single transform passes along each axis, including the persistent pipelined
inverse passes, and the fused kernels of the Schur-CG iteration) and reports the documented
algorithmic bytes; kfbi_profile_pass records one launch of a fused kernel per CG iteration
inside real evaluations (the z pass counts the iterations with the fused vector updates).  A
float64 context checks the double-precision kernels as well.
"""
import sys

import pytest

import kfbi_inputs as KI

pytestmark = pytest.mark.gpu

# fields (of N^3 values) read or written by one launch, as documented in include/kfbi.h
FIELDS = {0: 2, 1: 2, 2: 2, 3: 2, 4: 2, 5: 6, 6: 9, 7: 4, 8: 3, 9: 3}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def K():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2303_04992_amd as K
    return K


@pytest.mark.parametrize("prec,size", [("mixed", 4), ("fp64", 8)])
def test_time_pass_reports_documented_bytes(K, prec, size):
    cfg = KI.WORKLOADS["sphere32"]
    op = K.Operator(cfg, K.MIXED_FP32 if prec == "mixed" else K.FP64)
    M = cfg.N ** 3
    for kind, f in FIELDS.items():
        for axis in (range(3) if kind < 5 else [0]):
            _say(f"[time_pass {prec}] kind {kind} axis {axis}")
            ms, by = op.time_pass(kind, axis, 3)
            assert ms > 0.0, (kind, axis, ms)
            assert by == f * M * size, (kind, axis, by)


def test_profile_pass_counts_one_launch_per_cg_iteration(K):
    import torch
    cfg = KI.WORKLOADS["sphere32"]
    op = K.Operator(cfg, K.MIXED_FP32)
    xyz, _ = op.points()
    phi = torch.as_tensor(KI.exact_u(cfg.solution, xyz[:, 0], xyz[:, 1], xyz[:, 2]), device="cuda")
    op.eval(phi)
    for kind in (5, 6, 7, 8, 9):
        op.profile_pass(kind, -1, True)
        op.eval(phi)
        n, ms, by = op.profile_pass(kind, -1, False)
        iters = op.last_info["cg_iters"]
        # the first iteration of each inner solve uses the z pass without the vector updates
        expect = iters - op.last_info["refine_rounds"] if kind == 6 else iters
        _say(f"[profile_pass] kind {kind}: {n} launches, {ms:.3f} ms, CG iterations {iters}")
        assert n == expect, (kind, n, iters)
        assert ms > 0.0 and by == FIELDS[kind] * cfg.N ** 3 * 4
