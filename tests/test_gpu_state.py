"""GPU regression test of the state a context keeps between calls.  An evaluation leaves the
right-hand side F (and, in the mixed form, its float32 copy) zero outside the irregular nodes,
so that the next evaluation only assigns those nodes; every other writer (the adjoint, the
volume force of a BVP, the probe adjoint) marks the buffers for a dense clear.  Interleaving
those calls on one context must leave K phi unchanged: each evaluation is compared with the
first one of the same context (the kernels reduce in a fixed order, so the values repeat to
rounding level, far below the parity tolerances).
"""
import sys

import numpy as np
import pytest

import kfbi_inputs as KI

pytestmark = pytest.mark.gpu


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


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
@pytest.mark.parametrize("name", ["sphere32", "ellip128"])
def test_interleaved_calls_leave_evaluations_unchanged(K, prec, name):
    import torch
    cfg = KI.WORKLOADS[name].with_N(64) if name == "ellip128" else KI.WORKLOADS[name]
    op = K.Operator(cfg, K.MIXED_FP32 if prec == "mixed" else K.FP64)
    xyz, _ = op.points()
    phi = torch.as_tensor(KI.random_density(len(xyz), seed=2), device="cuda")
    g = torch.as_tensor(KI.exact_u(cfg.solution, xyz[:, 0], xyz[:, 1], xyz[:, 2]), device="cuda")
    f = lambda x, y, z: KI.body_force(cfg.solution, x, y, z, cfg.mu, cfg.lam)
    ref = op.eval(phi).cpu().numpy()
    scale = np.linalg.norm(ref)

    def check(after):
        out = op.eval(phi).cpu().numpy()
        d = np.linalg.norm(out - ref) / scale
        _say(f"[state {name} {prec}] eval after {after}: rel diff {d:.2e}")
        assert d < 1e-12, (after, d)

    check("eval")
    op.eval_adjoint(phi)
    check("eval_adjoint")
    op.solve_bvp(g, f, return_fields=False)
    check("solve_bvp with body force")
    op.set_probes(KI.probe_points(cfg, 64))
    op.probe_adjoint(torch.ones((64, 3), dtype=torch.float64, device="cuda"))
    check("probe_adjoint")
    op.eval(2.0 * phi)
    check("eval of another density")


def test_stored_force_survives_a_force_free_solve(K):
    """The body force of the last kfbi_solve_bvp with f != NULL (its crossing jumps and its
    volume values, kept together) is what kfbi_probe(use_force=1) adds, also after a force-free
    BVP solve on the same context; the probe values match the oracle's unified interface solve
    with that force."""
    import torch
    from oracle.kfbi import Oracle
    cfg = KI.WORKLOADS["sphere32"]
    op = K.Operator(cfg, K.FP64, cg_rtol=1e-13)
    probes = KI.probe_points(cfg, 256, seed=0)
    op.set_probes(probes)
    xyz, _ = op.points()
    g = torch.as_tensor(KI.exact_u(cfg.solution, xyz[:, 0], xyz[:, 1], xyz[:, 2]), device="cuda")
    f = lambda x, y, z: KI.body_force(cfg.solution, x, y, z, cfg.mu, cfg.lam)
    phi = torch.as_tensor(KI.random_density(op.n, seed=4), device="cuda")
    op.solve_bvp(g, f, return_fields=False)
    forced = op.probe(phi, use_force=True).cpu().numpy()
    free = op.probe(phi, use_force=False).cpu().numpy()
    op.solve_bvp(g, None, return_fields=False)
    again = op.probe(phi, use_force=True).cpu().numpy()
    d = np.abs(again - forced).max() / np.abs(forced).max()
    _say(f"[force] probe with the stored force after a force-free solve: rel diff {d:.2e}")
    assert d < 1e-12
    assert np.abs(forced - free).max() > 1e-3 * np.abs(forced).max()
    O = Oracle(cfg, form="average")
    _, uo, _ = O.interface_solve(phi.cpu().numpy(), f)
    import test_gpu_autograd as TA
    ref = TA._trilinear(uo, probes, cfg.N, cfg.lo, cfg.h)
    r = np.abs(forced - ref).max() / np.abs(ref).max()
    _say(f"   against the oracle: rel max {r:.2e}")
    assert r < 1e-10
