"""GPU tests of kfbi_eval_batch (several densities in one call, in lockstep): every right-hand
side equals its own kfbi_eval (the same kernels on the same values, each stopping by the same
rule), matches the oracle to the parity tolerances (float64 1e-10, mixed 1e-6, in l2 and max),
and the batch serves the finite-difference check of the C4 geometry (Stokes star at 256^3):
32 evaluations K(phi0 +- eps d) for 16 directions against the hand-written transpose.
"""
import sys

import numpy as np
import pytest

import kfbi_inputs as KI

pytestmark = pytest.mark.gpu


def _say(m):
    print(m, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def K():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2303_04992_amd as K
    return K


def _errs(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b)), float(np.abs(a - b).max() / np.abs(b).max())


def _densities(cfg, xyz, n, k):
    ue = KI.exact_u(cfg.solution, xyz[:, 0], xyz[:, 1], xyz[:, 2])
    out = [ue] + [KI.random_density(n, seed=10 + i) for i in range(k - 1)]
    return np.stack(out)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("name,N,trace", [("sphere32", 32, "average"), ("ellip128", 32, "interior"),
                                          ("star128", 64, "average")])
def test_batch_equals_single_evaluations(K, name, N, trace, prec):
    """Five right-hand sides (a group of four and one more in the fit stage), two calls in a
    row (the second reuses the arenas), and a smaller batch afterwards."""
    cfg = KI.WORKLOADS[name].with_N(N)
    op = K.Operator(cfg, prec, trace=trace, cg_rtol=1e-12 if prec == 0 else 1e-9)
    xyz, _ = op.points()
    phis = _densities(cfg, xyz, op.n, 5)
    single = np.stack([op.eval(p).cpu().numpy() for p in phis])
    its = op.last_info["cg_iters"]
    for rep in range(2):
        batch = op.eval_batch(phis).cpu().numpy()
        worst = max(max(_errs(batch[r], single[r])) for r in range(len(phis)))
        _say(f"[batch {name} N={N} prec={prec} {trace}] call {rep}: worst rel diff vs single {worst:.2e}, "
             f"cg (sum) {op.last_info['cg_iters']}, single last {its}")
        assert worst < 1e-12
    small = op.eval_batch(phis[:2]).cpu().numpy()
    assert max(max(_errs(small[r], single[r])) for r in range(2)) < 1e-12
    # the context's own evaluation is untouched by the batches
    again = op.eval(phis[1]).cpu().numpy()
    assert max(_errs(again, single[1])) < 1e-12


@pytest.mark.parametrize("prec,tol", [(0, 1e-10), (1, 1e-6)])
def test_batch_matches_oracle_per_rhs(K, prec, tol):
    from oracle.kfbi import Oracle
    cfg = KI.WORKLOADS["star128"].with_N(64)
    O = Oracle(cfg, form="average")
    op = K.Operator(cfg, prec, cg_rtol=1e-12 if prec == 0 else 3e-6, inner_rtol=3e-6)
    xyz, _ = op.points()
    phis = _densities(cfg, xyz, op.n, 3)
    out = op.eval_batch(phis).cpu().numpy()
    for r in range(len(phis)):
        l2, mx = _errs(out[r], O.eval(phis[r]))
        _say(f"[batch oracle prec={prec}] rhs {r}: rel l2 {l2:.3e} rel max {mx:.3e}")
        assert l2 < tol and mx < tol


def test_batch_serves_finite_differences_on_the_c4_geometry(K):
    """Stokes star at 256^3 (float64): the gradient of l(phi) = 1/2 |K phi - t|^2 by the
    transpose (BIEEval backward) against central differences on 16 random directions, the 32
    evaluations K(phi0 +- eps d) in two batches of 16.  l is quadratic in phi, so the agreement
    is limited by the CG tolerance only."""
    import torch
    cfg = KI.WORKLOADS["star256"]
    op = K.Operator(cfg, K.FP64, cg_rtol=1e-13)
    xyz, _ = op.points()
    phi0 = torch.as_tensor(KI.exact_u(cfg.solution, xyz[:, 0], xyz[:, 1], xyz[:, 2]), device="cuda")
    target = 0.9 * phi0 + 0.05
    phi = phi0.clone().requires_grad_(True)
    L = 0.5 * ((K.BIEEval.apply(phi, op) - target) ** 2).sum()
    L.backward()
    grad = phi.grad.detach()
    dirs = torch.as_tensor(KI.random_directions(op.n, 16, seed=1), device="cuda")
    eps = 1e-2 * torch.linalg.norm(phi0).item()
    stack = torch.cat([phi0 + eps * dirs, phi0 - eps * dirs])  # (32, n, 3)
    with torch.no_grad():
        outs = torch.cat([op.eval_batch(stack[:16]), op.eval_batch(stack[16:])])
        loss = 0.5 * ((outs - target) ** 2).sum(dim=(1, 2))
        worst = 0.0
        for k in range(16):
            fd = (loss[k] - loss[16 + k]).item() / (2 * eps)
            an = float((grad * dirs[k]).sum().item())
            worst = max(worst, abs(fd - an) / max(abs(fd), 1e-30))
    _say(f"[batch fd] star256: worst rel diff over 16 directions {worst:.2e} (loss {L.item():.6e})")
    assert worst < 1e-6
