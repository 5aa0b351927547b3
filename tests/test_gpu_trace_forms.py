"""GPU parity of the average trace form (K phi = 1/2 phi + mean of the two one-sided limits,
with the fitted jump value at the control point) against the oracle, its transpose, and the
GMRES iteration counts of the two forms.

Tolerances as in the interior-form parity tests: 1e-10 relative for the float64 path, 1e-6
for the mixed path.
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


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("name,N", [("sphere32", 32), ("star128", 64), ("ellip128", 64)])
def test_average_eval_matches_oracle(K, name, N):
    from oracle.kfbi import Oracle
    cfg = KI.WORKLOADS[name].with_N(N)
    _say(f"[average fp64] {name} N={N}")
    op = K.Operator(cfg, K.FP64, cg_rtol=1e-12, trace="average")
    O = Oracle(cfg, form="average")
    xyz, _ = op.points()
    for phi in (KI.exact_u(cfg.solution, xyz[:, 0], xyz[:, 1], xyz[:, 2]), KI.random_density(op.n)):
        r = _rel(op.eval(phi).cpu().numpy(), O.eval(phi))
        _say(f"   rel l2 {r:.3e}")
        assert r < 1e-10


def test_average_eval_mixed_matches_oracle(K):
    from oracle.kfbi import Oracle
    cfg = KI.WORKLOADS["star128"].with_N(64)
    _say("[average mixed] star128 N=64")
    op = K.Operator(cfg, K.MIXED_FP32, cg_rtol=1e-9, inner_rtol=1e-5, trace="average")
    O = Oracle(cfg, form="average")
    phi = KI.random_density(op.n)
    r = _rel(op.eval(phi).cpu().numpy(), O.eval(phi))
    _say(f"   rel l2 {r:.3e}")
    assert r < 1e-6


def test_average_adjoint_matches_oracle_and_transposes(K):
    from oracle.kfbi import Oracle
    cfg = KI.WORKLOADS["ellip128"].with_N(32)
    _say("[average adjoint] ellip128 N=32")
    op = K.Operator(cfg, K.FP64, cg_rtol=1e-13, trace="average")
    O = Oracle(cfg, form="average")
    rng = np.random.default_rng(12)
    x = rng.standard_normal((op.n, 3))
    y = rng.standard_normal((op.n, 3))
    kty = op.eval_adjoint(y).cpu().numpy()
    assert _rel(kty, O.eval_adjoint(y)) < 1e-10
    lhs = float(np.vdot(op.eval(x).cpu().numpy(), y))
    rhs = float(np.vdot(x, kty))
    _say(f"   <Kx,y>={lhs:.12e} <x,K^T y>={rhs:.12e}")
    assert abs(lhs - rhs) < 1e-10 * (abs(lhs) + np.linalg.norm(x) * np.linalg.norm(y))


def test_average_bvp_matches_oracle(K):
    from oracle.kfbi import Oracle
    cfg = KI.WORKLOADS["sphere32"]
    _say("[average bvp] sphere32")
    op = K.Operator(cfg, K.FP64, cg_rtol=1e-13, gmres_rtol=1e-11, trace="average")
    O = Oracle(cfg, form="average")
    xyz, _ = op.points()
    g = KI.exact_u(cfg.solution, xyz[:, 0], xyz[:, 1], xyz[:, 2])
    f = lambda x, y, z: KI.body_force(cfg.solution, x, y, z, cfg.mu, cfg.lam)
    phi, u, p = op.solve_bvp(g, f)
    it = op.last_info["gmres_iters"]
    phio, uo, po, ito, _ = O.solve_bvp(g, f, tol=1e-11)
    r = _rel(phi.cpu().numpy(), phio)
    _say(f"   gmres {it} (oracle {ito})  rel phi {r:.3e}")
    assert r < 1e-8
    assert abs(it - ito) <= 2


@pytest.mark.parametrize("name,N", [("sphere32", 64), ("star128", 64)])
def test_average_form_needs_fewer_gmres_iterations(K, name, N):
    """Random (grid-scale rough) right-hand side, GMRES to 1e-8: the average form converges in
    well under half the iterations of the interior form."""
    import torch
    cfg = KI.WORKLOADS[name].with_N(N)
    its = {}
    for trace in ("interior", "average"):
        op = K.Operator(cfg, K.FP64, cg_rtol=1e-12, gmres_rtol=1e-8, gmres_maxit=600, trace=trace)
        b = torch.as_tensor(KI.random_directions(op.n, 1, seed=1)[0], device="cuda")
        try:
            y = op.solve_adjoint(b)  # K^T has the spectrum of K
        except K.KfbiError as e:  # the interior form may not get there within gmres_maxit
            assert trace == "interior" and e.status == K.ENOCONV
            its[trace] = 600
            continue
        its[trace] = op.last_info["gmres_iters"]
        res = torch.linalg.norm(op.eval_adjoint(y) - b) / torch.linalg.norm(b)
        assert res.item() < 1e-7
    _say(f"[gmres counts] {name} N={N}: {its}")
    assert its["average"] < 0.5 * its["interior"], its
