"""GPU checks of the solver contracts behind K phi, through the C ABI:

* the MAC solve stops only when its residual is below the requested tolerance: the grid
  solution of kfbi_interface_solve is put back into the oracle's corrected MAC system
  (A_u u + G p = F_u, D u + c p = F_p, with the oracle's own right-hand side F for the same
  density) and the residual is recomputed in float64 on the host.  For the float64 path the
  pressure equation's residual is the Schur-complement residual b - S p (the velocity is
  back-substituted exactly), and it must be <= cg_rtol |b|; for the mixed path the full-system
  residual must be <= cg_rtol |F|, the refinement's stop rule;
* kfbi_solve_bvp_adjoint equals the composition of kfbi_probe_adjoint and kfbi_solve_adjoint;
* the stage times and model bytes reported in kfbi_info are consistent.
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


def _oracle_system(O, phi):
    """The oracle's corrected right-hand side (F_u, F_p) of the double-layer interface problem."""
    jumps = O.Jmat @ (O.Fit @ np.asarray(phi).ravel())
    return O.split_rhs(O.Cmat @ jumps)


@pytest.mark.parametrize("name", ["star128", "ellip128"])
@pytest.mark.parametrize("prec,rtol", [(0, 1e-8), (0, 1e-10), (1, 1e-5), (1, 1e-8)])
def test_mac_solve_meets_its_tolerance(K, name, prec, rtol):
    from oracle.kfbi import Oracle
    cfg = KI.WORKLOADS[name].with_N(64)
    O = Oracle(cfg, form="interior")
    mac = O.mac
    stokes = cfg.pde == KI.STOKES
    phi = KI.random_density(O.n)
    Fu, Fp = _oracle_system(O, phi)
    op = K.Operator(cfg, prec, cg_rtol=rtol, inner_rtol=1e-5)
    u, p = op.interface_solve(phi)
    info = op.last_info
    u = [x.cpu().numpy() for x in op.split_u(u)]
    p = p.cpu().numpy()
    Au, Dp = mac.apply(u, p)
    ru = [np.where(np.arange(cfg.N + 1).reshape([-1 if d == m else 1 for d in range(3)]) % cfg.N == 0, 0.0,
                   Fu[m] - Au[m]) for m in range(3)]
    rp = Fp - Dp
    if stokes:  # the continuity equation holds modulo constants (D u = F_p - mean F_p)
        rp = rp - rp.mean()
    nru = np.sqrt(sum(float(np.vdot(r, r)) for r in ru))
    nrp = float(np.linalg.norm(rp))
    if prec == 0:
        w = [mac.poisson(Fu[m], m) for m in range(3)]
        b = mac.project(Fp - mac.D(w))
        rel = nrp / np.linalg.norm(b)
        _say(f"[fp64 stop] {name} rtol {rtol:g}: cg {info['cg_iters']}  |b - S p|/|b| = {rel:.3e}  "
             f"|r_u| = {nru:.2e} (|F_u| {np.sqrt(sum(float(np.vdot(f, f)) for f in Fu)):.2e})")
        assert rel <= rtol
    else:
        Fp0 = Fp - Fp.mean() if stokes else Fp
        nF = np.sqrt(sum(float(np.vdot(f, f)) for f in Fu) + float(np.vdot(Fp0, Fp0)))
        rel = np.sqrt(nru ** 2 + nrp ** 2) / nF
        _say(f"[mixed stop] {name} rtol {rtol:g}: cg {info['cg_iters']} rounds {info['refine_rounds']}  "
             f"|r|/|F| = {rel:.3e}")
        assert rel <= rtol


def test_solve_bvp_adjoint_matches_composition(K):
    import torch
    cfg = KI.WORKLOADS["ellip128"].with_N(32)
    op = K.Operator(cfg, K.FP64, cg_rtol=1e-13, gmres_rtol=1e-12)
    op.set_probes(KI.probe_points(cfg, 256, seed=3))
    v = torch.as_tensor(np.random.default_rng(5).standard_normal((op.nprobe, 3)), device="cuda")
    pb_ref = op.probe_adjoint(v)
    gb_ref = op.solve_adjoint(pb_ref)
    gb, pb = op.solve_bvp_adjoint(v)
    dp = (torch.linalg.norm(pb - pb_ref) / torch.linalg.norm(pb_ref)).item()
    dg = (torch.linalg.norm(gb - gb_ref) / torch.linalg.norm(gb_ref)).item()
    _say(f"[bvp adjoint] phi_bar {dp:.2e}  g_bar {dg:.2e}  gmres {op.last_info['gmres_iters']}")
    assert dp < 1e-12 and dg < 1e-12
    gb2, none = op.solve_bvp_adjoint(v, want_phi=False)
    assert none is None
    assert (torch.linalg.norm(gb2 - gb_ref) / torch.linalg.norm(gb_ref)).item() < 1e-12
    with pytest.raises(K.KfbiError) as e:
        op.solve_bvp_adjoint(v, want_g=False, want_phi=False)
    assert e.value.status == K.EINVAL


@pytest.mark.parametrize("prec", [0, 1])
def test_info_stages_and_model_bytes(K, prec):
    import torch
    cfg = KI.WORKLOADS["star128"].with_N(64)
    op = K.Operator(cfg, prec)
    xyz, _ = op.points()
    phi = torch.as_tensor(KI.exact_u(cfg.solution, xyz[:, 0], xyz[:, 1], xyz[:, 2]), device="cuda")
    op.eval(phi)  # the first evaluation also clears the right-hand side densely
    op.eval(phi)
    a = op.last_info
    op.eval(phi)
    b = op.last_info
    st = a["ms_stage"]
    _say(f"[info] prec {prec}: {a['ms_total']:.3f} ms, stages {st}, model bytes {a['model_bytes'] / 1e6:.1f} MB, "
         f"cg {a['cg_iters']}")
    assert all(v >= 0 for v in st.values())
    assert abs(sum(st.values()) - a["ms_total"]) <= 1e-3 * a["ms_total"] + 1e-3
    assert st["cg"] > 0 and st["rhs"] > 0 and st["backsub"] > 0
    assert a["model_bytes"] == b["model_bytes"] and a["cg_iters"] == b["cg_iters"]
    # at least the Schur CG iterations' own traffic (29 fields of N^3 per iteration, float32 in
    # the mixed form's inner solves)
    s = 8 if prec == 0 else 4
    assert a["model_bytes"] > 29 * cfg.N ** 3 * s * a["cg_iters"]
    op.eval_adjoint(phi)
    c = op.last_info
    assert c["model_bytes"] > 0 and abs(sum(c["ms_stage"].values()) - c["ms_total"]) <= 1e-3 * c["ms_total"] + 1e-3
