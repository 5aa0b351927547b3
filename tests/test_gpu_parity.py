"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Every comparison is made in two norms over all control points and components: relative l2,
||K_gpu - K_oracle||_2 / ||K_oracle||_2, and relative max, max|K_gpu - K_oracle| / max|K_oracle|,
so that one bad control point cannot hide in the l2 average.  Both trace forms of K (average,
the default, and interior, the literal Sec. 4.4 reading) are checked in every case.

Tolerances: the float64 path matches the oracle to 1e-10 -- both sides solve the Schur
system by CG to 1e-12 / 1e-13 relative residual, so their results differ only at that level;
the mixed path (float32 transforms and inner CG inside float64 refinement) to 1e-6, the
accuracy the mixed form is specified for, both at a tight refinement tolerance (1e-9) and at
the benchmark's settings (refinement 8e-6, inner CG 8e-6) on rough (random) densities.
"""
import json
import os
import sys

import numpy as np
import pytest

import kfbi_inputs as KI

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
FORMS = ("average", "interior")
# the benchmark's mixed settings (bench.py defaults)
BENCH_REFINE, BENCH_INNER = 8e-6, 8e-6


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


def _errs(a, b):
    """(relative l2, relative max) of a against the reference b."""
    a, b = np.asarray(a), np.asarray(b)
    return (float(np.linalg.norm(a - b) / np.linalg.norm(b)), float(np.abs(a - b).max() / np.abs(b).max()))


def _check(tag, a, b, tol):
    l2, mx = _errs(a, b)
    _say(f"   {tag}: rel l2 {l2:.3e}  rel max {mx:.3e}")
    assert l2 < tol and mx < tol, (tag, l2, mx)


def _golden(tag):
    path = os.path.join(HERE, "golden", f"{tag}.npz")
    if not os.path.exists(path):
        pytest.skip(f"oracle reference {tag} not generated (tests/golden/make_oracle_reference.py)")
    return np.load(path), json.load(open(path.replace(".npz", ".json")))


# (workload, N) at sizes the oracle finishes in seconds; several tiles and a ragged number of
# control points each; the torus cases are the geometry of the paper's Examples 5.3 (Stokes)
# and 5.6 (Navier)
CASES = [("sphere32", 32), ("star128", 64), ("ellip128", 64), ("star512n", 64), ("ex53", 32), ("ex56", 64)]


@pytest.mark.parametrize("name,N", CASES)
def test_eval_fp64_matches_oracle(K, name, N):
    from oracle.kfbi import Oracle
    cfg = KI.WORKLOADS[name].with_N(N)
    O = Oracle(cfg, form="average")
    for form in FORMS:
        _say(f"[parity fp64] {name} N={N} trace={form}")
        op = K.Operator(cfg, K.FP64, cg_rtol=1e-12, trace=form)
        xyz, _ = op.points()
        assert xyz.shape == O.points.shape
        assert np.abs(xyz - O.points).max() < 1e-13
        for tag, phi in (("u_exact", KI.exact_u(cfg.solution, xyz[:, 0], xyz[:, 1], xyz[:, 2])),
                         ("random", KI.random_density(op.n))):
            _check(tag, op.eval(phi).cpu().numpy(), O.eval(phi, form=form), 1e-10)


@pytest.mark.parametrize("name,N", [("sphere32", 32), ("star128", 64), ("ellip128", 64), ("ex56", 64)])
def test_eval_mixed_matches_oracle(K, name, N):
    """Mixed form at a tight refinement tolerance (1e-9) and, from 64^3 up, at the benchmark's
    settings, on a random density (grid-scale rough, the hardest input for the float32 inner
    solves).  The benchmark's settings are chosen for its sizes: at 32^3 they leave 1.1e-6 on
    this input, so there only the tight tolerance is held to 1e-6."""
    from oracle.kfbi import Oracle
    cfg = KI.WORKLOADS[name].with_N(N)
    O = Oracle(cfg, form="average")
    phi = KI.random_density(O.n)
    ref = O.eval_both(phi)
    for form in FORMS:
        for refine, inner in ((1e-9, 1e-5),) + (((BENCH_REFINE, BENCH_INNER),) if N >= 64 else ()):
            _say(f"[parity mixed] {name} N={N} trace={form} refine={refine} inner={inner}")
            op = K.Operator(cfg, K.MIXED_FP32, cg_rtol=refine, inner_rtol=inner, trace=form)
            _check("random", op.eval(phi).cpu().numpy(), ref[form], 1e-6)
            _say(f"   info {op.last_info['cg_iters']} cg, {op.last_info['refine_rounds']} rounds")


@pytest.mark.parametrize("tag", ["star128", "ellip128", "star256"])
def test_full_size_matches_stored_oracle(K, tag):
    """At the workloads' own sizes (128^3 for the star Stokes and rotated-ellipsoid Navier
    workloads, 256^3 for the headline star) the oracle's K phi for phi = u_exact and for a
    random density, in both trace forms (tests/golden/make_oracle_reference.py), against the
    float64 path (1e-10), the mixed path at refinement 1e-9 (1e-6) and at the benchmark's
    settings (1e-6)."""
    z, meta = _golden(tag)
    cfg = KI.WORKLOADS[tag]
    assert cfg.N == meta["N"]
    runs = ((K.FP64, 1e-12, 0.0, 1e-10), (K.MIXED_FP32, 1e-9, 1e-5, 1e-6),
            (K.MIXED_FP32, BENCH_REFINE, BENCH_INNER, 1e-6))
    for form in FORMS:
        for prec, rtol, inner, tol in runs:
            _say(f"[full size] {tag} precision={prec} cg_rtol={rtol} trace={form}")
            op = K.Operator(cfg, prec, cg_rtol=rtol, inner_rtol=inner, trace=form)
            assert op.n == meta["n_points"]
            xyz, _ = op.points()
            for inp in ("uexact", "random"):
                phi = (KI.exact_u(cfg.solution, xyz[:, 0], xyz[:, 1], xyz[:, 2]) if inp == "uexact"
                       else KI.random_density(op.n))
                _check(f"{inp}", op.eval(phi).cpu().numpy(), z[f"Kphi_{inp}_{form}"], tol)
            _say(f"   info {op.last_info['cg_iters']} cg, {op.last_info['refine_rounds']} rounds, "
                 f"{op.last_info['ms_total']:.2f} ms")
            del op


def test_constant_density_identity_full_size(K):
    """K c = c holds exactly for the discrete scheme (any size); at 256^3 the GPU result
    differs from c only by the CG tolerance."""
    cfg = KI.WORKLOADS["star256"]
    c = np.array([0.3, -0.7, 1.1])
    for form in FORMS:
        _say(f"[identity] star256 K c = c trace={form}")
        op = K.Operator(cfg, K.FP64, cg_rtol=1e-12, trace=form)
        out = op.eval(np.tile(c, (op.n, 1))).cpu().numpy()
        err = np.abs(out - c).max()
        _say(f"   max |Kc - c| = {err:.3e}  cg {op.last_info['cg_iters']}")
        assert err < 1e-9


@pytest.mark.parametrize("name,N", [("sphere32", 32), ("ellip128", 32), ("ex53", 32)])
def test_adjoint_matches_oracle_and_transposes(K, name, N):
    from oracle.kfbi import Oracle
    cfg = KI.WORKLOADS[name].with_N(N)
    O = Oracle(cfg, form="average")
    rng = np.random.default_rng(11)
    x = rng.standard_normal((O.n, 3))
    y = rng.standard_normal((O.n, 3))
    ref = O.eval_adjoint_both(y)
    for form in FORMS:
        _say(f"[adjoint] {name} N={N} trace={form}")
        op = K.Operator(cfg, K.FP64, cg_rtol=1e-13, trace=form)
        kty = op.eval_adjoint(y).cpu().numpy()
        _check("K^T y", kty, ref[form], 1e-10)
        lhs = float(np.vdot(op.eval(x).cpu().numpy(), y))
        rhs = float(np.vdot(x, kty))
        _say(f"   <Kx,y>={lhs:.12e} <x,K^T y>={rhs:.12e}")
        assert abs(lhs - rhs) < 1e-10 * (abs(lhs) + np.linalg.norm(x) * np.linalg.norm(y))


def test_bvp_matches_oracle(K):
    from oracle.kfbi import Oracle
    cfg = KI.WORKLOADS["sphere32"]
    O = Oracle(cfg, form="average")
    for form in FORMS:
        _say(f"[bvp] sphere32 trace={form}")
        op = K.Operator(cfg, K.FP64, cg_rtol=1e-13, gmres_rtol=1e-11, trace=form)
        O.form = form
        xyz, _ = op.points()
        g = KI.exact_u(cfg.solution, xyz[:, 0], xyz[:, 1], xyz[:, 2])
        f = lambda x, y, z: KI.body_force(cfg.solution, x, y, z, cfg.mu, cfg.lam)
        phi, u, p = op.solve_bvp(g, f)
        it = op.last_info["gmres_iters"]
        phio, uo, po, ito, _ = O.solve_bvp(g, f, tol=1e-11)
        _say(f"   gmres {it} (oracle {ito})")
        _check("phi", phi.cpu().numpy(), phio, 1e-8)
        u1, u2, u3 = op.split_u(u)
        for a, b in zip((u1, u2, u3), uo):
            assert np.abs(a.cpu().numpy() - b).max() < 1e-8 * np.abs(b).max()
        assert abs(it - ito) <= 2


def test_error_paths(K):
    cfg = KI.WORKLOADS["sphere32"].with_N(16)
    op = K.Operator(cfg, K.FP64)
    phi = np.zeros((op.n, 3))
    phi[3, 1] = np.nan
    for call in (op.eval, op.eval_adjoint):
        with pytest.raises(K.KfbiError) as e:
            call(phi)
        assert e.value.status == K.EINVAL
    # the context stays usable after a rejected input
    ok = op.eval(np.ones((op.n, 3))).cpu().numpy()
    assert np.abs(ok - 1.0).max() < 1e-9
    op2 = K.Operator(cfg, K.FP64, cg_maxit=1)
    with pytest.raises(K.KfbiError) as e:
        op2.eval(KI.random_density(op2.n))
    assert e.value.status == K.ENOCONV


def test_512_navier_matches_stored_oracle_sample(K):
    """Navier, lambda = 100 (nu = 0.495), star r = 0.5 + 0.12 sin 5t cos 3p at 512^3, both trace
    forms: the mixed form's K phi (phi = exact velocity) and K^T w (w = random density) against
    the oracle's values on a seeded sample of 4096 control points
    (tests/golden/make_oracle_reference.py star512n --sample 4096 --adjoint --inputs uexact), to
    the mixed form's 1e-6, and the float64 K phi to 1e-10."""
    z, meta = _golden("star512n")
    cfg = KI.WORKLOADS["star512n"]
    idx = z["idx"]
    for form in FORMS:
        _say(f"[512] star512n mixed, trace={form}")
        op = K.Operator(cfg, K.MIXED_FP32, cg_rtol=1e-9, inner_rtol=1e-5, trace=form)
        assert op.n == meta["n_points"]
        xyz, _ = op.points()
        phi = KI.exact_u(cfg.solution, xyz[:, 0], xyz[:, 1], xyz[:, 2])
        _check("K phi (sample)", op.eval(phi).cpu().numpy()[idx], z[f"Kphi_uexact_{form}"], 1e-6)
        _say(f"   info {op.last_info['cg_iters']} cg, {op.last_info['ms_total']:.1f} ms")
        _check("K^T w (sample)", op.eval_adjoint(KI.random_density(op.n)).cpu().numpy()[idx],
               z[f"KTw_random_{form}"], 1e-6)
        del op
        op = K.Operator(cfg, K.FP64, cg_rtol=1e-12, trace=form)
        _check("K phi float64 (sample)", op.eval(phi).cpu().numpy()[idx], z[f"Kphi_uexact_{form}"], 1e-10)
        del op


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("trace", ["average", "interior"])
def test_degenerate_inputs(K, prec, trace):
    """Zero density, zero cotangent and zero Dirichlet data give exact zeros (the mixed
    refinement and GMRES take their zero-norm exits), on a ragged control-point count."""
    import torch
    cfg = KI.WORKLOADS["ellip128"].with_N(32)
    op = K.Operator(cfg, prec, trace=trace)
    z = torch.zeros((op.n, 3), dtype=torch.float64, device="cuda")
    assert op.n % 256 != 0
    assert torch.count_nonzero(op.eval(z)).item() == 0
    assert torch.count_nonzero(op.eval_adjoint(z)).item() == 0
    phi, u, p = op.solve_bvp(z)
    assert torch.count_nonzero(phi).item() == 0 and op.last_info["gmres_iters"] == 0
    assert torch.count_nonzero(u).item() == 0
