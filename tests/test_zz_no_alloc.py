"""GPU test of kfbi_eval_noalloc, the evaluation for callers that cannot allocate: its work
buffers come from the library's static device scratch.  Through the C ABI it must give what
kfbi_eval gives on the same context (the same kernels on the same inputs: to the parity
tolerance of the precision, float64 1e-10 and mixed 1e-6, in l2 and max), on two calls in a
row with the second on a smaller context (the scratch keeps the first call's contents), and
leave the context's own evaluation unchanged.  A context whose evaluation needs more than the
scratch holds is rejected with EINVAL.
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


def _cmp(a, b):
    a, b = a.cpu().numpy(), b.cpu().numpy()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b)), float(np.abs(a - b).max() / np.abs(b).max())


@pytest.mark.parametrize("prec,tol", [(0, 1e-10), (1, 1e-6)])
def test_noalloc_matches_eval_on_shrinking_inputs(K, prec, tol):
    import torch
    for name, N in (("star128", 64), ("sphere32", 32)):
        cfg = KI.WORKLOADS[name].with_N(N)
        for trace in ("average", "interior"):
            _say(f"[noalloc] {name} N={N} precision={prec} trace={trace}")
            op = K.Operator(cfg, prec, trace=trace)
            phi = torch.as_tensor(KI.random_density(op.n, seed=5), device="cuda")
            ref = op.eval(phi)
            got = op.eval_noalloc(phi)
            l2, mx = _cmp(got, ref)
            _say(f"   noalloc vs eval: rel l2 {l2:.2e} rel max {mx:.2e} (cg {op.last_info['cg_iters']})")
            assert l2 < tol and mx < tol
            again = op.eval(phi)
            l2, mx = _cmp(again, ref)
            assert l2 < 1e-12 and mx < 1e-12, "the context's own evaluation changed"
            del op


def test_noalloc_rejects_contexts_beyond_the_scratch(K):
    cfg = KI.WORKLOADS["star128"]  # N = 128: the evaluation needs more than 64 MiB
    op = K.Operator(cfg, K.MIXED_FP32)
    with pytest.raises(K.KfbiError) as e:
        op.eval_noalloc(np.zeros((op.n, 3)))
    assert e.value.status == K.EINVAL
    _say(f"[noalloc] N=128 rejected: {e.value}")


def test_noalloc_reports_non_finite_input(K):
    cfg = KI.WORKLOADS["sphere32"].with_N(16)
    op = K.Operator(cfg, K.FP64)
    phi = np.zeros((op.n, 3))
    phi[0, 0] = np.inf
    with pytest.raises(K.KfbiError) as e:
        op.eval_noalloc(phi)
    assert e.value.status == K.EINVAL
    out = op.eval_noalloc(np.ones((op.n, 3))).cpu().numpy()
    assert np.abs(out - 1.0).max() < 1e-9
