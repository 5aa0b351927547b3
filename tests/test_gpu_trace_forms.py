"""GMRES iteration counts of the two trace forms of K (the average form, 1/2 phi + mean of the
two one-sided limits with the fitted jump value at the control point, and the interior form,
the literal Sec. 4.4 reading).  The parity of both forms against the oracle (evaluation,
transpose, BVP) is in test_gpu_parity.py.
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
