"""GPU checks of the transform engine through the C ABI (kfbi_apply_pass): every one-dimensional
pass of the FFT-based Poisson solver (Sec. 4.2, item ii) -- orthonormal DCT-II, DST-II, DCT-III,
DST-III of length N and the DST-I on the interior indices of the face-normal axis -- along each
axis against the definitions (scipy.fft's orthonormal transforms), in float64 (1e-13) and in the
mixed form's float32 (1e-6); and the matrix-core DCT-II along x (split-bfloat16 products,
float32 accumulation) against the same definition.  Errors in relative l2 and relative max.
"""
import sys

import numpy as np
import pytest
import scipy.fft as sfft

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


def _reference(kind, f, axis):
    if kind == 0:
        return sfft.dct(f, 2, axis=axis, norm="ortho")
    if kind == 1:
        return sfft.dst(f, 2, axis=axis, norm="ortho")
    if kind == 2:
        return sfft.dct(f, 3, axis=axis, norm="ortho")
    if kind == 3:
        return sfft.dst(f, 3, axis=axis, norm="ortho")
    # DST-I on indices 1..N-1 (index 0 is the box face, zero in the result)
    out = np.zeros_like(f)
    sl = [slice(None)] * 3
    sl[axis] = slice(1, None)
    out[tuple(sl)] = sfft.dst(f[tuple(sl)], 1, axis=axis, norm="ortho")
    return out


def _errs(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b)), float(np.abs(a - b).max() / np.abs(b).max())


@pytest.mark.parametrize("prec,N,tol", [(0, 32, 1e-13), (1, 64, 1e-6)])
def test_every_pass_matches_its_definition(K, prec, N, tol):
    cfg = KI.WORKLOADS["sphere32"].with_N(N)
    op = K.Operator(cfg, prec)
    f = np.random.default_rng(21).standard_normal((N, N, N))
    worst = 0.0
    for kind in range(5):
        for axis in range(3):
            g = op.apply_pass(kind, axis, f).cpu().numpy()
            l2, mx = _errs(g, _reference(kind, f, axis))
            worst = max(worst, l2, mx)
            assert l2 < tol and mx < tol, (kind, axis, l2, mx)
    _say(f"[transforms prec={prec} N={N}] worst rel error over 5 kinds x 3 axes: {worst:.2e}")


@pytest.mark.parametrize("N", [128, 256])
def test_matrix_core_dct2_matches_its_definition(K, N):
    """Split-bfloat16 products: each product keeps hi*hi + hi*lo + lo*hi of the two bfloat16
    pairs, dropping lo*lo (2^-16 of it) and the roundings of the lo parts (2^-17 each), so one
    product is off by at most ~3 * 2^-17 = 2.3e-5 of its size; over the N terms of a row the
    error is at most 2.3e-5 sum_x |C_kx f_x|, which for these random fields is below ~1e-4 of
    max |Y| (and its l2 average far smaller).  float32 accumulation adds ~N 2^-24."""
    cfg = KI.WORKLOADS["sphere32"].with_N(N)
    op = K.Operator(cfg, K.MIXED_FP32)
    f = np.random.default_rng(22).standard_normal((N, N, N))
    g = op.apply_pass(K.K_GEMM_X, 0, f).cpu().numpy()
    ref = _reference(0, f, 0)
    l2, mx = _errs(g, ref)
    r = op.apply_pass(0, 0, f).cpu().numpy()
    l2r, mxr = _errs(r, ref)
    _say(f"[matrix-core DCT-II N={N}] rel l2 {l2:.2e} rel max {mx:.2e} (radix float32: {l2r:.2e}, {mxr:.2e})")
    assert l2 < 1e-5 and mx < 1e-4
    with pytest.raises(K.KfbiError) as e:  # along x only
        op.apply_pass(K.K_GEMM_X, 1, f)
    assert e.value.status == K.EINVAL


def test_matrix_core_pass_needs_a_float32_context(K):
    op = K.Operator(KI.WORKLOADS["sphere32"].with_N(128), K.FP64)
    with pytest.raises(K.KfbiError) as e:
        op.apply_pass(K.K_GEMM_X, 0, np.zeros((128,) * 3))
    assert e.value.status == K.EINVAL


def test_passes_at_512(K):
    """At N = 512 the length-512 transforms take three radix-8 passes in 512-thread blocks and the
    length-1024 DST-I two radix-32 passes; both precisions against the definitions, along the
    contiguous axis (tile staged in LDS), the strided axis read directly and the persistent
    pipelined path (inverse kinds along x and y)."""
    N = 512
    f = np.random.default_rng(23).standard_normal((N, N, N))
    cases = [(0, 2), (1, 0), (2, 1), (3, 2), (3, 0), (4, 1)]
    refs = {c: _reference(c[0], f, c[1]) for c in cases}
    for prec, tol in ((K.FP64, 1e-13), (K.MIXED_FP32, 1e-6)):
        op = K.Operator(KI.WORKLOADS["sphere32"].with_N(N), prec)
        for kind, axis in cases:
            _say(f"[transforms N=512 prec={prec}] kind {kind} axis {axis}")
            g = op.apply_pass(kind, axis, f).cpu().numpy()
            l2, mx = _errs(g, refs[(kind, axis)])
            _say(f"    rel l2 {l2:.2e} rel max {mx:.2e}")
            assert l2 < tol and mx < tol, (prec, kind, axis, l2, mx)
            del g
        del op
