"""Parity of the planar complex MFMA product (FP32 and FP64) with NumPy's
complex128 product of the same (rounded) operands.  Several tiles plus a
ragged zero-padded edge per size; Hermitian-lower launches leave the upper
tiles untouched."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2403_07042_amd")
from paper_2403_07042_amd import _lib as L  # noqa: E402


def dev(x, dtype):
    return torch.from_numpy(np.ascontiguousarray(x).astype(dtype)).cuda()


def planes(rng, ld, n, dtype):
    z = np.zeros((ld, ld), np.complex128)
    z[:n, :n] = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    re = z.real.astype(dtype)
    im = z.imag.astype(dtype)
    return re, im


def run(prec, ld, n, tile, conj_m, lower, alpha, beta, seed=0, conj_a=False, b_rows=False):
    dtype = np.float64 if prec == L.FP64 else np.float32
    rng = np.random.default_rng(seed)
    ar, ai = planes(rng, ld, n, dtype)
    mr, mi = planes(rng, ld, n, dtype)
    xr, xi = planes(rng, ld, n, dtype)
    sentinel = 7.0
    cr = np.full((ld, ld), sentinel, dtype)
    ci = np.full((ld, ld), sentinel, dtype)
    t = [dev(v, dtype) for v in (ar, ai, mr, mi, xr, xi, cr, ci)]
    p = [ctypes.c_void_p(v.data_ptr()) for v in t]
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    print(f"cgemm prec={prec} ld={ld} n={n} tile={tile} conj_a={conj_a} conj_b={conj_m} "
          f"b_rows={b_rows} lower={lower}", flush=True)
    L.check(L.load().qme_cgemm(prec, ld, *p, alpha, beta, int(conj_a), int(conj_m), int(b_rows),
                               int(lower), tile, s))
    torch.cuda.synchronize()
    got = t[6].cpu().numpy().astype(np.float64) + 1j * t[7].cpu().numpy().astype(np.float64)
    a = ar.astype(np.float64) + 1j * ai
    m = mr.astype(np.float64) + 1j * mi
    x = xr.astype(np.float64) + 1j * xi
    opa = a.conj() if conj_a else a
    opb = m if b_rows else m.T
    if conj_m:
        opb = opb.conj()
    ref = alpha * (opa @ opb) + beta * x
    mask = np.ones((ld, ld), bool)
    if lower:
        bi = np.arange(ld)[:, None] // tile
        bj = np.arange(ld)[None, :] // tile
        mask = bi >= bj
        assert np.all(got[~mask] == sentinel + 1j * sentinel)
    err = np.abs(got - ref)[mask].max()
    scale = np.abs(ref[mask]).max()
    return err, scale


@pytest.mark.parametrize("ld,n,tile", [(64, 64, 64), (192, 150, 64), (256, 256, 128),
                                       (512, 500, 128), (384, 333, 64),
                                       (32, 32, 32), (96, 70, 32), (320, 301, 32)])
@pytest.mark.parametrize("conj_m", [True, False])
@pytest.mark.parametrize("lower", [False, True])
def test_cgemm_fp32(ld, n, tile, conj_m, lower):
    err, scale = run(L.FP32, ld, n, tile, conj_m, lower, 1.0, 1.0)
    # FP32 accumulation of n products of unit-variance entries: rounding grows
    # at most linearly in n (typically as sqrt(n)) on results of size ~sqrt(n)
    assert err < 1e-6 * n + 1e-5


@pytest.mark.parametrize("ld,n,tile", [(32, 32, 32), (96, 70, 32), (128, 128, 64),
                                       (320, 300, 64)])
@pytest.mark.parametrize("conj_m", [True, False])
@pytest.mark.parametrize("lower", [False, True])
def test_cgemm_fp64(ld, n, tile, conj_m, lower):
    err, scale = run(L.FP64, ld, n, tile, conj_m, lower, 1.0, 1.0)
    assert err < 1e-13 * scale


def test_cgemm_alpha_beta():
    err, scale = run(L.FP64, 128, 100, 64, True, False, -0.5, 2.0)
    assert err < 1e-13 * scale
    err, scale = run(L.FP32, 128, 100, 64, False, False, 3.0, 0.0)
    assert err < 3.0 * (1e-6 * 100 + 1e-5)


@pytest.mark.parametrize("prec,ld,n,tile", [(L.FP32, 192, 150, 64), (L.FP32, 256, 256, 128),
                                            (L.FP64, 96, 70, 32), (L.FP64, 128, 128, 64)])
@pytest.mark.parametrize("conj_a,conj_b,b_rows", [(True, True, False), (False, False, True),
                                                  (True, False, True), (False, True, True)])
def test_cgemm_operand_forms(prec, ld, n, tile, conj_a, conj_b, b_rows):
    err, scale = run(prec, ld, n, tile, conj_b, False, 1.0, 1.0, conj_a=conj_a, b_rows=b_rows)
    if prec == L.FP32:
        assert err < 1e-6 * n + 1e-5
    else:
        assert err < 1e-13 * scale


def test_cgemm_accumulate_in_place():
    """C = A B + C (the adjoint's G accumulation): X and C are one buffer."""
    rng = np.random.default_rng(4)
    ld, n = 128, 100
    ar, ai = planes(rng, ld, n, np.float32)
    br, bi = planes(rng, ld, n, np.float32)
    cr, ci = planes(rng, ld, n, np.float32)
    t = [dev(v, np.float32) for v in (ar, ai, br, bi, cr, ci)]
    p = [ctypes.c_void_p(v.data_ptr()) for v in t]
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    L.check(L.load().qme_cgemm(L.FP32, ld, p[0], p[1], p[2], p[3], p[4], p[5], p[4], p[5],
                               1.0, 1.0, 0, 0, 1, 0, 64, s))
    torch.cuda.synchronize()
    got = t[4].cpu().numpy() + 1j * t[5].cpu().numpy()
    a = ar + 1j * ai.astype(np.float64)
    b = br + 1j * bi.astype(np.float64)
    ref = a @ b + (cr + 1j * ci.astype(np.float64))
    assert np.abs(got - ref).max() < 1e-6 * n + 1e-5


@pytest.mark.parametrize("ld,n", [(64, 64), (192, 150), (512, 500)])
@pytest.mark.parametrize("conj_a,conj_b,lower", [(False, True, False), (False, True, True),
                                                 (True, True, False), (False, False, True),
                                                 (True, False, False), (False, False, False),
                                                 (True, True, True), (True, False, True)])
def test_cgemm_bf16x3(ld, n, conj_a, conj_b, lower):
    """Split-bf16 products of FP32 operands: accurate to FP32 rounding."""
    err, scale = run(L.BF16X3, ld, n, 64, conj_b, lower, 1.0, 1.0, conj_a=conj_a)
    assert err < 1e-6 * n + 1e-5
