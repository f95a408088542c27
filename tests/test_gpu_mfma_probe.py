"""What the gfx950 16x16x4 MFMA instructions compute (GPU; a probe built by
``build()`` from tests/probe/mfma_probe.hip).

FP32 (v_mfma_f32_16x16x4f32): a single product of two full-mantissa FP32
operands equals the FP32 rounding of the exact product, and a K-term tile
product stays within a small multiple of 2^-24 of sum |a_ik b_kj| -- true
FP32 arithmetic, not products of shortened mantissas.  The accumulator
layout is: register q of lane l holds row 4 (l / 16) + q, column l % 16.

FP64 (v_mfma_f64_16x16x4f64): errors at the 2^-53 level, and a different
accumulator layout: register q of lane l holds row 4 q + l / 16.
"""
import ctypes
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "probe", "libmfmaprobe.so")


@pytest.fixture(scope="module")
def probe():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    if not os.path.exists(LIB):
        pytest.fail(f"{LIB} missing: run __graft_entry__.build()")
    L = ctypes.CDLL(LIB)
    for name in ("mfma_probe_f32", "mfma_probe_f64"):
        fn = getattr(L, name)
        fn.restype = ctypes.c_int
        fn.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                       ctypes.c_void_p, ctypes.c_void_p]
    return L, torch


def _run(probe, A, B, dtype):
    L, torch = probe
    dA = torch.as_tensor(A, device="cuda").contiguous()
    dB = torch.as_tensor(B, device="cuda").contiguous()
    out = torch.empty(256, dtype=dA.dtype, device="cuda")
    fn = L.mfma_probe_f32 if dtype == np.float32 else L.mfma_probe_f64
    st = fn(dA.data_ptr(), dB.data_ptr(), A.shape[1], out.data_ptr(),
            torch.cuda.current_stream().cuda_stream)
    assert st == 0
    torch.cuda.synchronize()
    return out.cpu().numpy().reshape(4, 64)


def _unpack(raw, layout):
    """16 x 16 tile from the raw registers: layout 'f32' or 'f64'."""
    C = np.empty((16, 16), dtype=np.float64)
    for q in range(4):
        for lane in range(64):
            r = 4 * (lane // 16) + q if layout == "f32" else 4 * q + lane // 16
            C[r, lane % 16] = raw[q, lane]
    return C


def test_fp32_single_products_are_correctly_rounded(probe):
    rng = np.random.default_rng(11)
    A = np.zeros((16, 4), dtype=np.float32)
    B = np.zeros((4, 16), dtype=np.float32)
    # full 24-bit mantissas: 1 + random 23-bit fractions
    A[:, 0] = (1.0 + rng.integers(1, 2 ** 23, 16) * 2.0 ** -23).astype(np.float32)
    B[0, :] = (1.0 + rng.integers(1, 2 ** 23, 16) * 2.0 ** -23).astype(np.float32)
    C = _unpack(_run(probe, A, B, np.float32), "f32")
    exact = A[:, :1].astype(np.float64) @ B[:1, :].astype(np.float64)
    np.testing.assert_array_equal(C, exact.astype(np.float32).astype(np.float64))
    # the products need all 48 bits: a 10-bit-mantissa product would be off
    assert np.max(np.abs(exact - np.round(exact * 2 ** 10) / 2 ** 10)) > 2.0 ** -20


@pytest.mark.parametrize("K", [4, 64, 256])
def test_fp32_tile_product_error_is_fp32_rounding(probe, K):
    rng = np.random.default_rng(K)
    A = rng.uniform(-1, 1, (16, K)).astype(np.float32)
    B = rng.uniform(-1, 1, (K, 16)).astype(np.float32)
    C = _unpack(_run(probe, A, B, np.float32), "f32")
    A64, B64 = A.astype(np.float64), B.astype(np.float64)
    exact = A64 @ B64
    scale = np.abs(A64) @ np.abs(B64)
    err = np.max(np.abs(C - exact) / scale)
    # K-term FP32 accumulation: within K 2^-24 (a bound), typically ~2^-24
    assert err <= K * 2.0 ** -24, err
    assert err <= 8 * 2.0 ** -24, err
    # the other register layout does not describe the result
    assert np.max(np.abs(_unpack(_run(probe, A, B, np.float32), "f64") - exact) / scale) > 1e-3


def test_fp64_tile_product_and_layout(probe):
    rng = np.random.default_rng(5)
    A = rng.uniform(-1, 1, (16, 64))
    B = rng.uniform(-1, 1, (64, 16))
    C = _unpack(_run(probe, A, B, np.float64), "f64")
    exact = A @ B
    scale = np.abs(A) @ np.abs(B)
    assert np.max(np.abs(C - exact) / scale) <= 64 * 2.0 ** -53
    assert np.max(np.abs(_unpack(_run(probe, A, B, np.float64), "f32") - exact) / scale) > 1e-3
