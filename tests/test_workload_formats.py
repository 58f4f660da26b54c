"""CPU tests of the storage formats of the synthetic inputs (not search
arithmetic): the FP8 e4m3 code table and nearest-even encoder, complex32."""
import numpy as np

from paper_1801_02391_amd import workloads as W


def test_e4m3_table_known_values():
    """OCP e4m3fn: max 448 (0x7e), min normal 2^-6 (0x08), min subnormal
    2^-9 (0x01), NaN at 0x7f, sign bit 0x80."""
    t = W.E4M3
    assert t[0x7E] == 448.0 and t[0x08] == 2.0 ** -6 and t[0x01] == 2.0 ** -9
    assert np.isnan(t[0x7F]) and np.isnan(t[0xFF]) and t[0x80] == 0.0 and t[0xFE] == -448.0
    assert np.all(np.diff(t[:127]) > 0)


def test_e4m3_encode_is_nearest_and_round_trips():
    rng = np.random.default_rng(0)
    V = (rng.standard_normal((2, 3, 4, 50)) + 1j * rng.standard_normal((2, 3, 4, 50))).astype(np.complex64)
    codes, scale = W.to_e4m3(V)
    D = W.from_e4m3(codes, scale)
    # every representable value round-trips exactly
    again, s2 = W.to_e4m3(D)
    assert np.array_equal(W.from_e4m3(again, s2), D)
    # nearest: error at most half the local spacing (relative 2^-4 for normals)
    x = V.real / scale[..., None]
    d = D.real / scale[..., None]
    assert np.all(np.abs(x - d) <= np.maximum(np.abs(x) * 2.0 ** -4, 2.0 ** -10) + 1e-6)
    # the per-channel maximum maps to 448 exactly
    amax = np.maximum(np.abs(V.real), np.abs(V.imag)).max(axis=-1)
    dm = np.maximum(np.abs(D.real), np.abs(D.imag)).max(axis=-1)
    assert np.allclose(dm, amax, rtol=1e-6)


def test_complex32_round_trip():
    rng = np.random.default_rng(1)
    V = (rng.standard_normal((2, 5)) + 1j * rng.standard_normal((2, 5))).astype(np.complex64)
    H = W.to_complex32(V)
    assert H.dtype == np.float16 and H.shape == (2, 5, 2)
    assert np.allclose(W.from_complex32(H), V, rtol=1e-3, atol=1e-3)
