"""Stored forms of site tensors (Section 3.3.2: tensors kept and moved in low
precision): the E4M3 and binary16 encodings of the input generator and the
oracle's decoder, pinned against their definitions and an independent
library conversion (torch's float8_e4m3fn and numpy's float16)."""
import numpy as np
import pytest

from oracle.sampler import _e4m3_value, decode_site
from paper_2512_20064_amd import synth


def test_e4m3_values_follow_the_format_definition():
    v = _e4m3_value(np.arange(256))
    assert v[0x00] == 0.0 and v[0x38] == 1.0 and v[0xB8] == -1.0
    assert v[0x7E] == 448.0 and v[0xFE] == -448.0          # largest finite
    assert v[0x08] == 2.0 ** -6                             # smallest normal
    assert v[0x01] == 2.0 ** -9 and v[0x07] == 7 * 2.0 ** -9  # subnormals
    assert v[0x39] == 1.125                                 # 3-bit mantissa step at 1
    assert np.isnan(v[0x7F]) and np.isnan(v[0xFF])
    assert np.isnan(v).sum() == 2                           # no infinities, two NaNs
    fin = v[:0x7F]
    assert np.all(np.diff(fin) > 0)                         # codes 0..0x7E increase


def test_e4m3_values_match_torch_and_generator_table():
    torch = pytest.importorskip("torch")
    codes = np.arange(256, dtype=np.uint8)
    t = torch.from_numpy(codes).view(torch.float8_e4m3fn).to(torch.float64).numpy()
    v = _e4m3_value(codes)
    nan = np.isnan(v)
    assert np.array_equal(np.isnan(t), nan)
    assert np.array_equal(t[~nan], v[~nan])
    assert np.array_equal(synth.E4M3_VALUES[~nan], v[~nan])


def test_e4m3_encoder_rounds_to_nearest_even_like_torch():
    torch = pytest.importorskip("torch")
    pos = _e4m3_value(np.arange(0x7F))
    mids = (pos[:-1] + pos[1:]) / 2                         # exact ties
    x = np.concatenate([mids, -mids, np.random.default_rng(0).uniform(-448, 448, 20000),
                        np.random.default_rng(1).uniform(-0.02, 0.02, 5000)])
    ours = synth.encode_e4m3(x)
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    assert np.array_equal(ours, ref)
    # ties go to the even mantissa
    tie = synth.encode_e4m3(mids)
    assert np.all((tie & 1) == 0)


def test_e4m3_round_trip_of_every_finite_code():
    codes = np.array([c for c in range(256) if c not in (0x7F, 0xFF, 0x80)])
    assert np.array_equal(synth.encode_e4m3(_e4m3_value(codes)), codes)
    assert synth.encode_e4m3(np.array([1e6, -1e6])).tolist() == [0x7E, 0xFE]  # saturates


def _site(seed, shape):
    rng = np.random.default_rng(seed)
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex64) * 0.1


@pytest.mark.parametrize("shape", [(130, 3, 50), (1, 4, 4), (128, 1, 128), (257, 2, 70)])
def test_cf8_blocks_scales_and_error_bound(shape):
    A = _site(3, shape)
    raw = synth.compress_site(A, "cf8")
    chi_l, d, chi_r = shape
    assert raw.size == synth.compressed_bytes(chi_l, d, chi_r, "cf8")
    n = chi_l * d * chi_r
    off = -(-2 * n // 256) * 256
    nbr, nbc = -(-chi_l // 128), -(-(d * chi_r) // 128)
    assert raw.size == off + 4 * nbr * nbc
    scales = raw[off:].view(np.float32).reshape(nbr, nbc)
    mat = A.reshape(chi_l, d * chi_r)
    for bi in range(nbr):
        for bj in range(nbc):
            blk = mat[bi * 128:(bi + 1) * 128, bj * 128:(bj + 1) * 128]
            amax = float(max(np.abs(blk.real).max(), np.abs(blk.imag).max()))
            # the smallest power of two that brings the block maximum to <= 448
            m, e = np.frexp(float(scales[bi, bj]))
            assert m == 0.5 and 224.0 < amax / float(scales[bi, bj]) <= 448.0
    dec = decode_site(raw, shape, "cf8").reshape(chi_l, d * chi_r)
    sc = np.repeat(np.repeat(scales.astype(np.float64), 128, 0), 128, 1)[:chi_l, :d * chi_r]
    for part in (np.real, np.imag):
        x = part(mat).astype(np.float64)
        err = np.abs(part(dec) - x)
        # round to nearest: half a mantissa step (2^-4 relative) for normals,
        # half the subnormal step (2^-10 of the scale) below 2^-6 of the scale
        assert np.all(err <= np.maximum(np.abs(x) * 2.0 ** -4, sc * 2.0 ** -10) * (1 + 1e-6))
    # every decoded value is exact in binary16 (power-of-two scales with
    # exponents in [-15, 7], E4M3 codes of at most 4 significant bits)
    for part in (np.real, np.imag):
        v = part(dec)
        assert np.array_equal(v.astype(np.float16).astype(np.float64), v)


def test_fp8_block_scale_edges():
    assert synth.fp8_block_scale(0.0) == 1.0
    assert synth.fp8_block_scale(448.0) == 1.0            # exactly 448 fits
    assert synth.fp8_block_scale(448.5) == 2.0
    assert synth.fp8_block_scale(0.875) == 2.0 ** -9     # 0.875 / 2^-9 = 448
    assert synth.fp8_block_scale(0.876) == 2.0 ** -8
    assert synth.fp8_block_scale(1e-3) == 2.0 ** -18     # 1e-3 / 2^-18 = 262.1


def test_cf16_is_numpy_binary16_and_c64_is_identity():
    A = _site(5, (20, 4, 33))
    dec = decode_site(synth.compress_site(A, "cf16"), A.shape, "cf16")
    assert np.array_equal(dec.real, A.real.astype(np.float16).astype(np.float64))
    assert np.array_equal(dec.imag, A.imag.astype(np.float16).astype(np.float64))
    assert np.array_equal(decode_site(synth.compress_site(A, "c64"), A.shape, "c64"), A.astype(np.complex128))
    assert synth.compressed_bytes(20, 4, 33, "cf16") == 4 * 20 * 4 * 33


@pytest.mark.parametrize("shape", [(130, 3, 50), (64, 4, 64), (257, 2, 170), (1, 4, 4)])
def test_structured_sites_are_right_canonical_and_torch_compression_matches(shape):
    """Large-bond generator: orthonormal rows (sum_i B_i B_i^H = I within
    complex64 rounding), branch weights c_i^2 ~ exp(-i) where chi_l <= chi_r,
    and the torch compressor writes the same bytes as the numpy one."""
    torch = pytest.importorskip("torch")
    B = synth.structured_site([1, 2], *shape)
    assert B.dtype == torch.complex64 and tuple(B.shape) == shape
    Bn = B.numpy().astype(np.complex128)
    assert synth.canonical_error(Bn) < 1e-6
    chi_l, d, chi_r = shape
    if chi_l <= chi_r:
        w = np.array([np.sum(np.abs(Bn[:, i, :]) ** 2) / chi_l for i in range(d)])
        c = np.exp(-np.arange(d)) / np.sum(np.exp(-np.arange(d)))
        assert np.allclose(w, c, atol=1e-6)
    for kind in ("c64", "cf16", "cf8"):
        assert np.array_equal(synth.compress_site(B.numpy(), kind), synth.compress_site_torch(B, kind).numpy()), kind
