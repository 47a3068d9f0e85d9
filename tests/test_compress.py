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


@pytest.mark.parametrize("shape", [(130, 3, 50), (64, 4, 64), (257, 2, 170), (1, 4, 4), (128, 3, 256)])
def test_structured_sites_are_right_canonical_and_torch_compression_matches(shape):
    """Large-bond generator: orthonormal rows (sum_i B_i B_i^H = I within
    complex64 rounding), with and without the branch mixers, and the torch
    compressor writes the same bytes as the numpy one."""
    torch = pytest.importorskip("torch")
    for mix in (False, True):
        B = synth.structured_site([1, 2], *shape, mix=mix)
        assert B.dtype == torch.complex64 and tuple(B.shape) == shape
        assert synth.canonical_error(B.numpy().astype(np.complex128)) < 1e-6
    for kind in ("c64", "cf16", "cf8"):
        assert np.array_equal(synth.compress_site(B.numpy(), kind), synth.compress_site_torch(B, kind).numpy()), kind


@pytest.mark.parametrize("shape", [(64, 4, 64), (128, 3, 256), (256, 6, 256), (32, 4, 64)])
def test_structured_sites_hidden_markov_weights(shape):
    """Without mixers, a left vector inside bond block a has conditionals
    T[a][.] = c_{(a+.) mod d}^2 exactly (c_i^2 ~ exp(-i)), whatever the vector,
    and branch i moves it into block (a+i) mod nb; with one block (small
    bonds) the weights are the plain profile c_i^2.  With mixers the weights
    depend on the vector itself, not only on its block."""
    torch = pytest.importorskip("torch")
    chi_l, d, chi_r = shape
    nb = synth.structured_blocks(chi_l, chi_r)
    assert nb == (4 if chi_l >= 64 else 1)
    B = synth.structured_site([3, 9], *shape, mix=False).numpy().astype(np.complex128)
    Bm = synth.structured_site([3, 9], *shape, mix=True).numpy().astype(np.complex128)
    T = synth.structured_weights(d, nb)
    c2 = np.exp(-np.arange(d)) / np.sum(np.exp(-np.arange(d)))
    assert np.allclose(T[0], c2) and np.allclose(T.sum(axis=1), 1.0)
    rng = np.random.default_rng(1)
    bl, br = chi_l // nb, chi_r // nb
    pm = []
    for a in range(nb):
        for _ in range(3):
            x = np.zeros(chi_l, complex)
            x[a * bl:(a + 1) * bl] = rng.standard_normal(bl) + 1j * rng.standard_normal(bl)
            x /= np.linalg.norm(x)
            W = np.einsum("l,lir->ir", x, B)
            q = np.sum(np.abs(W) ** 2, axis=1)
            assert np.allclose(q / q.sum(), T[a], atol=1e-6)
            for i in range(d):  # branch i lands in right block (a+i) mod nb only
                b = (a + i) % nb
                outside = np.delete(W[i], np.arange(b * br, (b + 1) * br))
                assert np.all(np.abs(outside) < 1e-6)
            Wm = np.einsum("l,lir->ir", x, Bm)
            qm = np.sum(np.abs(Wm) ** 2, axis=1)
            pm.append(qm / qm.sum())
    pm = np.array(pm)
    assert np.max(pm.max(axis=0) - pm.min(axis=0)) > 1e-2
