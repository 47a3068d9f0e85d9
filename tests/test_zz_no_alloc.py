"""mps_sample_noalloc (the allocation-free entry point) against mps_sample.

Both entry points run the same kernels on the same inputs, so outcomes and
logp must agree bit for bit; each case makes two calls in a row on one
handle, the second with a smaller input, so that the fixed scratch array is
reused with the first call's contents still in it.
"""
import numpy as np
import pytest

from paper_2512_20064_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def mpsmod():
    from paper_2512_20064_amd import mps
    mps.load()
    assert torch.cuda.is_available(), "no GPU visible"
    return mps


def _chain(seed, M, d, chi_max):
    dl = [d] * M
    return synth.to_c64(synth.random_mps(seed, dl, synth.ramp_bonds(dl, chi_max)))


def _call(mps, h, entry, dev_tensors, N, seed, n_offset=0):
    chi = [int(dev_tensors[0].shape[0])] + [int(t.shape[2]) for t in dev_tensors]
    d = [int(t.shape[1]) for t in dev_tensors]
    M = len(dev_tensors)
    outc = torch.full((N, M), -7, dtype=torch.int32, device="cuda")
    logp = torch.full((N,), float("nan"), dtype=torch.float64, device="cuda")
    fn = mps.mps_sample_noalloc if entry == "noalloc" else mps.mps_sample
    rc = fn(h, [t.data_ptr() for t in dev_tensors], mps.MPS_C64, chi, d, M, N, n_offset, seed,
            outc.data_ptr(), logp.data_ptr())
    torch.cuda.synchronize()
    assert rc == 0, (entry, rc, mps.mps_last_error())
    return outc.cpu().numpy(), logp.cpu().numpy(), mps.mps_get_stats(h)


# (form, fused_small, first call (seed, M, d, chi, N), second call, smaller)
CASES = [
    ("fp32", 1, (3, 20, 4, 64, 3000), (4, 12, 3, 48, 700)),
    ("fp32", 0, (5, 24, 4, 32, 4096), (6, 10, 2, 16, 333)),      # persistent small-bond kernel
    ("bf16x3", 1, (7, 20, 4, 64, 3000), (8, 12, 4, 40, 900)),
    ("fp16x3", 1, (9, 16, 3, 96, 2048), (10, 9, 2, 64, 257)),
    ("fp16f8", 1, (13, 14, 4, 128, 2048), (14, 9, 3, 64, 300)),
    ("fp16f6", 1, (15, 14, 4, 128, 2048), (16, 9, 3, 64, 300)),
]


@pytest.mark.parametrize("form,fused,first,second", CASES)
def test_noalloc_matches_sample(mpsmod, form, fused, first, second):
    from tests.parity_util import upload
    mps = mpsmod
    opt = mps.mps_options_init()
    opt.precision = mps.PRECISIONS[form]
    opt.fused_small = fused
    h = mps.mps_create(0, opt)
    try:
        for seed, M, d, chi, N in (first, second):
            _say(f"noalloc {form} fused_small={fused} seed={seed} M={M} d={d} chi={chi} N={N}")
            dev = upload(_chain(seed, M, d, chi))
            o_ref, l_ref, _ = _call(mps, h, "sample", dev, N, 1000 + seed, n_offset=17)
            o_na, l_na, st = _call(mps, h, "noalloc", dev, N, 1000 + seed, n_offset=17)
            assert (o_ref >= 0).all()
            np.testing.assert_array_equal(o_na, o_ref)
            np.testing.assert_array_equal(l_na.view(np.uint64), l_ref.view(np.uint64))
            assert 0 < st.scratch_bytes <= mps.NOALLOC_SCRATCH_BYTES
    finally:
        mps.mps_destroy(h)


def test_noalloc_chunks_inside_the_fixed_array(mpsmod):
    """A bond-1024 chain in bf16 hi+lo needs ~40 KB per sample plus a 64 MB
    packed site tensor: the fixed array holds only a few thousand samples per
    chunk, and the chunked call still gives mps_sample's bits (one chunk)."""
    from tests.parity_util import upload
    mps = mpsmod
    opt = mps.mps_options_init()
    opt.precision = mps.MPS_BF16X3
    h = mps.mps_create(0, opt)
    try:
        for seed, M, N in ((11, 12, 12000), (12, 11, 5000)):
            _say(f"noalloc chunked bf16x3 seed={seed} M={M} d=4 chi=1024 N={N}")
            dev = upload(_chain(seed, M, 4, 1024))
            o_ref, l_ref, st_ref = _call(mps, h, "sample", dev, N, 2000 + seed)
            o_na, l_na, st = _call(mps, h, "noalloc", dev, N, 2000 + seed)
            assert st_ref.n_chunk == N
            assert st.n_chunk < N
            np.testing.assert_array_equal(o_na, o_ref)
            np.testing.assert_array_equal(l_na.view(np.uint64), l_ref.view(np.uint64))
    finally:
        mps.mps_destroy(h)
