"""Staged site tensors: pinned host memory and compressed storage
(complex-fp16, complex-fp8 with 128 x 128 block scales), copied on a side
stream and expanded on the device (Section 3.3.2; Section 3.1: every site is
applied to all samples of the call before the next site)."""
import numpy as np
import pytest

from oracle.sampler import _e4m3_value
from paper_2512_20064_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _chain(M=10, d=3, chi=40, seed=31):
    dl = [d] * M
    return synth.to_c64(synth.random_mps(seed, dl, synth.ramp_bonds(dl, chi)))


def _expand_f32(raw, shape, kind):
    """complex64 values the device expansion produces: binary16 -> FP32 is
    exact; an fp8 entry is its code's value times its block scale, one FP32
    product."""
    chi_l, d, chi_r = shape
    n = chi_l * d * chi_r
    if kind == "c64":
        return raw[:8 * n].view(np.complex64).reshape(shape).copy()
    if kind == "cf16":
        ri = raw[:4 * n].view(np.float16).astype(np.float32).reshape(n, 2)
        return (ri[:, 0] + 1j * ri[:, 1]).astype(np.complex64).reshape(shape)
    codes = raw[:2 * n].reshape(chi_l, d * chi_r, 2)
    off = -(-2 * n // 256) * 256
    nbr, nbc = -(-chi_l // 128), -(-(d * chi_r) // 128)
    sc = raw[off:off + 4 * nbr * nbc].view(np.float32).reshape(nbr, nbc)
    sc = np.repeat(np.repeat(sc, 128, 0), 128, 1)[:chi_l, :d * chi_r]
    re = _e4m3_value(codes[..., 0]).astype(np.float32) * sc
    im = _e4m3_value(codes[..., 1]).astype(np.float32) * sc
    out = np.empty((chi_l, d * chi_r), dtype=np.complex64)
    out.real, out.imag = re, im
    return out.reshape(shape)


def _stored(tensors, kind, where):
    """uint8 torch tensors per site: where is 'device', 'host' (pinned) or
    'mixed' (even sites pinned host, odd sites device)."""
    out = []
    for k, A in enumerate(tensors):
        raw = torch.from_numpy(synth.compress_site(A, kind))
        on_host = where == "host" or (where == "mixed" and k % 2 == 0)
        out.append(raw.pin_memory() if on_host else raw.to("cuda"))
    return out


CASES = [("c64", "host"), ("cf16", "device"), ("cf16", "host"), ("cf8", "device"), ("cf8", "mixed")]


@pytest.mark.parametrize("form", ["fp32", "bf16x3", "fp16x3", "fp16f8", "fp16f6"])
@pytest.mark.parametrize("kind,where", CASES)
def test_staged_equals_resident_expanded_tensor(form, kind, where):
    """A staged call is bit-identical to a device-resident complex64 call on
    the expanded tensors (only where the bytes come from differs), across
    4 chunks with a ragged tail."""
    from paper_2512_20064_amd import mps
    from tests.parity_util import upload
    print(f"[gpu-case] staged {kind}/{where} vs resident {form}", flush=True)
    ch = _chain()
    shapes = [t.shape for t in ch]
    raws = [synth.compress_site(t, kind) for t in ch]
    expanded = [_expand_f32(r, s, kind) for r, s in zip(raws, shapes)]
    N, seed = 1000, 606
    # staged sites always take the per-site launches; so does the resident
    # reference here (bonds <= 32 would otherwise use the small-bond kernel)
    s = mps.Sampler(0, n_chunk=256, precision=form, fused_small=False)
    ref = s.sample(upload(expanded), N, seed)
    got = s.sample_stored(_stored(ch, kind, where), shapes, kind, N, seed)
    torch.cuda.synchronize()
    st = s.stats
    s.close()
    assert torch.equal(got["outcomes"], ref["outcomes"])
    assert torch.equal(got["logp"], ref["logp"])
    M = len(ch)
    assert st.staged_sites == M
    assert st.contract_launches == 4 * M
    if form != "fp32":
        assert st.pack_launches == M  # one packing per site, shared by the chunks
    nb_host = sum(r.size for k, r in enumerate(raws) if where == "host" or (where == "mixed" and k % 2 == 0))
    assert st.h2d_bytes == nb_host


def _fp8_shift(raw, shape):
    """The power of two t that the library applies to a complex-fp8 site with
    power-of-two block scales (every exponent brought into [-15, 7]), restated
    from its documented rule."""
    chi_l, d, chi_r = shape
    n = chi_l * d * chi_r
    off = -(-2 * n // 256) * 256
    nb = -(-chi_l // 128) * -(-(d * chi_r) // 128)
    sc = raw[off:off + 4 * nb].view(np.float32).astype(np.float64)
    m, e = np.frexp(sc)
    assert np.all(m == 0.5)  # powers of two
    e = e - 1
    assert e.max() - e.min() <= 22
    return -15 - e.min() if e.min() < -15 else (7 - e.max() if e.max() > 7 else 0)


def test_small_magnitude_fp8_sites_in_the_two_product_form():
    """Complex-fp8 sites whose block scales lie below 2^-15 (entries of order
    2^-15 here) are expanded times 2^t so that they sit on the binary16 grid
    and take the two-product fp16 contraction: the staged call is
    bit-identical to a resident fp16x3 call on the expanded tensors times
    2^t, and its draws and conditional probabilities match the oracle on the
    unshifted values (they are invariant to a per-site power of two)."""
    from paper_2512_20064_amd import mps
    from tests.parity_util import compare, upload, EPS_LOWP
    print("[gpu-case] small-magnitude cf8 host sites, fp16x3, shifted expansion", flush=True)
    ch = [np.ascontiguousarray(t * np.float32(2.0 ** -12)) for t in _chain()]
    shapes = [t.shape for t in ch]
    raws = [synth.compress_site(t, "cf8") for t in ch]
    shifts = [_fp8_shift(r, sh) for r, sh in zip(raws, shapes)]
    assert max(shifts) > 0
    expanded = [_expand_f32(r, sh, "cf8") for r, sh in zip(raws, shapes)]
    shifted = [np.ascontiguousarray(x * np.float32(2.0 ** t)) for x, t in zip(expanded, shifts)]
    N, seed = 1000, 707
    s = mps.Sampler(0, n_chunk=256, precision="fp16x3", fused_small=False)
    ref = s.sample(upload(shifted), N, seed)
    got = s.sample_stored(_stored(ch, "cf8", "host"), shapes, "cf8", N, seed, emit_n=200)
    torch.cuda.synchronize()
    s.close()
    assert torch.equal(got["outcomes"], ref["outcomes"])
    assert torch.equal(got["logp"], ref["logp"])
    gpu = {k: v.cpu().numpy() for k, v in got.items() if k != "status"}
    rep = compare(expanded, seed, gpu, rows=np.arange(200), eps=EPS_LOWP)
    print(rep, flush=True)


def _with_scales(raw, shape, fn):
    """Copy of complex-fp8 bytes with every block scale s replaced by fn(s)."""
    chi_l, d, chi_r = shape
    n = chi_l * d * chi_r
    off = -(-2 * n // 256) * 256
    nb = -(-chi_l // 128) * -(-(d * chi_r) // 128)
    out = raw.copy()
    sc = out[off:off + 4 * nb].view(np.float32)
    sc[:] = fn(sc.astype(np.float64)).astype(np.float32)
    return out


@pytest.mark.parametrize("variant", ["non_power_of_two", "exponent_span"])
def test_fp8_sites_off_the_fp16_grid_take_three_products(variant):
    """Complex-fp8 host sites that do not expand onto the binary16 grid --
    block scales that are not powers of two, or power-of-two scales whose
    exponents span more than 22 -- are contracted with all three fp16
    products: the staged call is bit-identical to a resident fp16x3 call on
    the expanded tensors (which always takes three products; dropping the
    site's low parts would change W), and matches the FP64 oracle on those
    values at the low-precision bar."""
    from paper_2512_20064_amd import mps
    from tests.parity_util import compare, upload, EPS_LOWP
    print(f"[gpu-case] cf8 host sites off the fp16 grid ({variant}), fp16x3", flush=True)
    ch = _chain(M=10, d=4, chi=300, seed=23)
    shapes = [t.shape for t in ch]
    raws = []
    for k, (t, sh) in enumerate(zip(ch, shapes)):
        if variant == "non_power_of_two":
            raws.append(_with_scales(synth.compress_site(t, "cf8"), sh, lambda s: s * 0.75))
        else:
            t2 = t.copy()
            if sh[0] > 128:  # first row block 2^-26 smaller: its scale exponent is 26 below the others'
                t2[:128] *= np.float32(2.0 ** -26)
            raws.append(synth.compress_site(t2, "cf8"))
    if variant == "non_power_of_two":
        sc = [r[-(-(2 * np.prod(sh)) // 256) * 256:].view(np.float32) for r, sh in zip(raws, shapes)]
        assert all((np.frexp(x.astype(np.float64))[0] != 0.5).any() for x in sc)
    else:
        assert any(sh[0] > 128 for sh in shapes)
    expanded = [_expand_f32(r, sh, "cf8") for r, sh in zip(raws, shapes)]
    stored = [torch.from_numpy(r).pin_memory() for r in raws]
    N, seed = 1200, 515
    s = mps.Sampler(0, n_chunk=512, precision="fp16x3", fused_small=False)
    ref = s.sample(upload(expanded), N, seed)
    got = s.sample_stored(stored, shapes, "cf8", N, seed, emit_n=256)
    torch.cuda.synchronize()
    s.close()
    assert torch.equal(got["outcomes"], ref["outcomes"])
    assert torch.equal(got["logp"], ref["logp"])
    gpu = {k: v.cpu().numpy() for k, v in got.items() if k != "status"}
    rep = compare(expanded, seed, gpu, rows=np.concatenate([np.arange(256), np.arange(N - 100, N)]), eps=EPS_LOWP)
    print(rep, flush=True)


@pytest.mark.parametrize("kind,form", [("cf16", "fp32"), ("cf8", "fp32"), ("cf16", "fp16x3"), ("cf8", "fp16x3")])
def test_staged_parity_with_oracle(kind, form):
    """Compressed pinned-host sites against the FP64 oracle run on the same
    (expanded) tensor values, forced-prefix protocol, the form's bars.  With
    complex-fp16 sites the fp16 split form runs two products per complex
    product (the site tensor's low parts are zero)."""
    from paper_2512_20064_amd import mps
    from tests.parity_util import compare, EPS_LOWP
    print(f"[gpu-case] staged {kind} host parity vs oracle {form}", flush=True)
    ch = _chain(M=14, d=4, chi=64, seed=7)
    shapes = [t.shape for t in ch]
    expanded = [_expand_f32(synth.compress_site(t, kind), t.shape, kind) for t in ch]
    N, seed = 1536, 99
    s = mps.Sampler(0, n_chunk=512, precision=form)
    r = s.sample_stored(_stored(ch, kind, "host"), shapes, kind, N, seed, emit_n=256)
    torch.cuda.synchronize()
    s.close()
    gpu = {k: v.cpu().numpy() for k, v in r.items() if k != "status"}
    rows = np.concatenate([np.arange(256), np.arange(N - 200, N)])
    kw = {} if form == "fp32" else {"eps": EPS_LOWP}
    rep = compare(expanded, seed, gpu, rows=rows, **kw)
    print(rep, flush=True)


def test_staged_profile_times_copies_and_expansions():
    from paper_2512_20064_amd import mps
    print("[gpu-case] staged profile counters", flush=True)
    ch = _chain(M=6, d=2, chi=256, seed=3)
    shapes = [t.shape for t in ch]
    s = mps.Sampler(0, n_chunk=128, profile=True, precision="bf16x3")
    r = s.sample_stored(_stored(ch, "cf16", "host"), shapes, "cf16", 300, 5)
    torch.cuda.synchronize()
    st = s.stats
    s.close()
    assert r["status"] == 0
    assert st.h2d_ms > 0 and st.expand_ms > 0 and st.contract_ms > 0 and st.pack_ms > 0
    assert st.staged_sites == 6 and st.pack_launches == 6 and st.contract_launches == 18


def test_pageable_host_sites_are_rejected():
    from paper_2512_20064_amd import mps
    print("[gpu-case] pageable host pointer rejected", flush=True)
    ch = _chain(M=3, d=2, chi=4)
    raws = [np.ascontiguousarray(synth.compress_site(t, "c64")) for t in ch]
    chi = [1] + [t.shape[2] for t in ch]
    d = [t.shape[1] for t in ch]
    out = torch.empty((8, 3), dtype=torch.int32, device="cuda")
    h = mps.mps_create(0)
    try:
        rc = mps.mps_sample(h, [r.ctypes.data for r in raws], mps.MPS_C64, chi, d, 3, 8, 0, 1, out.data_ptr(), 0)
        assert rc == mps.MPS_EINVAL, (rc, mps.mps_last_error())
        assert "pinned" in mps.mps_last_error()
    finally:
        mps.mps_destroy(h)


def test_site_past_end_of_allocation_is_rejected():
    """A site tensor whose shape runs past the end of its device allocation is
    rejected before anything is launched (the extent comes from
    hipMemGetAddressRange)."""
    import ctypes
    from paper_2512_20064_amd import mps
    print("[gpu-case] site tensor past the end of its allocation rejected", flush=True)
    hip = ctypes.CDLL("libamdhip64.so")
    p = ctypes.c_void_p()
    assert hip.hipMalloc(ctypes.byref(p), ctypes.c_size_t(1 << 16)) == 0
    h = mps.mps_create(0)
    try:
        base, size = ctypes.c_void_p(), ctypes.c_size_t()
        if hip.hipMemGetAddressRange(ctypes.byref(base), ctypes.byref(size), p) != 0:
            pytest.skip("hipMemGetAddressRange does not report this allocation")
        # two sites of 128 B each: (1, 4, 4) and (4, 4, 1); the second starts
        # 64 B before the end of the allocation
        sites = [base.value, base.value + size.value - 64]
        out = torch.empty((8, 2), dtype=torch.int32, device="cuda")
        rc = mps.mps_sample(h, sites, mps.MPS_C64, [1, 4, 1], [4, 4], 2, 8, 0, 1, out.data_ptr(), 0)
        assert rc == mps.MPS_EINVAL, (rc, mps.mps_last_error())
        assert "past the end" in mps.mps_last_error()
    finally:
        mps.mps_destroy(h)
        assert hip.hipFree(p) == 0


def test_staged_with_displacement_equals_resident():
    """Per-sample displacement (Eq. 7) on a staged (pinned-host cf16) chain is
    bit-identical to the same displacement on the resident expanded chain."""
    from paper_2512_20064_amd import mps
    from tests.parity_util import upload
    print("[gpu-case] staged cf16 host + displacement vs resident", flush=True)
    ch = _chain(M=8, d=4, chi=32, seed=17)
    shapes = [t.shape for t in ch]
    expanded = [_expand_f32(synth.compress_site(t, "cf16"), t.shape, "cf16") for t in ch]
    N, seed = 700, 3
    rng = np.random.default_rng(5)
    mu = (0.3 * (rng.standard_normal((N, len(ch))) + 1j * rng.standard_normal((N, len(ch))))).astype(np.complex64)
    mu_d = torch.from_numpy(mu).to("cuda")
    s = mps.Sampler(0, n_chunk=256)
    ref = s.sample(upload(expanded), N, seed, displace=mu_d)
    got = s.sample_stored(_stored(ch, "cf16", "host"), shapes, "cf16", N, seed, displace=mu_d)
    torch.cuda.synchronize()
    s.close()
    assert torch.equal(got["outcomes"], ref["outcomes"]) and torch.equal(got["logp"], ref["logp"])
