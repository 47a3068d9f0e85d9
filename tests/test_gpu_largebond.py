"""Parity at the measured workloads' full sizes, in the launch configurations
the benchmark times, on sampled rows that the oracle computes one by one:

* chi = 10^4 window streamed from pinned host memory in complex-fp16
  (fp16 hi+lo, two products, and bf16 hi+lo; 2^17 samples in chunks of
  65536, sites outer) -- the oracle follows the first 8 sites (ramp
  1 .. 4096 and the first 10^4 x 4 x 10^4 site), which fixes every
  conditional probability up to there;
* uneven chain M = 2048, d_k in {2..6}, chi <= 4096 (bf16 hi+lo, one
  8192-sample chunk) -- first 10 sites;
* the batched 256-chain ensemble (FP32, and fp16f6 with per-shape tuned
  tiles; N = 8192 each) -- whole chains, for a few chains and rows.

The large-bond sites are the structured right-canonical sites of the input
generator: bond blocks visited as a hidden Markov chain, with per-column
branch mixers, so that the conditional probabilities at the chi >= 4096
sites depend on the sampled prefix.  Each test asserts that they do (their
spread over the compared rows), so that a wrong row, a wrong branch in the
gather or a wrapped index changes what is compared.  The compared rows
include row 65535 of a 65536-sample chunk at chi = 10^4, whose W entries
lie past 2^31 elements.  A second call on the compared prefix alone must
reproduce the same outcomes (a site never looks at later sites), and its
logp is checked against the oracle's path probability.
"""
import numpy as np
import pytest

from paper_2512_20064_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SPREAD_MIN = 1e-2


def _assert_prefix_dependent(ref, seed, outcomes, rows, sites, n_index=None):
    """The oracle's conditionals at `sites` vary over the compared rows."""
    import oracle
    f = oracle.forced_probs(synth.promote(ref), outcomes[rows], seed,
                            n_index=np.asarray(rows if n_index is None else n_index))
    spreads = []
    for k in sites:
        p = f["probs"][:, k, :]
        p = p[:, ~np.isnan(p).any(axis=0)]
        spreads.append(float((p.max(axis=0) - p.min(axis=0)).max()))
    assert min(spreads) > SPREAD_MIN, spreads
    return spreads


@pytest.mark.parametrize("form", ["fp16x3", "bf16x3", "fp16f8", "fp16f6"])
def test_chi10000_streamed_window_prefix_parity(form):
    """fp16x3 runs two MFMA products per complex product on these fp16-exact
    sites (the streamed workload's default); bf16x3 runs three."""
    from oracle.sampler import decode_site
    from paper_2512_20064_amd import mps
    from tests.parity_util import compare
    print(f"[gpu-case] chi=1e4 cf16 pinned window, N=2^17, {form}", flush=True)
    M, chi_max = 20, 10000
    dl = [4] * M
    sites, bonds = synth.structured_chain(5, dl, chi_max, pool=4, device="cuda")
    host, stored = {}, []
    for A in sites:
        if id(A) not in host:
            b = synth.compress_site_torch(A, "cf16")
            h = torch.empty(b.numel(), dtype=torch.uint8, pin_memory=True)
            h.copy_(b)
            host[id(A)] = h
        stored.append(host[id(A)])
    shapes = [(bonds[k], 4, bonds[k + 1]) for k in range(M)]
    del sites
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    N, seed = 1 << 17, 2024
    s = mps.Sampler(0, n_chunk=65536, precision=form)
    r = s.sample_stored(stored, shapes, "cf16", N, seed, emit_n=N)
    torch.cuda.synchronize()
    st = s.stats
    assert r["status"] == 0 and st.staged_sites == M and st.contract_launches == 2 * M
    P = 8
    assert shapes[P - 2] == (4096, 4, chi_max) and shapes[P - 1] == (chi_max, 4, chi_max)
    ref = [decode_site(stored[k].numpy(), shapes[k], "cf16") for k in range(P)]
    gpu = {"outcomes": r["outcomes"][:, :P].cpu().numpy(), "logp": r["logp"].cpu().numpy(),
           "probs": r["probs"][:, :P].cpu().numpy(), "u": r["u"][:, :P].cpu().numpy()}
    del r
    rows = np.array([0, 1, 2, 3, 4, 5, 6, 7, 65535, 65536, 100000, N - 1])
    spreads = _assert_prefix_dependent(ref, seed, gpu["outcomes"], rows, [P - 2, P - 1])
    rep = compare(ref, seed, gpu, rows=rows, eps=1e-3, check_logp=False)
    print("spread", spreads, rep, flush=True)
    # the prefix alone: same outcomes, and logp checked along the path
    rp = s.sample_stored(stored[:P], shapes[:P], "cf16", N, seed)
    torch.cuda.synchronize()
    s.close()
    out_p = rp["outcomes"].cpu().numpy()
    assert np.array_equal(out_p, gpu["outcomes"])
    rep = compare(ref, seed, {"outcomes": out_p, "logp": rp["logp"].cpu().numpy()}, rows=rows, eps=1e-3)
    print("prefix call", rep, flush=True)


@pytest.mark.parametrize("form", ["bf16x3", "fp16f8", "fp16f6"])
def test_uneven_chain_prefix_parity(form):
    from paper_2512_20064_amd import mps
    from tests.parity_util import compare
    print(f"[gpu-case] uneven M=2048 chi<=4096, 8192-sample chunk, {form}", flush=True)
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([4, 0, 0xD])))
    dl = [int(x) for x in rng.integers(2, 7, size=2048)]
    sites, bonds = synth.structured_chain(4, dl, 4096, pool=2, device="cuda")
    N, seed = 8192, 1003
    P = 10
    s = mps.Sampler(0, n_chunk=8192, precision=form)
    r = s.sample(sites, N, seed, emit_n=N, emit_dmax=6)
    torch.cuda.synchronize()
    assert r["status"] == 0
    big = [k for k in range(P) if max(bonds[k], bonds[k + 1]) == 4096]
    assert len(big) >= 2 and any(bonds[k] == bonds[k + 1] == 4096 for k in big)
    ref = [sites[k].cpu().numpy() for k in range(P)]
    gpu = {"outcomes": r["outcomes"][:, :P].cpu().numpy(), "logp": r["logp"].cpu().numpy(),
           "probs": r["probs"][:, :P].cpu().numpy(), "u": r["u"][:, :P].cpu().numpy()}
    del r
    rows = np.concatenate([np.arange(8), np.array([1000, 4095, 4096, N - 1])])
    spreads = _assert_prefix_dependent(ref, seed, gpu["outcomes"], rows, big)
    rep = compare(ref, seed, gpu, rows=rows, eps=1e-3, check_logp=False)
    print("spread", spreads, rep, flush=True)
    rp = s.sample(sites[:P], N, seed)
    torch.cuda.synchronize()
    s.close()
    out_p = rp["outcomes"].cpu().numpy()
    assert np.array_equal(out_p, gpu["outcomes"])
    rep = compare(ref, seed, {"outcomes": out_p, "logp": rp["logp"].cpu().numpy()}, rows=rows, eps=1e-3)
    print("prefix call", rep, flush=True)


@pytest.mark.parametrize("form", ["fp32", "fp16f6"])
def test_full_ensemble_sampled_parity(form):
    """The batched ensemble in FP32 (its configured form, bar 1e-5) and in the
    headline low-precision form with per-shape tuned tiles (bar 1e-3)."""
    from paper_2512_20064_amd import mps
    from tests.parity_util import compare, upload
    print(f"[gpu-case] 256-chain ensemble, N=8192, {form}", flush=True)
    specs = synth.ensemble_specs(seed=2, B=256)
    chains = []
    for b, (Mb, db, cb) in enumerate(specs):
        dl = [db] * Mb
        chains.append(synth.to_c64(synth.random_mps(7, dl, synth.ramp_bonds(dl, cb), mps_id=b, pool=4)))
    dev = [upload(c) for c in chains]
    N, seed = 8192, 77
    s = mps.Sampler(0, n_chunk=8192, precision=form)
    if form != "fp32":
        prep = mps.prepare_batch(dev)
        s.autotune_tiles(prep, N)
        outs = s.sample_batch(prep, N, seed)
    else:
        outs = s.sample_batch(dev, N, seed)
    torch.cuda.synchronize()
    assert s.status == 0
    s.close()
    biggest = max(range(256), key=lambda b: specs[b][2] * specs[b][1] * specs[b][0])
    rows = np.concatenate([np.arange(6), np.array([4096, N - 1])])
    for b in sorted({0, 128, 255, biggest}):
        gpu = {"outcomes": outs[b][0].cpu().numpy(), "logp": outs[b][1].cpu().numpy()}
        rep = compare(chains[b], seed, gpu, rows=rows, mps_id=b, eps=1e-5 if form == "fp32" else 1e-3)
        print(b, specs[b], rep, flush=True)
