"""Batched sweep over many chains (mps_sample_batch) against single-chain
calls and the oracle."""
import numpy as np
import pytest

from paper_2512_20064_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _ensemble(n, seed=2):
    specs = synth.ensemble_specs(seed=seed, B=n, M_lo=6, M_hi=24, chis=(4, 16, 32, 48, 130), ds=(2, 3, 4))
    chains = []
    for b, (M, d, chi) in enumerate(specs):
        dl = [d] * M
        chains.append(synth.to_c64(synth.random_mps(seed, dl, synth.ramp_bonds(dl, chi), mps_id=b)))
    return chains


@pytest.mark.parametrize("form", ["fp32", "bf16x3", "fp16", "fp16x3", "fp16f8", "fp16f6"])
def test_batch_equals_single_chain_calls(form):
    """Chain b of a batch is bit-identical to mps_sample on chain b with mps_id = b."""
    from paper_2512_20064_amd import mps
    from tests.parity_util import upload
    print(f"[gpu-case] batch of 12 mixed chains vs single calls {form}", flush=True)
    chains = _ensemble(12)
    dev = [upload(c) for c in chains]
    N, seed = 700, 4242
    s = mps.Sampler(0, n_chunk=300, precision=form)
    outs = s.sample_batch(dev, N, seed)
    torch.cuda.synchronize()
    # chains with bonds <= 32 (d <= 4 here) take the persistent FP32 kernel
    small = [c for c in chains if max(max(t.shape[0], t.shape[2]) for t in c) <= 32]
    big = [c for c in chains if not any(c is x for x in small)]
    assert s.status == 0 and s.stats.contract_launches == (max(len(c) for c in big) if big else 0) * 3  # 3 chunks
    assert s.stats.fused_launches == (3 if small else 0)
    # descriptors prepared once give the same bits, call after call
    prep = mps.prepare_batch(dev)
    for _ in range(2):
        again = s.sample_batch(prep, N, seed)
        torch.cuda.synchronize()
        for (o1, l1), (o2, l2) in zip(outs, again):
            assert torch.equal(o1, o2) and torch.equal(l1, l2)
    s.close()
    for b, c in enumerate(dev):
        one = mps.Sampler(0, n_chunk=300, precision=form, mps_id=b)
        r = one.sample(c, N, seed)
        torch.cuda.synchronize()
        assert torch.equal(r["outcomes"], outs[b][0]), b
        assert torch.equal(r["logp"], outs[b][1]), b
        one.close()


def test_batch_chain_parity_with_oracle():
    """One chain of a batch against the FP64 oracle keyed with its own mps_id."""
    import oracle
    from paper_2512_20064_amd import mps
    from tests.parity_util import upload
    print("[gpu-case] batch chain parity vs oracle", flush=True)
    chains = _ensemble(6, seed=5)
    dev = [upload(c) for c in chains]
    N, seed = 512, 77
    s = mps.Sampler(0)
    outs = s.sample_batch(dev, N, seed)
    torch.cuda.synchronize()
    s.close()
    for b in (0, 3, 5):
        o = outs[b][0].cpu().numpy()
        lp = outs[b][1].cpu().numpy()
        f = oracle.forced_probs(synth.promote(chains[b]), o, seed, mps_id=b)
        p_path = np.take_along_axis(f["probs"], o[:, :, None], axis=2)[:, :, 0]
        assert np.all(np.abs(lp - np.log(p_path).sum(axis=1)) <= (1e-5 / p_path).sum(axis=1) + 1e-9)
        # outside a 1e-5 band around the oracle CDF the draws agree
        d = np.array([t.shape[1] for t in chains[b]])
        C, u = f["cdf"], f["u"]
        dist = np.full(u.shape, np.inf)
        for j in range(C.shape[2] - 1):
            dist = np.minimum(dist, np.where((j < d - 1)[None, :] & ~np.isnan(C[:, :, j]),
                                             np.abs(u - C[:, :, j]), np.inf))
        assert np.all((o == f["s_draw"]) | (dist <= d[None, :] * 1e-5))
