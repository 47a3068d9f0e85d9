"""Parity at full size, in the launch configuration the benchmark times.

Resident chain M=1024, d=4, chi=1024 (bond ramp 1..1024 at both ends),
complex64, one 65536-sample chunk.  The oracle cannot redo 65536 x 1024
site-samples, so it checks sampled rows one by one along the GPU's own path
(forced prefix): rows spread over the first, middle and last row tiles of
the chunk, with the debug emits (probabilities and uniforms) on the first 16.
"""
import numpy as np
import pytest

from paper_2512_20064_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CHUNK = 65536
SEED = 1003


EPS = {"fp32": 1e-5, "bf16x3": 1e-3, "fp16x3": 1e-3, "fp16f8": 1e-3, "fp16f6": 1e-3}


@pytest.mark.timeout(900)
@pytest.mark.parametrize("form", ["fp32", "bf16x3", "fp16x3", "fp16f8", "fp16f6"])
def test_resident_chain_sampled_rows(form):
    from paper_2512_20064_amd import mps
    from tests.parity_util import compare
    print(f"[gpu-case] full size M=1024 d=4 chi=1024 chunk=65536 {form}", flush=True)
    t128, d, chi = synth.resident_chain(tensor_seed=3, M=1024, d=4, chi_max=1024, pool=16)
    t64 = synth.to_c64(t128)
    del t128
    cache, dev = {}, []
    for t in t64:
        if id(t) not in cache:
            cache[id(t)] = torch.from_numpy(t).to("cuda")
            dev.append(cache[id(t)])
        else:
            dev.append(cache[id(t)].clone())
    s = mps.Sampler(0, n_chunk=CHUNK, precision=form)
    r = s.sample(dev, CHUNK, SEED, n_offset=0, emit_n=16)
    torch.cuda.synchronize()
    assert r["status"] == 0
    rng = np.random.default_rng(0)
    rows = np.concatenate([np.arange(16), [127, 128, 4095, 32767, 32768, 65534, 65535],
                           rng.choice(np.arange(16, CHUNK), size=9, replace=False)])
    outc = r["outcomes"].cpu().numpy()
    sub = {"outcomes": outc[rows], "logp": r["logp"].cpu().numpy()[rows],
           "probs": r["probs"].cpu().numpy(), "u": r["u"].cpu().numpy()}
    assert outc.min() >= 0 and outc.max() <= 3
    s.close()
    del dev, cache, r
    torch.cuda.empty_cache()
    rep = compare(t64, SEED, sub, n_index=rows, eps=EPS[form])
    print(rep, flush=True)
