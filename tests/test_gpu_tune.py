"""Autotuner (mps_autotune): the chosen chunk and tile order are among the
candidates, and sampling with them is bit-identical to the defaults (the
results never depend on chunking or tile order)."""
import pytest

from paper_2512_20064_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("form", ["fp32", "bf16x3"])
def test_autotune_picks_a_candidate_and_keeps_results(form, tmp_path):
    from paper_2512_20064_amd import mps
    from tests.parity_util import upload
    print(f"[gpu-case] autotune {form}", flush=True)
    dl = [4] * 16
    ch = upload(synth.to_c64(synth.random_mps(12, dl, synth.ramp_bonds(dl, 128))))
    N, seed = 40000, 8
    s = mps.Sampler(0, precision=form)
    cache = str(tmp_path / "tune.json")
    rep = s.autotune(ch, N, seed=1, cache=cache)
    print(rep, flush=True)
    assert rep["n_chunk"] in (8192, 16384, 32768, 40000)
    assert rep["tile_group"] in (1, 2, 4, 8)
    assert rep["candidates"] + rep["skipped"] == 16 and rep["candidates"] > 0
    assert rep["probe_sites"] == 5  # ramp 1, 4, 16, 64 then the first 128 x 4 x 128 site
    assert rep["rate"] > 0 and rep["default_rate"] > 0 and not rep["cached"]
    tuned = s.sample(ch, N, seed)
    torch.cuda.synchronize()
    assert s.stats.n_chunk == rep["n_chunk"]
    ref = mps.Sampler(0, precision=form).sample(ch, N, seed)
    torch.cuda.synchronize()
    assert torch.equal(tuned["outcomes"], ref["outcomes"]) and torch.equal(tuned["logp"], ref["logp"])
    s2 = mps.Sampler(0, precision=form)
    again = s2.autotune(ch, N, cache=cache)
    assert again["cached"] and again["n_chunk"] == rep["n_chunk"] and s2.opt.tile_group == rep["tile_group"]
    s.close()
    s2.close()
