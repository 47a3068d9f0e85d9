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


def _mixed_chain():
    """Bonds that are not multiples of the tiles (100, 200, 50, 40) and d_k
    in {2..5}: every site shape has ragged column tiles in both variants."""
    dl = [2, 3, 4, 5, 4, 3, 4, 2, 5, 3, 4, 4]
    chi = [1, 2, 6, 24, 100, 200, 200, 100, 50, 40, 14, 4, 1]
    return synth.to_c64(synth.random_mps(31, dl, chi)), dl, chi


@pytest.mark.parametrize("form", ["fp32", "bf16x3", "fp16x3", "fp16f8", "fp16f6", "fp16"])
def test_tile_choices_are_bit_identical(form, tmp_path):
    """Every site shape on the wide tile, every one on the narrow tile, and the
    tuner's choice give the same outcomes, logp and conditional
    probabilities; the choices are cached by shape and reinstalled."""
    import numpy as np
    from paper_2512_20064_amd import mps
    from tests.parity_util import upload
    print(f"[gpu-case] tile choices {form}", flush=True)
    t, dl, chi = _mixed_chain()
    dev = upload(t)
    N, seed, rows = 3000, 17, 3000
    shapes = sorted({(chi[k], dl[k], chi[k + 1]) for k in range(len(dl))})
    s = mps.Sampler(0, precision=form, n_chunk=rows, fused_small=False)
    runs = {}
    for name, tile in (("wide", mps.MPS_TILE_WIDE), ("narrow", mps.MPS_TILE_NARROW)):
        s.set_tiles([dict(chi_l=a, d=b, chi_r=c, tile=tile, rows=rows) for a, b, c in shapes])
        runs[name] = s.sample(dev, N, seed, emit_n=N)
        torch.cuda.synchronize()
    cache = str(tmp_path / "tiles.json")
    s.set_tiles([])
    choice = s.autotune_tiles(dev, rows, cache=cache)
    print([(c["chi_l"], c["d"], c["chi_r"], c["tile"], round(c["ms_wide"], 4), round(c["ms_narrow"], 4))
           for c in choice], flush=True)
    assert sorted((c["chi_l"], c["d"], c["chi_r"]) for c in choice) == shapes
    assert all(c["rows"] == rows and c["ms_wide"] > 0 and c["ms_narrow"] > 0 and not c["cached"] for c in choice)
    runs["tuned"] = s.sample(dev, N, seed, emit_n=N)
    torch.cuda.synchronize()
    s2 = mps.Sampler(0, precision=form, n_chunk=rows, fused_small=False)
    again = s2.autotune_tiles(dev, rows, cache=cache)
    assert all(c["cached"] for c in again)
    assert [c["tile"] for c in again] == [c["tile"] for c in sorted(choice, key=lambda c: (c["chi_l"], c["d"], c["chi_r"]))]
    runs["cached"] = s2.sample(dev, N, seed, emit_n=N)
    torch.cuda.synchronize()
    ref = runs["wide"]
    for name, r in runs.items():
        assert torch.equal(r["outcomes"], ref["outcomes"]), name
        assert torch.equal(r["logp"], ref["logp"]), name
        assert np.array_equal(r["probs"].cpu().numpy(), ref["probs"].cpu().numpy(), equal_nan=True), name
    s.close()
    s2.close()


@pytest.mark.parametrize("form", ["fp32", "bf16x3", "fp16f8", "fp16f6"])
def test_narrow_tiles_match_the_oracle(form):
    """The narrow tiles on their own against the FP64 oracle (forced prefix)."""
    from paper_2512_20064_amd import mps
    from tests.parity_util import compare, upload
    print(f"[gpu-case] narrow tiles vs oracle {form}", flush=True)
    t, dl, chi = _mixed_chain()
    N, seed, rows = 1500, 23, 1500
    s = mps.Sampler(0, precision=form, n_chunk=rows, fused_small=False)
    s.set_tiles([dict(chi_l=chi[k], d=dl[k], chi_r=chi[k + 1], tile=mps.MPS_TILE_NARROW, rows=rows)
                 for k in range(len(dl))])
    r = s.sample(upload(t), N, seed, emit_n=N)
    torch.cuda.synchronize()
    g = {"outcomes": r["outcomes"].cpu().numpy(), "logp": r["logp"].cpu().numpy(),
         "probs": r["probs"].cpu().numpy(), "u": r["u"].cpu().numpy()}
    s.close()
    print(compare(t, seed, g, eps=1e-5 if form == "fp32" else 1e-3), flush=True)


def test_batch_with_tuned_tiles_is_bit_identical():
    """A batch of chains of different shapes: tuned tiles and the default
    wide tiles give the same bits in mps_sample_batch."""
    import numpy as np
    from paper_2512_20064_amd import mps
    from tests.parity_util import upload
    print("[gpu-case] batch tuned tiles bf16x3", flush=True)
    rng = np.random.default_rng(5)
    chains = []
    for b in range(5):
        dl = [int(x) for x in rng.integers(2, 5, size=int(rng.integers(6, 12)))]
        chains.append(upload(synth.to_c64(synth.random_mps(40 + b, dl, synth.ramp_bonds(dl, [64, 96, 160, 48, 130][b])))))
    N, seed = 2048, 3
    s = mps.Sampler(0, precision="bf16x3", n_chunk=N)
    prep = mps.prepare_batch(chains)
    ref = s.sample_batch(prep, N, seed)
    torch.cuda.synchronize()
    choice = s.autotune_tiles(prep, N)
    print(sum(c["tile"] for c in choice), "of", len(choice), "shapes narrow", flush=True)
    got = s.sample_batch(prep, N, seed)
    torch.cuda.synchronize()
    for (o1, l1), (o2, l2) in zip(ref, got):
        assert torch.equal(o1, o2) and torch.equal(l1, l2)
    s.close()
