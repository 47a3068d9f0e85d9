"""Pins for the FP64 oracle: closed forms, invariants, brute force, a library cross-check.

Each test checks the oracle against something other than itself, chosen so
that a plausible slip (dropped term, wrong index, transposed operand, wrong
draw rule) fails at least one of them.  CPU only.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import sampler as osamp
from oracle.philox import philox4x64, philox4x64_np, uniforms, bits_to_uniform, MASK64
from paper_2512_20064_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")


# ----------------------------------------------------------------- RNG ----

def test_philox_matches_numpy_library():
    """numpy's Philox (a library implementation of the same published
    algorithm) advances its counter before producing a block, so its first
    block for counter c equals the definition at c + 1."""
    rng = np.random.default_rng(7)
    for _ in range(20):
        key = [int(x) for x in rng.integers(0, 2**63, size=2, dtype=np.int64)]
        ctr = [int(x) for x in rng.integers(0, 2**63, size=4, dtype=np.int64)]
        bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(ctr, dtype=np.uint64))
        got = [int(v) for v in bg.random_raw(4)]
        c = list(ctr)
        c[0] = (c[0] + 1) & MASK64
        assert got == list(philox4x64(tuple(c), tuple(key)))


def test_philox_vectorised_equals_scalar():
    rng = np.random.default_rng(11)
    c = rng.integers(0, 2**64 - 1, size=(4, 64), dtype=np.uint64, endpoint=True)
    c[:, :4] = np.uint64(MASK64)  # carries and top bits
    c[:, 4:8] = 0
    key = (0xFFFFFFFFFFFFFFFF, 12345)
    out = philox4x64_np(c[0], c[1], c[2], c[3], *key)
    for j in range(c.shape[1]):
        ref = philox4x64(tuple(int(c[i, j]) for i in range(4)), key)
        assert tuple(int(o[j]) for o in out) == ref


def test_uniform_open_interval():
    u = bits_to_uniform(np.array([0, MASK64], dtype=np.uint64))
    assert u[0] == 2.0 ** -53 and u[1] == 1.0 - 2.0 ** -53
    assert np.all((u > 0) & (u < 1))
    uu = uniforms(5, 0, np.arange(200000), 3)
    assert abs(uu.mean() - 0.5) < 5e-3 and abs(uu.var() - 1 / 12) < 2e-3


# ----------------------------------------------------------- generator ----

def test_ramp_bonds():
    chi = synth.ramp_bonds([4] * 32, 32)
    assert chi[:5] == [1, 4, 16, 32, 32] and chi[-5:] == [32, 32, 16, 4, 1]
    chi = synth.ramp_bonds([4] * 1024, 1024)
    assert chi[:7] == [1, 4, 16, 64, 256, 1024, 1024]
    assert chi[-7:] == [1024, 1024, 256, 64, 16, 4, 1]
    dl = [2, 5, 3, 6, 2, 4]
    chi = synth.ramp_bonds(dl, 10)
    for k in range(6):
        assert chi[k] <= dl[k] * chi[k + 1]


def test_generator_right_canonical():
    tensors, d, chi = synth.small_chain(1, M=12, d=4, chi_max=32)
    for B in tensors:
        assert synth.canonical_error(B) <= 1e-12
    pooled = synth.random_mps(2, [3] * 10, synth.ramp_bonds([3] * 10, 20), pool=2)
    for B in pooled:
        assert synth.canonical_error(B) <= 1e-12


# ---------------------------------------------------------- invariants ----

def test_total_weight_is_one_on_canonical_chain():
    """sum_i B_i B_i^H = I makes S = ||l||^2 = 1 at every site; a transposed
    or mis-reshaped contraction breaks it."""
    tensors, d, chi = synth.small_chain(1)
    r = oracle.sample(tensors, seed=1001, N=512, want_probs=True)
    assert np.max(np.abs(r["S"] - 1.0)) <= 1e-12
    assert np.max(np.abs(np.nansum(r["probs"], axis=2) - 1.0)) <= 1e-12


def test_draw_rule_ties_and_zero_branches():
    C = np.array([[0.25, 0.5, 1.0]] * 4)
    u = np.array([0.25, np.nextafter(0.25, 1), np.nextafter(0.25, 0), 0.9999])
    assert list(osamp.draw(C, u)) == [0, 1, 0, 2]
    Cz = np.array([[0.5, 0.5, 1.0]])  # branch 1 has zero weight
    assert osamp.draw(Cz, np.array([0.5]))[0] == 0
    assert osamp.draw(Cz, np.array([np.nextafter(0.5, 1)]))[0] == 2
    # clamp: rounding could leave C_{d-1} below u
    assert osamp.draw(np.array([[0.3, 0.9999999]]), np.array([0.99999995]))[0] == 1


def test_product_state_closed_form():
    """chi = 1: p_k(i) = |A_k[0,i,0]|^2 regardless of the prefix, so every
    outcome is predicted from the closed form without any contraction."""
    rng = np.random.default_rng(3)
    M, d, N, seed = 9, 4, 2000, 77
    tensors = []
    for k in range(M):
        a = rng.standard_normal(d) + 1j * rng.standard_normal(d)
        a *= np.exp(-0.5 * np.arange(d))
        tensors.append((a / np.linalg.norm(a)).reshape(1, d, 1))
    r = oracle.sample(tensors, seed=seed, N=N)
    u = uniforms(seed, 0, np.arange(N)[:, None], np.arange(M)[None, :])
    logp = np.zeros(N)
    for k in range(M):
        p = np.abs(tensors[k][0, :, 0]) ** 2
        cdf = np.cumsum(p) / p.sum()
        want = np.minimum(np.searchsorted(cdf, u[:, k], side="left"), d - 1)
        assert np.array_equal(r["outcomes"][:, k], want)
        logp += np.log(p[want] / p.sum())
    assert np.allclose(r["logp"], logp, rtol=0, atol=1e-12)


def test_exact_two_branch_example():
    g = json.load(open(GOLDEN))["product_state"]["exact_example"]
    a = np.array([complex(*z) for z in g["site"]]).reshape(1, 2, 1)
    r = oracle.sample([a], seed=5, N=4000, want_probs=True)
    assert np.allclose(r["probs"][:, 0, :], g["p"], atol=1e-15)
    u = r["u"][:, 0]
    assert np.array_equal(r["outcomes"][:, 0], (u > 0.36).astype(np.int32))


def _w_state(M):
    t = []
    for k in range(M):
        cl = 1 if k == 0 else 2
        cr = 1 if k == M - 1 else 2
        B = np.zeros((cl, 2, cr), dtype=np.complex128)
        if k < M - 1:
            B[0, 0, 0] = math.sqrt((M - k - 1) / (M - k))
            B[0, 1, 1] = math.sqrt(1.0 / (M - k))
            if cl == 2:
                B[1, 0, 1] = 1.0
        else:
            B[0, 1, 0] = 1.0
            if cl == 2:
                B[1, 0, 0] = 1.0
        t.append(B)
    return t


def _ghz_state(M, d):
    t = []
    for k in range(M):
        cl = 1 if k == 0 else d
        cr = 1 if k == M - 1 else d
        B = np.zeros((cl, d, cr), dtype=np.complex128)
        for a in range(d):
            B[0 if k == 0 else a, a, 0 if k == M - 1 else a] = 1 / math.sqrt(d) if k == 0 else 1.0
        t.append(B)
    return t


def test_golden_w_state():
    for case in json.load(open(GOLDEN))["w_state"]["cases"]:
        M = case["M"]
        t = _w_state(M)
        for B in t:
            assert synth.canonical_error(B) <= 1e-15
        r = oracle.sample(t, seed=9, N=40000)
        o = r["outcomes"]
        assert np.all(o.sum(axis=1) == 1)  # exactly one excitation
        assert np.allclose(r["logp"], case["logp"], atol=1e-12)
        freq = np.bincount(np.argmax(o, axis=1), minlength=M) / o.shape[0]
        p = case["p_one_hot"]
        assert np.all(np.abs(freq - p) <= 5 * math.sqrt(p * (1 - p) / o.shape[0]))
        configs, pb = oracle.brute_force(t)
        assert np.isclose(pb.sum(), 1.0, atol=1e-14)
        assert np.allclose(pb[configs.sum(axis=1) == 1], p, atol=1e-14)


def test_golden_ghz_state():
    for case in json.load(open(GOLDEN))["ghz_state"]["cases"]:
        t = _ghz_state(case["M"], case["d"])
        r = oracle.sample(t, seed=10, N=30000)
        o = r["outcomes"]
        assert np.all(o == o[:, :1])
        assert np.allclose(r["logp"], case["logp"], atol=1e-12)
        freq = np.bincount(o[:, 0], minlength=case["d"]) / o.shape[0]
        p = case["p_each"]
        assert np.all(np.abs(freq - p) <= 5 * math.sqrt(p * (1 - p) / o.shape[0]))


# ---------------------------------------------------------- brute force ----

TINY = [(6, 2, 4), (7, 2, 8), (4, 3, 9), (3, 4, 4)]


def _tv(tensors, seed, n):
    dims = [t.shape[1] for t in tensors]
    configs, p = oracle.brute_force(tensors)
    r = oracle.sample(tensors, seed=seed, N=n)
    hist = np.bincount(oracle.config_index(r["outcomes"], dims), minlength=len(p)) / n
    idx = oracle.config_index(configs, dims)
    return 0.5 * np.sum(np.abs(hist[idx] - p)), p


@pytest.mark.parametrize("M,d,chi", TINY)
def test_brute_force_total_variation(M, d, chi):
    tensors = synth.random_mps(100 + M, [d] * M, synth.ramp_bonds([d] * M, chi))
    tv, p = _tv(tensors, seed=2024, n=10**6)
    assert abs(p.sum() - 1.0) <= 1e-12
    assert tv <= 5e-3, tv


def test_brute_force_chi_square_larger_chain():
    from scipy import stats
    M, d, chi = 5, 4, 16
    tensors = synth.random_mps(55, [d] * M, synth.ramp_bonds([d] * M, chi))
    configs, p = oracle.brute_force(tensors)
    n = 400000
    r = oracle.sample(tensors, seed=99, N=n)
    counts = np.bincount(oracle.config_index(r["outcomes"], [d] * M), minlength=len(p))
    idx = oracle.config_index(configs, [d] * M)
    expected = p * n
    counts = counts[idx]
    big = expected >= 5  # pool the sparse tail into one cell
    obs = np.append(counts[big], counts[~big].sum())
    exp = np.append(expected[big], expected[~big].sum())
    chi2, pval = stats.chisquare(obs, exp)
    assert pval > 1e-4, (chi2, pval)


def test_site0_marginal():
    tensors, d, chi = synth.small_chain(1, M=8, d=4, chi_max=16)
    p0 = np.sum(np.abs(tensors[0][0]) ** 2, axis=1)
    n = 200000
    r = oracle.sample(tensors, seed=31, N=n)
    freq = np.bincount(r["outcomes"][:, 0], minlength=4) / n
    assert np.all(np.abs(freq - p0) <= 5 * np.sqrt(p0 * (1 - p0) / n) + 1e-12)


def test_logp_is_log_amplitude():
    """Chain rule: sum_k ln p_k(s_k | prefix) = ln |psi(s)|^2, evaluated by the
    direct matrix product, a different algorithm."""
    tensors, d, chi = synth.small_chain(1)
    r = oracle.sample(tensors, seed=1001, N=64)
    for n in range(64):
        assert abs(r["logp"][n] - math.log(oracle.amplitude_norm2(tensors, r["outcomes"][n]))) <= 1e-10


# ------------------------------------------------------- chunk / forced ----

def test_chunk_offset_invariance():
    tensors, d, chi = synth.small_chain(1, M=16)
    full = oracle.sample(tensors, seed=3, N=700)
    a = oracle.sample(tensors, seed=3, N=300)
    b = oracle.sample(tensors, seed=3, N=400, n_offset=300)
    assert np.array_equal(full["outcomes"], np.vstack([a["outcomes"], b["outcomes"]]))
    # BLAS may block a different batch size differently: FP64 rounding only
    assert np.allclose(full["logp"], np.concatenate([a["logp"], b["logp"]]), rtol=0, atol=1e-12)


def test_forced_prefix_self_consistency():
    tensors, d, chi = synth.small_chain(1, M=16)
    r = oracle.sample(tensors, seed=4, N=300)
    f = oracle.forced_probs(tensors, r["outcomes"], seed=4)
    assert np.array_equal(f["s_draw"], r["outcomes"])
    assert np.array_equal(f["logp"], r["logp"])
    lp = np.sum(np.log(np.take_along_axis(f["probs"], r["outcomes"][:, :, None], axis=2)[:, :, 0]), axis=1)
    assert np.allclose(lp, r["logp"], atol=1e-12)
    # forcing a different path changes later conditionals but they stay normalised
    other = (r["outcomes"] + 1) % d[0]
    g = oracle.forced_probs(tensors, other, seed=4)
    assert np.allclose(np.nansum(g["probs"], axis=2), 1.0, atol=1e-12)


def test_dead_samples_are_flagged():
    tensors, d, chi = synth.small_chain(1, M=10, d=3, chi_max=9)
    bad = [t.copy() for t in tensors]
    bad[4] = np.zeros_like(bad[4])
    r = oracle.sample(bad, seed=8, N=50)
    assert np.all(r["outcomes"][:, 4:] == -1) and np.all(r["outcomes"][:, :4] >= 0)
    assert np.all(np.isneginf(r["logp"]))
    nan = [t.copy() for t in tensors]
    nan[2] = nan[2] * np.nan
    r = oracle.sample(nan, seed=8, N=5)
    assert np.all(r["outcomes"][:, 2:] == -1)


# --------------------------------------------------- planted mistakes ----

def test_planted_mistakes_are_caught(monkeypatch):
    """Plant slips in the oracle (CPU) and check the pins above would fail."""
    M, d, chi = 4, 3, 9
    tensors = synth.random_mps(104, [d] * M, synth.ramp_bonds([d] * M, chi))
    # 1) off-by-one in the inverse CDF
    real_draw = osamp.draw
    monkeypatch.setattr(osamp, "draw", lambda C, u: np.minimum(real_draw(C, u) + 1, C.shape[-1] - 1).astype(np.int32))
    tv, _ = _tv(tensors, seed=2024, n=200000)
    assert tv > 0.05
    monkeypatch.setattr(osamp, "draw", real_draw)
    # 2) transposed bond indices in the site tensors (contract over chi_r)
    sw = [np.ascontiguousarray(t.transpose(2, 1, 0)) for t in tensors[::-1]]
    configs, p = oracle.brute_force(tensors)
    r = oracle.sample(sw, seed=1, N=200000)
    # sampled right-to-left chain read left-to-right is a different distribution
    hist = np.bincount(oracle.config_index(r["outcomes"], [d] * M), minlength=len(p)) / 200000
    assert 0.5 * np.abs(hist[oracle.config_index(configs, [d] * M)] - p).sum() > 0.05
