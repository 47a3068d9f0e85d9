"""Pins for the displacement step of the oracle (Section 3.4.1, Eq. 7)."""
import math

import numpy as np
import pytest
from scipy.special import eval_genlaguerre

import oracle
from paper_2512_20064_amd import synth


def _laguerre_displacement(mu, d):
    """<m|D(mu)|n> of the untruncated displacement operator (Cahill and Glauber):
    sqrt(n!/m!) mu^(m-n) e^(-|mu|^2/2) L_n^(m-n)(|mu|^2) for m >= n, and the
    transposed form with -mu^* for m < n."""
    D = np.zeros((d, d), dtype=np.complex128)
    x = abs(mu) ** 2
    for m in range(d):
        for n in range(d):
            if m >= n:
                D[m, n] = math.sqrt(math.factorial(n) / math.factorial(m)) * mu ** (m - n) * \
                    math.exp(-x / 2) * eval_genlaguerre(n, m - n, x)
            else:
                D[m, n] = math.sqrt(math.factorial(m) / math.factorial(n)) * (-np.conj(mu)) ** (n - m) * \
                    math.exp(-x / 2) * eval_genlaguerre(m, n - m, x)
    return D


@pytest.mark.parametrize("d", [2, 3, 4, 6, 8])
def test_displacement_matches_laguerre_closed_form(d):
    """Both factors of Eq. 7 are triangular, so the d x d product is the exact
    top-left block of the untruncated operator."""
    rng = np.random.default_rng(d)
    mus = (rng.standard_normal(6) + 1j * rng.standard_normal(6)) * 0.8
    D = oracle.displacement(mus, d)
    for m, mu in enumerate(mus):
        assert np.max(np.abs(D[m] - _laguerre_displacement(mu, d))) <= 1e-12


def test_displacement_identity_and_coherent_column():
    assert np.array_equal(oracle.displacement(np.zeros(3), 5), np.broadcast_to(np.eye(5), (3, 5, 5)))
    mu = 0.7 - 0.4j
    D = oracle.displacement(np.array([mu]), 6)[0]
    col = np.exp(-abs(mu) ** 2 / 2) * np.array([mu ** i / math.sqrt(math.factorial(i)) for i in range(6)])
    assert np.allclose(D[:, 0], col, atol=1e-15)


def test_displaced_vacuum_is_poisson():
    """chi = 1 chain whose every site is the vacuum: with displacement mu the
    photon-number probabilities are Poisson(|mu|^2), renormalised over the d
    levels, at every site and whatever the prefix."""
    M, d, N, seed = 6, 5, 20000, 3
    vac = np.zeros((1, d, 1), dtype=np.complex128)
    vac[0, 0, 0] = 1.0
    rng = np.random.default_rng(8)
    mu = (rng.standard_normal((N, M)) + 1j * rng.standard_normal((N, M))) * 0.6
    r = oracle.sample([vac] * M, seed=seed, N=N, displace=mu, want_probs=True)
    lam = np.abs(mu) ** 2
    pois = np.exp(-lam)[..., None] * lam[..., None] ** np.arange(d) / np.array([math.factorial(i) for i in range(d)])
    pois /= pois.sum(axis=2, keepdims=True)
    assert np.max(np.abs(r["probs"] - pois)) <= 1e-12
    # the draws follow those probabilities (sites pooled, a chi-square style bound per level)
    hist = np.zeros(d)
    for i in range(d):
        hist[i] = np.mean(r["outcomes"] == i)
    assert np.all(np.abs(hist - pois.mean(axis=(0, 1))) <= 5 * np.sqrt(pois.mean(axis=(0, 1)) / (N * M)) + 1e-3)


def test_zero_displacement_is_the_plain_sampler():
    tensors, d, chi = synth.small_chain(1, M=10, d=4, chi_max=16)
    a = oracle.sample(tensors, seed=2, N=300)
    b = oracle.sample(tensors, seed=2, N=300, displace=np.zeros((300, 10), dtype=np.complex128))
    assert np.array_equal(a["outcomes"], b["outcomes"]) and np.array_equal(a["logp"], b["logp"])


def test_displaced_logp_is_log_of_displaced_amplitude():
    """With displacement the sampled configuration's probability is the
    product of the normalised conditionals; check it against a direct chain
    of (D_k applied to the branch) products for a few samples."""
    tensors, d, chi = synth.small_chain(5, M=8, d=3, chi_max=9)
    N = 40
    rng = np.random.default_rng(1)
    mu = (rng.standard_normal((N, 8)) + 1j * rng.standard_normal((N, 8))) * 0.3
    r = oracle.sample(tensors, seed=4, N=N, displace=mu)
    for n in range(N):
        # direct: amplitude vector after each site, renormalised by the total weight
        v = np.ones((1, 1), dtype=np.complex128)
        lp = 0.0
        for k, A in enumerate(tensors):
            W = np.einsum("l,lir->ir", v[0], A)
            W = oracle.displacement(np.array([mu[n, k]]), A.shape[1])[0] @ W
            q = np.sum(np.abs(W) ** 2, axis=1)
            s = r["outcomes"][n, k]
            lp += math.log(q[s] / q.sum())
            v = (W[s] / math.sqrt(q[s]))[None, :]
        assert abs(lp - r["logp"][n]) <= 1e-10
