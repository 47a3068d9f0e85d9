"""Plain FP64 MPS sampler: the oracle the HIP sweep is checked against.

Test infrastructure only.  Nothing on the product path imports this module;
the tests, the smoke check and the CPU-baseline leg of the benchmark do.

What is computed (Section 2.2, the sequential sampling workflow, and
Section 3.3.1, Algorithm 1), one pass over the chain per batch of samples,
left to right, every sample independent of the others:

  l_0 = [1]                                   (the open left end, chi_0 = 1)
  for site k:
      W[n, i, r] = sum_l l[n, l] A_k[l, i, r]          contraction, no conjugate
      q[n, i]    = sum_r |W[n, i, r]|^2                 branch weights
      P[n, j]    = q[n, 0] + ... + q[n, j]              left-to-right prefix sums
      S[n]       = P[n, d-1]
      C[n, j]    = P[n, j] / S[n]                       so C[n, d-1] == 1 exactly
      s[n]       = #{ j : u[n, k] > C[n, j] }, at most d-1    (strict compare)
      logp[n]   += ln q[n, s] - ln S[n]
      l[n, :]    = W[n, s, :] / sqrt(q[n, s])           gather + renormalise

Readings of the paper taken here (each listed with its reason in the design
notes of the repository):

* Algorithm 1 forms the branch probabilities as ``dot(temp_tensor, Lambda)``.
  The input tensors are taken right-canonical, B_k = Gamma_k diag(Lambda_k),
  so Lambda is absorbed and the weight of branch i is the squared 2-norm of
  W[n, i, :].
* Site tensors are laid out (chi_l, d, chi_r) and contracted over their first
  index, so each branch is a contiguous run of the right bond.
* The paper rescales each sample by its own maximum (Section 3.3.1); any
  positive per-sample scale cancels in C and in q_s/S, so the oracle
  renormalises by the 2-norm of the chosen branch.
* The threshold comparison is strict, so a uniform equal to C_j selects a
  later branch and a zero-weight branch is never selected for u in (0, 1);
  the index is clamped to d-1 as a guard.
* A sample whose S is not a positive finite number stops: outcome -1 from
  that site on, logp = -inf, left vector zero.
"""
from __future__ import annotations

import itertools

import numpy as np

from .philox import uniforms


def draw(C: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Inverse-CDF index per row: #{j : u > C[:, j]}, clamped to d-1 (Algorithm 1)."""
    d = C.shape[-1]
    s = np.sum(u[..., None] > C, axis=-1)
    return np.minimum(s, d - 1).astype(np.int32)


def _check_chain(tensors):
    assert len(tensors) >= 1
    assert tensors[0].shape[0] == 1, "open left end: chi_0 must be 1"
    for a, b in zip(tensors[:-1], tensors[1:]):
        assert a.shape[2] == b.shape[0], "bond mismatch"


def displacement(mu: np.ndarray, d: int) -> np.ndarray:
    """Displacement operators D(mu) on a d-level Fock space, one per entry of mu.

    Eq. 7 (Section 3.4.1): D(mu) = e^{-|mu|^2/2} e^{mu a^+} e^{-mu^* a}.  Both
    factors are exponentials of nilpotent matrices, so each is its finite power
    series sum_{k<d} X^k / k!, summed here term by term.  Returns an array of
    shape mu.shape + (d, d), complex128.
    """
    mu = np.asarray(mu, dtype=np.complex128)
    a = np.diag(np.sqrt(np.arange(1, d, dtype=np.float64)), 1).astype(np.complex128)  # a|n> = sqrt(n)|n-1>
    ad = a.T.copy()
    X = mu[..., None, None] * ad  # mu a^+
    Y = -np.conj(mu)[..., None, None] * a  # -mu^* a
    eye = np.broadcast_to(np.eye(d, dtype=np.complex128), X.shape)
    EX, EY = eye.copy(), eye.copy()
    PX, PY = eye.copy(), eye.copy()
    for k in range(1, d):
        PX = PX @ X / k
        PY = PY @ Y / k
        EX = EX + PX
        EY = EY + PY
    return np.exp(-np.abs(mu) ** 2 / 2)[..., None, None] * (EX @ EY)


def sample(tensors, seed: int, N: int, n_offset: int = 0, mps_id: int = 0,
           forced: np.ndarray | None = None, want_probs: bool = False,
           n_index: np.ndarray | None = None, displace: np.ndarray | None = None):
    """Sample N configurations (global indices n_offset .. n_offset+N-1, or
    the explicit global indices ``n_index`` when given).

    tensors: list of M complex arrays (chi_k, d_k, chi_{k+1}); promoted to
    complex128.  With ``forced`` (int array [N, M]) the chosen branch at each
    site is taken from it instead of the draw: the forced-prefix mode used to
    read the conditional probabilities along another sampler's path.  With
    ``displace`` (complex [N, M]) the physical index of each sample's W is
    transformed by the displacement operator D(mu[n, k]) before the branch
    weights are formed (the per-sample random displacement of MPS-based GBS
    simulation, Section 3.4.1).

    Returns a dict with
      outcomes [N, M] int32  (-1 after a sample stops),
      logp     [N]    float64,
      and with want_probs or forced:
      probs    [N, M, dmax] float64 conditional probabilities q_i / S (NaN padded),
      s_draw   [N, M] int32   the oracle's own inverse-CDF choice,
      u        [N, M] float64 the uniforms,
      cdf      [N, M, dmax] float64 C_j (NaN padded),
      S        [N, M] float64 the total weight S before normalising.
    """
    _check_chain(tensors)
    M = len(tensors)
    dmax = max(t.shape[1] for t in tensors)
    if n_index is not None:
        n = np.asarray(n_index, dtype=np.uint64)
        assert n.shape == (N,)
    else:
        n = np.arange(N, dtype=np.uint64) + np.uint64(n_offset)
    l = np.ones((N, 1), dtype=np.complex128)
    alive = np.ones(N, dtype=bool)
    logp = np.zeros(N, dtype=np.float64)
    outcomes = np.full((N, M), -1, dtype=np.int32)
    record = want_probs or forced is not None
    if record:
        probs = np.full((N, M, dmax), np.nan)
        cdf = np.full((N, M, dmax), np.nan)
        S_all = np.full((N, M), np.nan)
        s_draw = np.full((N, M), -1, dtype=np.int32)
        u_all = np.zeros((N, M))
    rows = np.arange(N)
    for k in range(M):
        A = np.asarray(tensors[k], dtype=np.complex128)
        chi_l, d, chi_r = A.shape
        assert l.shape[1] == chi_l
        W = (l @ A.reshape(chi_l, d * chi_r)).reshape(N, d, chi_r)
        if displace is not None:
            W = displacement(np.asarray(displace)[:, k], d) @ W
        q = np.sum(W.real ** 2 + W.imag ** 2, axis=2)
        P = np.cumsum(q, axis=1)
        S = P[:, d - 1]
        ok = alive & np.isfinite(S) & (S > 0)
        Ssafe = np.where(ok, S, 1.0)
        C = P / Ssafe[:, None]
        C[:, d - 1] = np.where(ok, 1.0, C[:, d - 1])  # P[d-1]/S is exactly 1 already
        u = uniforms(seed, mps_id, n, k)
        s_orc = draw(C, u)
        s = s_orc if forced is None else np.asarray(forced[:, k], dtype=np.int64)
        if forced is not None:  # a forced path that stops (-1) or leaves the range stops here
            ok = ok & (s >= 0) & (s < d)
        s = np.where(ok, s, 0)
        qs = q[rows, s]
        ok = ok & (qs > 0)
        if record:
            probs[:, k, :d] = np.where(ok[:, None], q / Ssafe[:, None], np.nan)
            cdf[:, k, :d] = np.where(ok[:, None], C, np.nan)
            s_draw[:, k] = np.where(ok, s_orc, -1)
            u_all[:, k] = u
            S_all[:, k] = np.where(alive, S, np.nan)
        outcomes[:, k] = np.where(ok, s, -1)
        with np.errstate(divide="ignore", invalid="ignore"):
            logp = np.where(ok, logp + np.log(np.where(ok, qs, 1.0)) - np.log(Ssafe), -np.inf)
            scale = np.where(ok, 1.0 / np.sqrt(np.where(ok, qs, 1.0)), 0.0)
        l = W[rows, s, :] * scale[:, None]
        alive = ok
    out = {"outcomes": outcomes, "logp": logp}
    if record:
        out.update(probs=probs, cdf=cdf, s_draw=s_draw, u=u_all, S=S_all)
    return out


def forced_probs(tensors, outcomes: np.ndarray, seed: int, n_offset: int = 0, mps_id: int = 0,
                 n_index: np.ndarray | None = None, displace: np.ndarray | None = None):
    """Conditional probabilities p_k(i | s_0..s_{k-1}) along given outcomes."""
    return sample(tensors, seed, outcomes.shape[0], n_offset=n_offset, mps_id=mps_id,
                  forced=outcomes, n_index=n_index, displace=displace)


# --------------------------------------------------------------------------
# Direct evaluations that do not go through conditionals; used to pin the
# sampler above.
# --------------------------------------------------------------------------

def amplitude_norm2(tensors, s) -> float:
    """|psi(s)|^2 by the plain matrix product A_0[:, s_0, :] ... A_{M-1}[:, s_{M-1}, :].

    With an open right end wider than one (chi_M > 1) the right environment is
    the identity, so the squared norm of the final row vector is returned.
    """
    v = np.ones((1, 1), dtype=np.complex128)
    for A, sk in zip(tensors, s):
        v = v @ np.asarray(A, dtype=np.complex128)[:, int(sk), :]
    return float(np.sum(np.abs(v) ** 2))


def brute_force(tensors) -> tuple[np.ndarray, np.ndarray]:
    """All d_0 x ... x d_{M-1} configurations and their |psi(s)|^2.

    Enumerates configurations explicitly (itertools.product), so it is only
    for tiny chains.
    """
    dims = [t.shape[1] for t in tensors]
    configs = np.array(list(itertools.product(*[range(d) for d in dims])), dtype=np.int32)
    p = np.array([amplitude_norm2(tensors, c) for c in configs])
    return configs, p


def config_index(outcomes: np.ndarray, dims) -> np.ndarray:
    """Mixed-radix index of each configuration row (first site most significant)."""
    idx = np.zeros(outcomes.shape[0], dtype=np.int64)
    for k, d in enumerate(dims):
        idx = idx * d + outcomes[:, k]
    return idx


# --------------------------------------------------------------------------
# Decoders of the compressed storage kinds (the oracle's own code; used to
# evaluate exactly the tensor the sampler sees).
# --------------------------------------------------------------------------

def _e4m3_value(code: np.ndarray) -> np.ndarray:
    """OCP FP8 E4M3: sign bit, 4-bit exponent (bias 7), 3-bit mantissa;
    exponent 0 is subnormal (m/8 * 2^-6); S.1111.111 is NaN."""
    code = np.asarray(code, dtype=np.int64)
    s = np.where(code & 0x80, -1.0, 1.0)
    e = (code >> 3) & 0xF
    m = (code & 0x7).astype(np.float64)
    normal = (1.0 + m / 8.0) * np.exp2(e - 7.0)
    sub = (m / 8.0) * 2.0 ** -6
    v = s * np.where(e == 0, sub, normal)
    return np.where((e == 0xF) & (m == 7), np.nan, v)


def decode_site(raw: np.ndarray, shape, kind: str) -> np.ndarray:
    """complex128 site tensor of the given shape from its stored bytes."""
    chi_l, d, chi_r = shape
    n = chi_l * d * chi_r
    raw = np.asarray(raw, dtype=np.uint8)
    if kind == "c64":
        return raw[:8 * n].view(np.complex64).astype(np.complex128).reshape(shape)
    if kind == "cf16":
        ri = raw[:4 * n].view(np.float16).astype(np.float64).reshape(n, 2)
        return (ri[:, 0] + 1j * ri[:, 1]).reshape(shape)
    if kind == "cf8":
        blk = 128
        codes = raw[:2 * n].reshape(chi_l, d * chi_r, 2)
        off = -(-2 * n // 256) * 256
        nbr, nbc = -(-chi_l // blk), -(-(d * chi_r) // blk)
        scales = raw[off:off + 4 * nbr * nbc].view(np.float32).astype(np.float64).reshape(nbr, nbc)
        sc = np.repeat(np.repeat(scales, blk, axis=0), blk, axis=1)[:chi_l, :d * chi_r]
        re = _e4m3_value(codes[..., 0]) * sc
        im = _e4m3_value(codes[..., 1]) * sc
        return (re + 1j * im).reshape(shape)
    raise ValueError(kind)
