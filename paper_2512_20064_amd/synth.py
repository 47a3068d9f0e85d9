"""Seeded synthetic inputs: random right-canonical matrix product states.

This module only builds inputs.  It holds none of the sampling arithmetic
(no contraction, no probabilities, no draws); both the FP64 oracle and the
HIP sampler consume what it returns.

The paper samples MPS produced from Gaussian Boson Sampling data, which are
not available here.  The stand-in keeps their shape (Section 2.2: a chain of
M site tensors, physical dimension d, bond dimension chi, the bond growing
from the open ends, Section 3.4.2) and their decaying photon-number weights:

* G = (N(0,1) + i N(0,1)) / sqrt(2), drawn from PCG64 seeded by
  (tensor_seed, mps_id, k), shape (chi_l, d, chi_r);
* physical slice i is multiplied by exp(-i/2);
* B = Q^H from the reduced QR of G.reshape(chi_l, d*chi_r)^H, with the
  column phases of Q fixed so that diag(R) is real and non-negative (QR is
  unique only up to those phases).

B then has orthonormal rows, i.e. sum_i B_i B_i^H = I (right-canonical form),
which is what the sampler's Lambda-free measurement assumes.

Site tensors are stored as complex arrays of shape (chi_l, d, chi_r):
row-major [left bond][physical][right bond], so each physical branch of a
row is a contiguous run of chi_r complex numbers.
"""
from __future__ import annotations

import numpy as np

# Seed tag that separates pooled plateau tensors from per-site tensors.
_POOL_TAG = 0x504F4F4C


def ramp_bonds(d: list[int], chi_max: int) -> list[int]:
    """Bond dimensions chi_0..chi_M of an open chain with a bond cap.

    chi_k = min(chi_max, prod_{j<k} d_j, prod_{j>=k} d_j): the largest bond a
    right-canonical chain with open ends can carry (a row-orthonormal
    chi_l x d*chi_r matrix needs chi_l <= d*chi_r), capped at chi_max.  This
    is the edge-to-centre growth of Section 3.4.2 in its exact-simulation
    form.
    """
    M = len(d)
    chi = []
    for k in range(M + 1):
        left = 1
        for j in range(k):
            left = min(left * d[j], chi_max)
        right = 1
        for j in range(k, M):
            right = min(right * d[j], chi_max)
        chi.append(min(chi_max, left, right))
    return chi


def _site_from_gaussian(G: np.ndarray) -> np.ndarray:
    chi_l, d, chi_r = G.shape
    G = G * np.exp(-0.5 * np.arange(d))[None, :, None]
    X = G.reshape(chi_l, d * chi_r).conj().T          # (d*chi_r, chi_l)
    Q, R = np.linalg.qr(X, mode="reduced")
    diag = np.diagonal(R)
    ph = np.where(np.abs(diag) > 0, diag / np.where(diag == 0, 1, np.abs(diag)), 1.0)
    Q = Q * ph[None, :]
    return np.ascontiguousarray(Q.conj().T.reshape(chi_l, d, chi_r))


def gaussian_site(seed_words: list[int], chi_l: int, d: int, chi_r: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed_words)))
    shape = (chi_l, d, chi_r)
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (re + 1j * im) / np.sqrt(2.0)


def random_site(tensor_seed: int, mps_id: int, k: int, chi_l: int, d: int, chi_r: int) -> np.ndarray:
    """Right-canonical complex128 site tensor (chi_l, d, chi_r) for site k."""
    if chi_l > d * chi_r:
        raise ValueError(f"chi_l={chi_l} > d*chi_r={d * chi_r}: no right-canonical tensor")
    return _site_from_gaussian(gaussian_site([tensor_seed, mps_id, k], chi_l, d, chi_r))


def random_mps(tensor_seed: int, d: list[int] | int, chi: list[int], M: int | None = None,
               mps_id: int = 0, pool: int = 0) -> list[np.ndarray]:
    """A right-canonical MPS as a list of complex128 (chi_k, d_k, chi_{k+1}) arrays.

    ``pool`` > 0 reuses ``pool`` distinct tensors for every site of a repeated
    (chi_l, d, chi_r) shape: site k takes pooled tensor k mod pool of its shape.
    The chain is still right-canonical; the option only bounds generation time
    and host memory for chains whose distinct tensors would not fit (the list
    holds shared references; callers that need one device buffer per site
    upload each entry separately).
    """
    if isinstance(d, int):
        assert M is not None
        d = [d] * M
    M = len(d)
    assert len(chi) == M + 1
    sites: list[np.ndarray] = []
    cache: dict[tuple, np.ndarray] = {}
    for k in range(M):
        shape = (chi[k], d[k], chi[k + 1])
        if pool > 0:
            key = shape + (k % pool,)
            if key not in cache:
                G = gaussian_site([tensor_seed, mps_id, _POOL_TAG, *shape, k % pool], *shape)
                cache[key] = _site_from_gaussian(G)
            sites.append(cache[key])
        else:
            sites.append(random_site(tensor_seed, mps_id, k, *shape))
    return sites


def canonical_error(B: np.ndarray) -> float:
    """max |sum_i B_i B_i^H - I| for one site tensor (chi_l, d, chi_r)."""
    chi_l = B.shape[0]
    X = B.reshape(chi_l, -1)
    return float(np.max(np.abs(X @ X.conj().T - np.eye(chi_l))))


# --------------------------------------------------------------------------
# Named workloads.  Sizes follow the configurations the sampler is measured
# on; each returns (tensors, d, chi) with tensors in complex128.
# --------------------------------------------------------------------------

def small_chain(tensor_seed: int = 1, M: int = 32, d: int = 4, chi_max: int = 32, mps_id: int = 0):
    """Plain small chain: uniform d, bond cap chi_max, open ends."""
    dl = [d] * M
    chi = ramp_bonds(dl, chi_max)
    return random_mps(tensor_seed, dl, chi, mps_id=mps_id), dl, chi


def resident_chain(tensor_seed: int = 3, M: int = 1024, d: int = 4, chi_max: int = 1024,
                   pool: int = 16, mps_id: int = 0):
    """GBS-shaped resident chain (M=1024, d=4, chi=1024 by default).

    Ramp sites are distinct; the chi_max x d x chi_max plateau cycles over
    ``pool`` distinct tensors (1024 distinct QRs of 4096x1024 would take
    minutes on the host; every site still gets its own device buffer).
    """
    dl = [d] * M
    chi = ramp_bonds(dl, chi_max)
    return random_mps(tensor_seed, dl, chi, mps_id=mps_id, pool=pool), dl, chi


def uneven_chain(tensor_seed: int = 4, M: int = 2048, chi_max: int = 4096, d_lo: int = 2,
                 d_hi: int = 6, pool: int = 4, mps_id: int = 0):
    """Chain with per-site physical dimension d_k ~ U{d_lo..d_hi} and ramped bonds."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([tensor_seed, mps_id, 0xD])))
    dl = [int(x) for x in rng.integers(d_lo, d_hi + 1, size=M)]
    chi = ramp_bonds(dl, chi_max)
    return random_mps(tensor_seed, dl, chi, mps_id=mps_id, pool=pool), dl, chi


def ensemble_specs(seed: int = 2, B: int = 256, M_lo: int = 32, M_hi: int = 512,
                   chis=(16, 32, 64, 128, 256), ds=(2, 3, 4)):
    """(M_b, d_b, chi_max_b) for a batched ensemble of B chains."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 0xE])))
    out = []
    for _ in range(B):
        M = int(rng.integers(M_lo, M_hi + 1))
        chi = int(rng.choice(chis))
        d = int(rng.choice(ds))
        out.append((M, d, chi))
    return out


def to_c64(tensors: list[np.ndarray]) -> list[np.ndarray]:
    """complex64 casts, sharing casts of shared (pooled) arrays."""
    seen: dict[int, np.ndarray] = {}
    out = []
    for t in tensors:
        if id(t) not in seen:
            seen[id(t)] = np.ascontiguousarray(t.astype(np.complex64))
        out.append(seen[id(t)])
    return out


def promote(tensors: list[np.ndarray]) -> list[np.ndarray]:
    """complex128 copies of (e.g. complex64) tensors, sharing shared arrays."""
    seen: dict[int, np.ndarray] = {}
    out = []
    for t in tensors:
        if id(t) not in seen:
            seen[id(t)] = t.astype(np.complex128)
        out.append(seen[id(t)])
    return out


# --------------------------------------------------------------------------
# Compressed storage of site tensors (Section 3.3.2: tensors stored and moved
# in low precision).  These produce input bytes; both the sampler (which
# decodes them on the GPU) and the oracle (which decodes them with its own
# code) consume the same bytes.
#
#   complex-fp16: (re, im) as IEEE binary16, interleaved, 4 bytes per entry.
#   complex-fp8 : (re, im) as OCP FP8 E4M3 codes, interleaved, 2 bytes per
#                 entry, followed (at the next multiple of 256 bytes) by FP32
#                 scales, one per 128 x 128 block of the chi_l x (d*chi_r)
#                 complex matrix, row-major over blocks; an entry decodes to
#                 code_value * scale of its block.  Each scale is the
#                 smallest power of two that brings the block's largest |re|
#                 or |im| to at most 448 (the largest E4M3 value), as the
#                 OCP microscaling formats do: then every decoded value is
#                 exactly representable in binary16 (for scale exponents in
#                 [-15, 7]), which the sampler's fp16 split form exploits.
# --------------------------------------------------------------------------

FP8_BLOCK = 128
E4M3_MAX = 448.0


def fp8_block_scale(amax: float) -> np.float32:
    """Smallest power of two s with amax / s <= 448 (1 for an all-zero block)."""
    if not amax > 0:
        return np.float32(1.0)
    m, e = np.frexp(np.float64(amax) / E4M3_MAX)  # amax / 448 = m 2^e, 0.5 <= m < 1
    return np.float32(np.ldexp(1.0, int(e) - 1 if m == 0.5 else int(e)))


def _e4m3_grid() -> np.ndarray:
    """Values of the 256 E4M3 codes (OCP 8-bit floating point, E4M3): sign,
    4 exponent bits with bias 7, 3 mantissa bits, subnormals, and the single
    NaN pattern S.1111.111 (no infinities)."""
    vals = np.empty(256)
    for c in range(256):
        s = -1.0 if c & 0x80 else 1.0
        e = (c >> 3) & 0xF
        m = c & 0x7
        if e == 0xF and m == 0x7:
            vals[c] = np.nan
        elif e == 0:
            vals[c] = s * (m / 8.0) * 2.0 ** -6
        else:
            vals[c] = s * (1.0 + m / 8.0) * 2.0 ** (e - 7)
    return vals


E4M3_VALUES = _e4m3_grid()


def encode_e4m3(x: np.ndarray) -> np.ndarray:
    """Round float values to the nearest E4M3 code (ties to an even mantissa),
    saturating at +-448."""
    x = np.clip(np.asarray(x, dtype=np.float64), -E4M3_MAX, E4M3_MAX)
    pos = E4M3_VALUES[:0x7F]  # non-negative finite codes 0x00..0x7E, increasing
    a = np.abs(x)
    idx = np.searchsorted(pos, a)  # pos[idx-1] < a <= pos[idx]
    idx = np.clip(idx, 1, len(pos) - 1)
    lo, hi = pos[idx - 1], pos[idx]
    pick_hi = (a - lo > hi - a) | ((a - lo == hi - a) & (idx % 2 == 0))
    code = np.where(pick_hi, idx, idx - 1).astype(np.uint8)
    code = np.where(a == 0, 0, code)
    return np.where(x < 0, code | 0x80, code).astype(np.uint8)


def compress_site(A: np.ndarray, kind: str) -> np.ndarray:
    """Bytes of one site tensor (chi_l, d, chi_r) in the given storage kind."""
    A = np.ascontiguousarray(A.astype(np.complex64))
    if kind == "c64":
        return A.view(np.uint8).reshape(-1).copy()
    if kind == "cf16":
        ri = np.stack([A.real, A.imag], axis=-1).astype(np.float16)
        return ri.view(np.uint8).reshape(-1).copy()
    if kind == "cf8":
        chi_l, d, chi_r = A.shape
        mat = A.reshape(chi_l, d * chi_r)
        nbr, nbc = -(-chi_l // FP8_BLOCK), -(-(d * chi_r) // FP8_BLOCK)
        scales = np.ones((nbr, nbc), dtype=np.float32)
        codes = np.empty((chi_l, d * chi_r, 2), dtype=np.uint8)
        for bi in range(nbr):
            for bj in range(nbc):
                blk = mat[bi * FP8_BLOCK:(bi + 1) * FP8_BLOCK, bj * FP8_BLOCK:(bj + 1) * FP8_BLOCK]
                amax = float(max(np.abs(blk.real).max(), np.abs(blk.imag).max()))
                sc = fp8_block_scale(amax)
                scales[bi, bj] = sc
                sl = (slice(bi * FP8_BLOCK, (bi + 1) * FP8_BLOCK), slice(bj * FP8_BLOCK, (bj + 1) * FP8_BLOCK))
                codes[sl + (0,)] = encode_e4m3(blk.real / np.float64(sc))
                codes[sl + (1,)] = encode_e4m3(blk.imag / np.float64(sc))
        head = codes.reshape(-1)
        off = -(-head.size // 256) * 256
        out = np.zeros(off + scales.size * 4, dtype=np.uint8)
        out[:head.size] = head
        out[off:] = scales.view(np.uint8).reshape(-1)
        return out
    raise ValueError(kind)


def compressed_bytes(chi_l: int, d: int, chi_r: int, kind: str) -> int:
    n = chi_l * d * chi_r
    if kind == "c64":
        return 8 * n
    if kind == "cf16":
        return 4 * n
    nb = -(-chi_l // FP8_BLOCK) * -(-(d * chi_r) // FP8_BLOCK)
    return -(-2 * n // 256) * 256 + 4 * nb


# --------------------------------------------------------------------------
# Large-bond workloads (chi in the thousands).  A QR of a chi x d*chi matrix
# per distinct tensor takes minutes to hours on the host at these sizes, so
# these tensors are built directly with orthonormal rows, on any torch
# device, from discrete Fourier rows with random phases:
#
# * chi_l <= chi_r: the bonds are cut into nb equal blocks (nb = 4 when both
#   bonds are multiples of 4 and chi_l >= 64, else 1).  Branch i maps left
#   block a to right block (a + i) mod nb with weight T[a][i] = c_{(a+i) mod d}^2,
#   c_i proportional to exp(-i/2) with sum_i c_i^2 = 1 (the decaying
#   photon-number profile, cyclically shifted per block):
#       B[L_a, i, R_(a+i)%nb] = sqrt(T[a][i]) diag(e^{i alpha}) F[:|L_a|, :] diag(e^{i beta}),
#   F the unitary DFT of the block size.  For every i the map a -> (a+i) mod nb
#   is a permutation, so rows of different left blocks never meet in one
#   right block, and within a block sum_i T[a][i] = 1: sum_i B_i B_i^H = I.
#   A left vector inside block a has conditionals T[a][.] exactly, and the
#   chosen branch moves it to another block, so the conditionals depend on
#   the prefix (a hidden Markov chain over the blocks).
# * chi_l > chi_r (right end of a ramp, chi_l <= d*chi_r):
#   B.reshape(chi_l, d*chi_r) = diag(e^{i alpha}) F[:chi_l, :] diag(e^{i beta}),
#   F the unitary DFT of size d*chi_r.
# * Then every column r of the right bond mixes the d branches with its own
#   d x d unitary V_r (the Q of I + 0.3 G_r, G_r complex Gaussian, diag(R)
#   made real and positive): B'[l, i, r] = sum_j B[l, j, r] V_r[j, i].  The
#   reshaped rows stay orthonormal (block-diagonal unitary on the right), and
#   the branch weights now also depend on how the left vector spreads over
#   the columns, not only on its block.
#
# The phases and mixers come from PCG64 seeded like the Gaussian sites, so a
# tensor is the same on every device up to the rounding of its evaluation.
# --------------------------------------------------------------------------

MIX_THETA = 0.3
HMM_BLOCKS = 4


def _dft_rows(torch, rows: int, n: int, pa, pb, device):
    """diag(e^{i pa}) F_n[:rows, :] diag(e^{i pb}) as complex64 (rows x n)."""
    import math
    r = torch.arange(rows, device=device, dtype=torch.int64)
    c = torch.arange(n, device=device, dtype=torch.int64)
    ang = torch.remainder(r[:, None] * c[None, :], n).to(torch.float64) * (-2.0 * math.pi / n)
    ang += torch.as_tensor(pa, device=device)[:, None]
    ang += torch.as_tensor(pb, device=device)[None, :]
    mag = torch.full_like(ang, 1.0 / math.sqrt(n))
    return torch.polar(mag, ang).to(torch.complex64)


def structured_blocks(chi_l: int, chi_r: int) -> int:
    """Number of bond blocks of a structured site with chi_l <= chi_r."""
    ok = chi_l >= 16 * HMM_BLOCKS and chi_l % HMM_BLOCKS == 0 and chi_r % HMM_BLOCKS == 0
    return HMM_BLOCKS if ok else 1


def structured_weights(d: int, nb: int) -> np.ndarray:
    """T[a][i]: weight of branch i for a left vector in block a (rows sum to 1)."""
    c = np.exp(-0.5 * np.arange(d))
    c2 = c * c / np.sum(c * c)
    return np.array([[c2[(a + i) % d] for i in range(d)] for a in range(nb)])


def branch_mixers(seed_words: list[int], chi_r: int, d: int, theta: float = MIX_THETA) -> np.ndarray:
    """V[r] (chi_r, d, d): per-column unitaries near the identity."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(w) for w in seed_words] + [0x313])))
    G = (rng.standard_normal((chi_r, d, d)) + 1j * rng.standard_normal((chi_r, d, d))) / np.sqrt(2.0)
    Q, R = np.linalg.qr(np.eye(d)[None] + theta * G)
    dg = np.diagonal(R, axis1=1, axis2=2)
    return Q * (dg / np.abs(dg))[:, None, :]


def structured_site(seed_words: list[int], chi_l: int, d: int, chi_r: int, device="cpu", mix: bool = True):
    """Right-canonical complex64 torch tensor (chi_l, d, chi_r) without a QR
    (construction above; mix=False leaves out the per-column mixers)."""
    import torch
    assert chi_l <= d * chi_r
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(w) for w in seed_words] + [0x5D])))
    two_pi = 2.0 * np.pi
    if chi_l <= chi_r:
        nb = structured_blocks(chi_l, chi_r)
        bl, br = chi_l // nb, chi_r // nb
        T = structured_weights(d, nb)
        out = torch.zeros((chi_l, d, chi_r), dtype=torch.complex64, device=device)
        for a in range(nb):
            for i in range(d):
                b = (a + i) % nb
                pa = rng.uniform(0, two_pi, bl)
                pb = rng.uniform(0, two_pi, br)
                blk = _dft_rows(torch, bl, br, pa, pb, device) * float(np.sqrt(T[a, i]))
                out[a * bl:(a + 1) * bl, i, b * br:(b + 1) * br] = blk
    else:
        pa = rng.uniform(0, two_pi, chi_l)
        pb = rng.uniform(0, two_pi, d * chi_r)
        out = _dft_rows(torch, chi_l, d * chi_r, pa, pb, device).reshape(chi_l, d, chi_r)
    if not mix or d == 1:
        return out.contiguous()
    V = torch.as_tensor(branch_mixers(seed_words, chi_r, d).astype(np.complex64), device=device)
    mixed = torch.zeros_like(out)
    for i in range(d):
        for j in range(d):
            mixed[:, i, :] += out[:, j, :] * V[:, j, i][None, :]
    return mixed


def structured_chain(tensor_seed: int, d: list[int], chi_max: int, pool: int = 4, device="cpu"):
    """Chain of structured sites with ramped bonds; a repeated shape cycles
    over ``pool`` distinct tensors (shared references).  Returns
    (tensors, chi)."""
    chi = ramp_bonds(d, chi_max)
    cache: dict[tuple, object] = {}
    sites = []
    for k in range(len(d)):
        shape = (chi[k], d[k], chi[k + 1])
        key = shape + (k % pool,)
        if key not in cache:
            cache[key] = structured_site([tensor_seed, _POOL_TAG, *key], *shape, device=device)
        sites.append(cache[key])
    return sites, chi


def compress_site_torch(A, kind: str):
    """compress_site for a complex64 torch tensor on any device (same bytes:
    binary16 by torch's round-to-nearest-even cast, E4M3 by the same
    nearest-even search over the code values as encode_e4m3, the same
    power-of-two block scales)."""
    import torch
    A = A.contiguous()
    chi_l, d, chi_r = A.shape
    ri = torch.view_as_real(A)
    if kind == "c64":
        return ri.reshape(-1).view(torch.uint8).clone()
    if kind == "cf16":
        return ri.to(torch.float16).reshape(-1).view(torch.uint8).clone()
    if kind != "cf8":
        raise ValueError(kind)
    ncol = d * chi_r
    mat = ri.reshape(chi_l, ncol, 2)
    nbr, nbc = -(-chi_l // FP8_BLOCK), -(-ncol // FP8_BLOCK)
    n = chi_l * ncol
    off = -(-2 * n // 256) * 256
    out = torch.zeros(off + 4 * nbr * nbc, dtype=torch.uint8, device=A.device)
    codes = out[:2 * n].view(chi_l, ncol, 2)
    scales = torch.empty((nbr, nbc), dtype=torch.float32, device=A.device)
    pos = torch.as_tensor(E4M3_VALUES[:0x7F], device=A.device)
    for bi in range(nbr):
        rows = slice(bi * FP8_BLOCK, min(chi_l, (bi + 1) * FP8_BLOCK))
        slab = mat[rows]                                         # (r, ncol, 2)
        r = slab.shape[0]
        padc = nbc * FP8_BLOCK - ncol
        amax = torch.nn.functional.pad(slab.abs().amax(dim=2), (0, padc)).view(r, nbc, FP8_BLOCK).amax(dim=(0, 2))
        m, e = torch.frexp(amax.to(torch.float64) / E4M3_MAX)
        e = torch.where(m == 0.5, e - 1, e)
        sc = torch.where(amax > 0, torch.ldexp(torch.ones_like(m), e).to(torch.float32), torch.ones_like(amax))
        scales[bi] = sc
        scol = sc.repeat_interleave(FP8_BLOCK)[:ncol].to(torch.float64)
        x = torch.clamp(slab.to(torch.float64) / scol[None, :, None], -E4M3_MAX, E4M3_MAX)
        a = x.abs()
        idx = torch.clamp(torch.searchsorted(pos, a), 1, pos.numel() - 1)
        lo, hi = pos[idx - 1], pos[idx]
        pick_hi = (a - lo > hi - a) | ((a - lo == hi - a) & (idx % 2 == 0))
        code = torch.where(pick_hi, idx, idx - 1)
        code = torch.where(a == 0, torch.zeros_like(code), code)
        code = torch.where(x < 0, code | 0x80, code)
        codes[rows] = code.to(torch.uint8)
    out[off:] = scales.reshape(-1).view(torch.uint8)
    return out
