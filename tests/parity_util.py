"""Helpers for comparing the HIP sweep with the FP64 oracle (forced-prefix protocol).

The GPU path and the oracle are run on the same complex64 tensor bytes (the
oracle promotes them to complex128).  A single draw that lands on the other
side of a CDF boundary would make the rest of a sample's chain diverge, so the
comparison follows the GPU's own path: the oracle evaluates the conditional
probabilities p_k(i | s_0..s_{k-1}) along the GPU outcomes and makes its own
draw at every site from the same uniform.

Bars (FP32 contraction):
  * uniforms bit-identical (both sides implement Philox4x64-10 from its
    definition);
  * |p_gpu - p_orc| <= eps_p = 1e-5 for every emitted (row, site, branch);
  * s_gpu == s_orc at every (row, site) whose uniform is farther than
    tau = d * eps_p from every oracle CDF value C_j, j < d-1 (the CDF error
    is at most the sum of the branch errors); in-band draws are counted;
  * |logp_gpu - sum_k ln p_orc(s_k)| <= sum_k eps_p / p_orc(s_k) + 1e-9
    (first-order error of ln p at each site).
"""
from __future__ import annotations

import numpy as np

import oracle
from paper_2512_20064_amd import synth

EPS_FP32 = 1e-5  # conditional-probability bar, FP32 contraction
EPS_LOWP = 1e-3  # conditional-probability bar, 16-bit split forms


def upload(tensors_c64, device="cuda"):
    import torch
    out = []
    for t in tensors_c64:
        out.append(torch.from_numpy(np.ascontiguousarray(t)).to(device))
    return out


def compare(tensors_c64, seed, gpu, rows=None, n_offset=0, eps=EPS_FP32, mps_id=0, n_index=None, displace=None,
            check_logp=True):
    """Forced-prefix comparison of a GPU result dict with the oracle.

    gpu: dict with numpy 'outcomes' [N, M], 'logp' [N], optional 'probs'
    [E, M, dmax] and 'u' [E, M] for the first E rows.  rows: which rows to
    check (default all); n_index: their global sample indices (default
    n_offset + rows); check_logp=False skips the logp bar (when only a prefix
    of the chain's sites is compared).  Returns a report dict; raises
    AssertionError on a violated bar.
    """
    outc = gpu["outcomes"]
    N, M = outc.shape
    if rows is None:
        rows = np.arange(N)
    rows = np.asarray(rows)
    t128 = synth.promote(tensors_c64)
    if n_index is None:
        n_index = n_offset + rows
    disp = None if displace is None else np.asarray(displace, dtype=np.complex128)[rows]
    f = oracle.forced_probs(t128, outc[rows], seed, mps_id=mps_id, n_index=np.asarray(n_index), displace=disp)
    d = np.array([t.shape[1] for t in tensors_c64])
    rep = {"rows": int(len(rows)), "sites": int(M)}

    # uniforms and probabilities from the debug emits, where present
    if "u" in gpu and gpu["u"] is not None:
        E = gpu["u"].shape[0]
        sel = rows < E
        if sel.any():
            assert np.array_equal(gpu["u"][rows[sel]], f["u"][sel]), "uniform streams differ"
            pg = gpu["probs"][rows[sel]]
            po = f["probs"][sel]
            dm = min(pg.shape[2], po.shape[2])
            diff = np.abs(pg[:, :, :dm] - po[:, :, :dm])
            valid = ~np.isnan(po[:, :, :dm])
            err = diff[valid]
            rep["prob_err_max"] = float(err.max()) if err.size else 0.0
            rep["prob_err_mean"] = float(err.mean()) if err.size else 0.0
            rep["prob_err_p999"] = float(np.quantile(err, 0.999)) if err.size else 0.0
            per_site = np.nanmax(np.where(valid, diff, np.nan), axis=(0, 2))
            rep["prob_err_worst_site"] = int(np.nanargmax(per_site))
            if per_site.size >= 8:  # growth along the chain: max error per eighth of the sites
                rep["prob_err_by_eighth"] = [float(np.nanmax(c)) for c in np.array_split(per_site, 8)]
            assert not np.isnan(diff[valid]).any(), "NaN probability on the GPU"
            assert rep["prob_err_max"] <= eps, rep

    # draws: equal outside the boundary band
    u = f["u"]
    C = f["cdf"]
    s_gpu = outc[rows]
    s_orc = f["s_draw"]
    tau = d[None, :] * eps
    dist = np.full(u.shape, np.inf)
    for j in range(C.shape[2] - 1):
        cj = C[:, :, j]
        inner = j < (d - 1)[None, :]
        dj = np.where(inner & ~np.isnan(cj), np.abs(u - cj), np.inf)
        dist = np.minimum(dist, dj)
    band = dist <= tau
    live = s_gpu >= 0
    mism = (s_gpu != s_orc) & live
    rep["in_band_draws"] = int((band & live).sum())
    rep["in_band_mismatches"] = int((mism & band).sum())
    rep["out_of_band_mismatches"] = int((mism & ~band).sum())
    assert rep["out_of_band_mismatches"] == 0, rep

    if not check_logp:  # e.g. a prefix of the chain: the GPU's logp covers every site
        return rep
    # logp along the GPU path
    p_path = np.take_along_axis(f["probs"], np.maximum(s_gpu, 0)[:, :, None], axis=2)[:, :, 0]
    lp_orc = np.sum(np.log(p_path), axis=1)
    bound = np.sum(eps / p_path, axis=1) + 1e-9
    lg = gpu["logp"][rows]
    whole = np.all(s_gpu >= 0, axis=1)
    dl = np.abs(lg - lp_orc)[whole]
    rep["logp_err_max"] = float(dl.max()) if dl.size else 0.0
    assert np.all(dl <= bound[whole]), (rep, float((dl - bound[whole]).max()))
    return rep
