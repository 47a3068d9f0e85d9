"""Throughput of the MPS sampling sweep on one MI355X.

A step is one chunk of samples (the paper's macro batch) taken through every
site of the chain: contraction, branch weights, normalisation, CDF, draw,
gather and renormalisation at each of the M sites.  Default workload: the
GBS-shaped resident chain, M = 1024 sites, d = 4, chi = 1024 (bond ramp
1, 4, 16, 64, 256 at both open ends), complex64 site tensors resident in HBM
(one device buffer per site, 32 GiB), 65536 samples per step; step s draws
global samples [s*65536, (s+1)*65536) of the N = 2^20 job.

Prints one JSON line: site-samples/s, the contraction kernel against the
FP32 MFMA roofline (event-timed live over the timed region), and the FP64
oracle timed on the host cores on a bounded sample of the same chain.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "site-samples/s at χ=1024,d=4; MFMA util; low-prec vs FP32 at 1e-3 prob err"
PEAK_TFLOPS = {"fp32": 157.3}
KERNEL_SRC = os.path.join(ROOT, "paper_2512_20064_amd", "csrc", "sweep_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "contract_f32_traffic.json")


def kernel_hash() -> str:
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def build_chain(args):
    from paper_2512_20064_amd import synth
    t0 = time.time()
    if args.workload == "resident":
        t128, d, chi = synth.resident_chain(tensor_seed=3, M=args.sites, d=4, chi_max=args.chi, pool=args.pool)
        name = (f"resident chain M={args.sites} d=4 chi={args.chi} (ramp at both ends) complex64, "
                f"{args.chunk} samples per step of an N=2^20 job")
    elif args.workload == "small":
        t128, d, chi = synth.small_chain(1, M=32, d=4, chi_max=32)
        name = "small chain M=32 d=4 chi=32 complex64"
    else:
        raise SystemExit(f"unknown workload {args.workload}")
    t64 = synth.to_c64(t128)
    log(f"generated chain in {time.time() - t0:.1f}s")
    return t128, t64, d, chi, name


def upload(t64):
    """One device buffer per site; pooled host tensors are copied once and
    cloned on the device."""
    import torch
    cache = {}
    dev = []
    for t in t64:
        key = id(t)
        if key not in cache:
            cache[key] = torch.from_numpy(t).to("cuda")
            dev.append(cache[key])
        else:
            dev.append(cache[key].clone())
    torch.cuda.synchronize()
    return dev


def cpu_baseline(t128, seed, n_samples, n_sites):
    """The FP64 oracle as it stands, on n_samples samples over the first n_sites
    sites (a chain window with an open right end)."""
    import oracle
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    window = t128[:n_sites]
    t0 = time.perf_counter()
    oracle.sample(window, seed=seed, N=n_samples)
    dt = time.perf_counter() - t0
    return {"value": n_samples * n_sites / dt, "unit": "site-samples/s", "cores": int(threads),
            "kind": "oracle",
            "sample": f"{n_samples} samples x first {n_sites} sites of the same chain, numpy FP64, {dt:.1f}s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="resident")
    ap.add_argument("--sites", type=int, default=1024)
    ap.add_argument("--chi", type=int, default=1024)
    ap.add_argument("--pool", type=int, default=16)
    ap.add_argument("--chunk", type=int, default=65536)
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-samples", type=int, default=256)
    ap.add_argument("--cpu-sites", type=int, default=96)
    ap.add_argument("--no-profile", action="store_true", help="do not event-time each launch")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build runs on one GPU only; multi-GPU sharding is design-only "
                                   "(samples shard by global index with no exchange)"}), flush=True)
        raise SystemExit(2)

    import torch
    from paper_2512_20064_amd import mps

    if not torch.cuda.is_available():
        raise SystemExit("bench needs a GPU")
    mps.load()
    t128, t64, d, chi, wname = build_chain(args)
    dev = upload(t64)
    M = len(dev)
    seed = 1003
    log(f"uploaded {M} sites, {sum(t.numel() * 8 for t in dev) / 2**30:.1f} GiB")

    sampler = mps.Sampler(0, n_chunk=args.chunk, profile=not args.no_profile)
    stream = torch.cuda.current_stream()
    step = 0

    def one_step():
        nonlocal step
        r = sampler.sample(dev, args.chunk, seed, n_offset=step * args.chunk, want_logp=True)
        step += 1
        return r

    for w in range(args.warmup):
        one_step()
        torch.cuda.synchronize()
        log(f"warmup step {w} done")
    torch.cuda.synchronize()
    c_ms = m_ms = c_fl = 0.0
    c_n = 0
    t0 = time.perf_counter()
    for s in range(args.steps):
        one_step()
        st = sampler.stats
        c_ms += st.contract_ms
        m_ms += st.measure_ms
        c_fl += st.contract_flops
        c_n += st.contract_launches
        log(f"timed step {s} done")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    site_samples = args.chunk * M * args.steps
    value = site_samples / dt

    roof = None
    if not args.no_profile and c_ms > 0:
        achieved = (c_fl / c_n) / (c_ms / c_n * 1e-3) / 1e12
        peak = PEAK_TFLOPS[args.precision]
        traffic = None
        if os.path.exists(TRAFFIC_FILE):
            tr = json.load(open(TRAFFIC_FILE))
            if tr.get("kernel_sha") == kernel_hash() and tr.get("chunk") == args.chunk:
                traffic = tr.get("bytes_per_launch")
        roof = {"bound": "mfma", "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s",
                "frac": round(achieved / peak, 4), "traffic": traffic,
                "kernel": "contract_f32", "avg_launch_ms": round(c_ms / c_n, 4),
                "launches": c_n, "measure_ms_share": round(m_ms / max(c_ms + m_ms, 1e-9), 4)}

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on the host")
        cpu = cpu_baseline(t128, seed, args.cpu_samples, min(args.cpu_sites, M))

    rec = {
        "metric": METRIC, "value": round(value, 1), "unit": "site-samples/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt / args.steps * 1e3, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wname, "sites": M, "d": 4, "chi": int(max(chi)), "samples_per_step": args.chunk,
                   "precision": args.precision, "tensor_bytes": int(sum(t.numel() * 8 for t in dev))},
        "roofline": roof, "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
