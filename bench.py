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
KERNEL_DIR = os.path.join(ROOT, "paper_2512_20064_amd", "csrc")
# Per form: MFMA peak of its operand type (MI355X, dense), MFMA products per
# algorithmic complex product, the contraction kernel and its source.
FORMS = {
    "fp32": {"peak": 157.3, "mfma_per_alg": 1, "kernel": "contract_f32_kernel", "src": "contract_f32.hip",
             "dtype": "f32"},
    "bf16x3": {"peak": 2516.6, "mfma_per_alg": 3, "kernel": "contract_lp_kernel<bf16,3>", "src": "contract_lp.hip",
               "dtype": "bf16x3"},
    "fp16": {"peak": 2516.6, "mfma_per_alg": 1, "kernel": "contract_lp_kernel<f16,1>", "src": "contract_lp.hip",
             "dtype": "f16"},
}


def kernel_hash(form) -> str:
    src = os.path.join(KERNEL_DIR, FORMS[form]["src"])
    return hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]


def traffic_for(form, chunk):
    """HBM bytes per launch of the contraction from committed counter runs,
    or None if they were taken on another version of the kernel."""
    path = os.path.join(ROOT, "profiles", f"traffic_{form}.json")
    if not os.path.exists(path):
        return None
    tr = json.load(open(path))
    if tr.get("kernel_sha") != kernel_hash(form) or tr.get("chunk") != chunk:
        return None
    return tr.get("bytes_per_launch")


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
    ap.add_argument("--precision", default="fp32", choices=sorted(FORMS))
    ap.add_argument("--beside", default="", help="comma-separated forms also timed (e.g. fp32)")
    ap.add_argument("--beside-steps", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-samples", type=int, default=1024)
    ap.add_argument("--cpu-sites", type=int, default=512)
    ap.add_argument("--no-profile", action="store_true", help="do not event-time each launch")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="also run one plain device copy of this many MiB (reference for HBM counters)")
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

    if args.copy_calibration:
        src = torch.empty(args.copy_calibration * 2**20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        src.fill_(1)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log(f"copy calibration: {args.copy_calibration} MiB device-to-device copy")

    def run_form(form, steps, warmup):
        sampler = mps.Sampler(0, n_chunk=args.chunk, profile=not args.no_profile, precision=form)
        step = [0]

        def one_step():
            r = sampler.sample(dev, args.chunk, seed, n_offset=step[0] * args.chunk, want_logp=True)
            step[0] += 1
            return r

        for w in range(warmup):
            one_step()
            torch.cuda.synchronize()
            log(f"{form} warmup step {w} done")
        torch.cuda.synchronize()
        c_ms = m_ms = p_ms = c_fl = 0.0
        c_n = 0
        t0 = time.perf_counter()
        for s_ in range(steps):
            one_step()
            st = sampler.stats
            c_ms += st.contract_ms
            m_ms += st.measure_ms
            p_ms += st.pack_ms
            c_fl += st.contract_flops
            c_n += st.contract_launches
            log(f"{form} timed step {s_} done")
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        sampler.close()
        out = {"value": args.chunk * M * steps / dt, "ms_per_step": dt / steps * 1e3, "dt": dt}
        if not args.no_profile and c_ms > 0:
            f = FORMS[form]
            alg = (c_fl / c_n) / (c_ms / c_n * 1e-3) / 1e12
            achieved = alg * f["mfma_per_alg"]
            out["roofline"] = {
                "bound": "mfma", "achieved": round(achieved, 2), "peak": f["peak"], "unit": "TFLOP/s",
                "frac": round(achieved / f["peak"], 4), "traffic": traffic_for(form, args.chunk),
                "kernel": f["kernel"], "algorithmic_tflops": round(alg, 2),
                "mfma_products_per_complex_product": f["mfma_per_alg"],
                "avg_launch_ms": round(c_ms / c_n, 4), "launches": c_n,
                "time_share": {"contract": round(c_ms * 1e-3 / dt, 4), "measure": round(m_ms * 1e-3 / dt, 4),
                               "pack": round(p_ms * 1e-3 / dt, 4)},
            }
        return out

    main_res = run_form(args.precision, args.steps, args.warmup)
    value, dt = main_res["value"], main_res["dt"]
    roof = main_res.get("roofline")
    beside = {}
    for form in [f for f in args.beside.split(",") if f and f != args.precision]:
        r = run_form(form, args.beside_steps, 0 if args.beside_steps == 0 else 1)
        beside[form] = {"value": round(r["value"], 1), "ms_per_step": round(r["ms_per_step"], 2),
                        "steps": args.beside_steps,
                        "frac": r.get("roofline", {}).get("frac")}

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on the host")
        cpu = cpu_baseline(t128, seed, args.cpu_samples, min(args.cpu_sites, M))

    rec = {
        "metric": METRIC, "value": round(value, 1), "unit": "site-samples/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt / args.steps * 1e3, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": FORMS[args.precision]["dtype"],
        "data": "synthetic",
        "config": {"workload": wname, "sites": M, "d": 4, "chi": int(max(chi)), "samples_per_step": args.chunk,
                   "precision": args.precision, "tensor_bytes": int(sum(t.numel() * 8 for t in dev))},
        "roofline": roof, "cpu_baseline": cpu,
    }
    if beside:
        rec["beside"] = beside
        if "fp32" in beside:
            rec["speedup_vs_fp32"] = round(value / beside["fp32"]["value"], 3)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
