"""Throughput of the MPS sampling sweep on one MI355X.

A step is one chunk of samples (the paper's macro batch) taken through every
site of the chain: contraction, branch weights, normalisation, CDF, draw,
gather and renormalisation at each of the M sites.  Default workload: the
GBS-shaped resident chain, M = 1024 sites, d = 4, chi = 1024 (bond ramp
1, 4, 16, 64, 256 at both open ends), complex64 site tensors resident in HBM
(one device buffer per site, 32 GiB), 65536 samples per step; step s draws
global samples [s*65536, (s+1)*65536) of the N = 2^20 job.

Prints one JSON line: site-samples/s of the low-precision headline form
(fp16f6: the fp16 product of the high parts plus both correction products in
FP6 E2M3 with per-record power-of-two scales, within 1e-3 of the FP64
oracle), the contraction kernel against the MFMA roofline of its operand
type (event-timed live over the timed region; algorithmic flops, with the
issued MFMA rate in fp16-product equivalents beside), the fp16f8, bf16x3 and
plain FP32 forms timed beside it, and the FP64 oracle timed on the host
cores on a bounded sample of the same chain.

Other workloads (one JSON line each, not the headline):
  --workload uneven   M = 2048, d_k in {2..6}, chi_k = min(prod d, 4096),
                      structured right-canonical sites on the device
                      (repeated shapes share a device buffer);
  --workload batch    256 independent chains (M in [32, 512], chi in
                      {16..256}, d in {2, 3, 4}), N = 8192 each: one batched
                      call against one call per chain;
  --workload stream   a 64-site window at chi = 10^4, d = 4, site tensors in
                      pinned host memory compressed to complex-fp16 (or fp8
                      with 128 x 128 block scales), copied on a side stream
                      while the previous site computes: per-site time, H2D
                      GB/s and the copy/compute overlap.
  --displace SIGMA    (resident, uneven, small) per-sample displacement of
                      the physical index (the GBS variant, Eq. 7), complex
                      Gaussian of scale SIGMA; the oracle baseline is
                      displaced the same way.
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
    "fp16x3": {"peak": 2516.6, "mfma_per_alg": 3, "kernel": "contract_lp_kernel<f16,3>", "src": "contract_lp.hip",
               "dtype": "f16x3"},
    # one fp16 product plus two FP8 products at twice the fp16 rate: two
    # fp16-product equivalents of MFMA time per complex product
    "fp16f8": {"peak": 2516.6, "mfma_per_alg": 2, "kernel": "contract_f16f8_wide", "src": "contract_lp.hip",
               "dtype": "f16+f8"},
    # the same with the two correction products in FP6 at four times the
    # fp16 rate: 1.5 fp16-product equivalents
    "fp16f6": {"peak": 2516.6, "mfma_per_alg": 1.5, "kernel": "contract_f16f6_wide", "src": "contract_lp.hip",
               "dtype": "f16+f6"},
}


def kernel_hash(form) -> str:
    src = os.path.join(KERNEL_DIR, FORMS[form]["src"])
    return hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]


def traffic_for(form, chunk, chi):
    """HBM bytes per launch of the contraction from committed counter runs,
    or None if they were taken on another version of the kernel or another
    launch shape (chunk rows, bond dimension)."""
    path = os.path.join(ROOT, "profiles", f"traffic_{form}.json")
    if not os.path.exists(path):
        return None
    tr = json.load(open(path))
    if tr.get("kernel_sha") != kernel_hash(form) or tr.get("chunk") != chunk or tr.get("chi") != chi:
        return None
    return tr.get("bytes_per_launch")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def build_chain(args):
    """(t128 or None, device-ready complex64 tensors, d, chi, name)."""
    from paper_2512_20064_amd import synth
    t0 = time.time()
    t128 = None
    if args.workload == "resident":
        t128, d, chi = synth.resident_chain(tensor_seed=3, M=args.sites, d=4, chi_max=args.chi, pool=args.pool)
        name = (f"resident chain M={args.sites} d=4 chi={args.chi} (ramp at both ends) complex64, "
                f"{args.chunk} samples per step of an N=2^20 job")
        t64 = synth.to_c64(t128)
    elif args.workload == "small":
        t128, d, chi = synth.small_chain(1, M=32, d=4, chi_max=32)
        name = "small chain M=32 d=4 chi=32 complex64"
        t64 = synth.to_c64(t128)
    elif args.workload == "uneven":
        rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([4, 0, 0xD])))
        d = [int(x) for x in rng.integers(2, 7, size=args.sites)]
        t64, chi = synth.structured_chain(4, d, args.chi, pool=2, device="cuda")
        name = (f"uneven chain M={args.sites} d_k~U{{2..6}} chi_k=min(prod d, {args.chi}) structured "
                f"right-canonical complex64 (repeated shapes share a device buffer), "
                f"{args.chunk} samples per step of an N=2^22 job")
    else:
        raise SystemExit(f"unknown workload {args.workload}")
    log(f"generated chain in {time.time() - t0:.1f}s")
    return t128, t64, d, chi, name


def tile_summary(choices, chains, seconds):
    """Per-shape tile choices of mps_autotune_tiles, with the number of sites
    of each shape (from the device tensors, one chain or a list of chains)
    and the estimated contraction time saved over the wide tile."""
    lists = chains if chains and isinstance(chains[0], (list, tuple)) else [chains]
    count = {}
    for c in lists:
        for t in c:
            sh = (int(t.shape[0]), int(t.shape[1]), int(t.shape[2]))
            count[sh] = count.get(sh, 0) + 1
    rows, wide, chosen = [], 0.0, 0.0
    for c in choices:
        n = count.get((c["chi_l"], c["d"], c["chi_r"]), 0)
        wide += n * c["ms_wide"]
        chosen += n * (c["ms_narrow"] if c["tile"] else c["ms_wide"])
        rows.append([c["chi_l"], c["d"], c["chi_r"], n, "narrow" if c["tile"] else "wide",
                     round(c["ms_wide"], 4), round(c["ms_narrow"], 4)])
    rows.sort(key=lambda r: -r[3] * max(r[5], r[6]))
    return {"shapes": len(choices), "narrow": sum(1 for c in choices if c["tile"]),
            "est_contract_ms_wide": round(wide, 2), "est_contract_ms_chosen": round(chosen, 2),
            "est_gain": round(wide / chosen, 4) if chosen > 0 else None, "tune_seconds": round(seconds, 1),
            "by_shape (chi_l, d, chi_r, sites, tile, ms wide, ms narrow; heaviest first)": rows[:24]}


def upload(t64, share=False):
    """One device buffer per site (pooled host tensors are copied once and
    cloned on the device), or, with share=True or device inputs, one buffer
    per distinct tensor."""
    import torch
    cache = {}
    dev = []
    for t in t64:
        key = id(t)
        if key not in cache:
            cache[key] = t if isinstance(t, torch.Tensor) else torch.from_numpy(t).to("cuda")
            dev.append(cache[key])
        else:
            dev.append(cache[key] if (share or isinstance(t, torch.Tensor)) else cache[key].clone())
    torch.cuda.synchronize()
    return dev


def distinct_bytes(dev):
    return int(sum(t.numel() * t.element_size() for t in {id(t): t for t in dev}.values()))


def host_info():
    """nproc, CPU model and the BLAS library numpy runs on (threadpoolctl)."""
    info = {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "cpu_model": None, "blas": None}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    info["cpu_model"] = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        from threadpoolctl import threadpool_info
        blas = [p for p in threadpool_info() if p.get("user_api") == "blas"]
        if blas:
            b = blas[0]
            info["blas"] = {"library": b.get("internal_api"), "version": b.get("version"),
                            "threads": b.get("num_threads"), "arch": b.get("architecture"),
                            "file": os.path.basename(b.get("filepath", ""))}
    except Exception:
        pass
    return info


def _oracle_rate(tensors, seed, n_samples, threads=None, displace=None):
    """site-samples/s of the FP64 oracle on samples 0 .. n_samples-1 of a chain
    (window with an open right end), with the BLAS thread count limited to
    `threads` (None: as configured); displace: complex [n_samples, sites]
    per-sample displacements, or None."""
    import oracle
    from threadpoolctl import threadpool_limits, threadpool_info
    with threadpool_limits(limits=threads, user_api="blas"):
        used = max([p.get("num_threads", 1) for p in threadpool_info() if p.get("user_api") == "blas"] or [1])
        t0 = time.perf_counter()
        oracle.sample(tensors, seed=seed, N=n_samples, displace=displace)
        dt = time.perf_counter() - t0
    return n_samples * len(tensors) / dt, dt, int(used)


def cpu_baseline(t128, seed, n_samples, n_sites, n_samples_1t, mu=None):
    """The FP64 oracle as it stands, timed on the host cores.

    value: all BLAS threads, samples 0 .. n_samples-1 (global indices) over
    the first n_sites sites of the benchmarked chain (the 5 ramp sites and
    the plateau after them).  Beside it: the same sites single-threaded on
    n_samples_1t samples, and the small parity chain (M = 32, d = 4,
    chi = 32, N = 4096) in full at both thread counts.  mu: the benchmark's
    per-sample displacements (complex [samples, M]) when it runs displaced;
    the chain legs then take the same displacements."""
    import numpy  # noqa: F401  (loads the BLAS that threadpoolctl reports)
    from paper_2512_20064_amd import synth
    hi = host_info()
    window = t128[:n_sites]
    mu_w = None if mu is None else mu[:, :n_sites]
    v, dt, used = _oracle_rate(window, seed, n_samples, displace=None if mu_w is None else mu_w[:n_samples])
    v1, dt1, _ = _oracle_rate(window, seed, n_samples_1t, threads=1,
                              displace=None if mu_w is None else mu_w[:n_samples_1t])
    small = synth.small_chain(1, M=32, d=4, chi_max=32)[0]
    vs, dts, _ = _oracle_rate(small, 1001, 4096)
    vs1, dts1, _ = _oracle_rate(small, 1001, 4096, threads=1)
    return {"value": v, "unit": "site-samples/s", "cores": used, "kind": "oracle",
            "sample": (f"global samples 0..{n_samples - 1} x first {n_sites} sites of the benchmarked chain "
                       f"(ramp 1,4,16,64,256 then chi=1024 plateau){'' if mu is None else ', displaced'}, "
                       f"numpy FP64 with {used} BLAS threads, {dt:.1f}s"),
            "single_thread": {"value": v1, "unit": "site-samples/s", "cores": 1,
                              "sample": f"global samples 0..{n_samples_1t - 1} x the same {n_sites} sites, "
                                        f"{dt1:.1f}s"},
            "small_chain_full": {"workload": "M=32 d=4 chi=32 N=4096 (whole job)", "unit": "site-samples/s",
                                 "value": vs, "cores": used, "seconds": round(dts, 2),
                                 "single_thread_value": vs1, "single_thread_seconds": round(dts1, 2)},
            "host": hi}


HBM_PEAK_GBS = 8000.0


def roofline_of(form, c_fl, c_n, c_ms, dt, m_ms, p_ms, chunk, chi, products=None, m_bytes=None, m_n=None,
                m_kernel="measure_rows_kernel"):
    """Roofline of the contraction kernel: algorithmic flops (8 d chi_l chi_r
    per site-sample, the complex contraction itself) per launch over the
    event-timed average launch, against the dense MFMA peak of the operand
    type.  A split form issues mfma_per_alg MFMA products per complex
    product; its issued MFMA rate is reported beside (mfma_issued), not as
    the achieved figure.  With m_bytes and m_n (the library's algorithmic
    bytes of the measurement launches and their count) the HBM-bound
    measurement kernel's rate against the HBM peak is reported beside."""
    f = FORMS[form]
    products = products or f["mfma_per_alg"]
    alg = (c_fl / c_n) / (c_ms / c_n * 1e-3) / 1e12
    issued = alg * products
    extra = {}
    if m_bytes and m_n and m_ms > 0:
        gbs = m_bytes / (m_ms * 1e-3) / 1e9
        extra["measure"] = {"bound": "hbm", "kernel": m_kernel, "achieved": round(gbs, 1),
                            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                            "bytes_per_launch": round(m_bytes / m_n), "avg_launch_ms": round(m_ms / m_n, 4),
                            "launches": m_n}
    return {
        "bound": "mfma", "achieved": round(alg, 2), "peak": f["peak"], "unit": "TFLOP/s",
        "frac": round(alg / f["peak"], 4), "traffic": traffic_for(form, chunk, chi),
        "kernel": f["kernel"] if products == f["mfma_per_alg"] else f["kernel"].replace(",3>", f",{products}>"),
        "alg_flops_per_launch": round(c_fl / c_n),
        "mfma_issued": {"tflops": round(issued, 2), "frac": round(issued / f["peak"], 4),
                        "products_per_complex_product": products},
        "avg_launch_ms": round(c_ms / c_n, 4), "launches": c_n,
        "time_share": {"contract": round(c_ms * 1e-3 / dt, 4), "measure": round(m_ms * 1e-3 / dt, 4),
                       "pack": round(p_ms * 1e-3 / dt, 4)},
        **extra,
    }


def roofline_small(f_fl, f_n, f_ms, dt):
    """Roofline of the persistent small-bond kernel (the whole sweep of chains
    with bonds <= 32 in one launch per chunk): algorithmic flops of its FP32
    contractions over the event-timed launch, against the FP32 MFMA peak.
    The kernel is latency-bound at these sizes, so the fraction is low."""
    alg = (f_fl / f_n) / (f_ms / f_n * 1e-3) / 1e12
    return {"bound": "mfma", "achieved": round(alg, 3), "peak": 157.3, "unit": "TFLOP/s",
            "frac": round(alg / 157.3, 5), "traffic": None, "kernel": "sweep_small_kernel",
            "alg_flops_per_launch": round(f_fl / f_n), "avg_launch_ms": round(f_ms / f_n, 4), "launches": f_n,
            "time_share": {"sweep_small": round(f_ms * 1e-3 / dt, 4)}}


def check_one_gpu(args):
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build runs on one GPU only; multi-GPU sharding is design-only "
                                   "(samples shard by global index with no exchange)"}), flush=True)
        raise SystemExit(2)


def run_chain_bench(args):
    import torch
    from paper_2512_20064_amd import mps

    t128, t64, d, chi, wname = build_chain(args)
    dev = upload(t64, share=args.workload == "uneven")
    del t64
    M = len(dev)
    seed = 1003
    log(f"{M} sites on the device, {distinct_bytes(dev) / 2**30:.1f} GiB")

    if args.copy_calibration:
        src = torch.empty(args.copy_calibration * 2**20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        src.fill_(1)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log(f"copy calibration: {args.copy_calibration} MiB device-to-device copy")

    tuned = {}
    tiles = {}
    mu = None
    # the displaced measurement keeps a sample's rows in registers for
    # d <= 4 and bonds <= 1024 (two waves per sample), else one wave per sample
    dl = d if isinstance(d, (list, tuple)) else [d] * M
    disp_kernel = ("measure_disp_pair_kernel" if max(dl) <= 4 and max(chi) <= 1024
                   else "measure_disp_kernel")
    if args.displace > 0:
        # per-sample displacements of the GBS variant (complex Gaussian, each
        # component of standard deviation sigma / sqrt(2)), one row per
        # sample of a step, drawn once outside the timed region and reused
        # for every step
        g = torch.Generator(device="cuda")
        g.manual_seed(77)
        mu = (torch.randn(args.chunk, M, 2, generator=g, device="cuda") * (args.displace / 2 ** 0.5))
        mu = torch.view_as_complex(mu).contiguous()
        log(f"displacements: sigma {args.displace}, {mu.numel() * 8 / 2**20:.0f} MiB")

    def run_form(form, steps, warmup):
        sampler = mps.Sampler(0, n_chunk=args.chunk, profile=not args.no_profile, precision=form,
                              graph=args.graph)
        if args.tile_tune:
            # contraction tile per distinct site shape at this chunk (outside
            # the timed region; bit-identical whatever it picks)
            t0 = time.perf_counter()
            ch = sampler.autotune_tiles(dev, args.chunk)
            tiles[form] = tile_summary(ch, dev, time.perf_counter() - t0)
            log(f"{form} tiles: {tiles[form]['narrow']} of {tiles[form]['shapes']} shapes narrow")
        if args.autotune:
            # tile order (and chunk, capped at the step size) for this chain and
            # form; tuning time is outside the timed region
            t0 = time.perf_counter()
            rep = sampler.autotune(dev, args.chunk, seed=seed)
            sampler.opt.n_chunk = args.chunk  # one launch sequence per step, as profiled
            tuned[form] = {"tile_group": rep["tile_group"], "probe_best_chunk": rep["n_chunk"],
                           "probe_sites": rep["probe_sites"], "candidates": rep["candidates"],
                           "gain_vs_default": round(rep["rate"] / rep["default_rate"], 4) if rep["default_rate"] else None,
                           "seconds": round(time.perf_counter() - t0, 1)}
            log(f"{form} autotune: {tuned[form]}")
        step = [0]
        # graph capture needs a stream of its own (not the legacy null stream)
        gstream = torch.cuda.Stream() if args.graph else None

        def one_step():
            r = sampler.sample(dev, args.chunk, seed, n_offset=step[0] * args.chunk, want_logp=True,
                               stream=gstream, displace=mu)
            step[0] += 1
            return r

        for w in range(warmup):
            one_step()
            torch.cuda.synchronize()
            log(f"{form} warmup step {w} done")
        torch.cuda.synchronize()
        c_ms = m_ms = p_ms = c_fl = f_ms = f_fl = m_b = 0.0
        c_n = f_n = m_n = 0
        t0 = time.perf_counter()
        for s_ in range(steps):
            one_step()
            st = sampler.stats
            c_ms += st.contract_ms
            m_ms += st.measure_ms
            m_b += st.measure_bytes
            m_n += st.measure_launches
            p_ms += st.pack_ms
            c_fl += st.contract_flops
            c_n += st.contract_launches
            f_ms += st.fused_ms
            f_fl += st.fused_flops
            f_n += st.fused_launches
            log(f"{form} timed step {s_} done")
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        sampler.close()
        out = {"value": args.chunk * M * steps / dt, "ms_per_step": dt / steps * 1e3, "dt": dt,
               "alg_tflops": (c_fl + f_fl) / dt / 1e12}
        if not args.no_profile and c_ms > 0:
            out["roofline"] = roofline_of(form, c_fl, c_n, c_ms, dt, m_ms, p_ms, args.chunk, args.chi,
                                          m_bytes=m_b, m_n=m_n,
                                          m_kernel=disp_kernel if mu is not None else "measure_rows_kernel")
        elif not args.no_profile and f_ms > 0:
            out["roofline"] = roofline_small(f_fl, f_n, f_ms, dt)
        return out

    main_res = run_form(args.precision, args.steps, args.warmup)
    value, dt = main_res["value"], main_res["dt"]
    roof = main_res.get("roofline")
    beside = {}
    for form in [f for f in args.beside.split(",") if f and f != args.precision]:
        r = run_form(form, args.beside_steps, 0 if args.beside_steps == 0 else 1)
        beside[form] = {"value": round(r["value"], 1), "ms_per_step": round(r["ms_per_step"], 2),
                        "steps": args.beside_steps,
                        "frac": r.get("roofline", {}).get("frac"),
                        "mfma_issued_frac": r.get("roofline", {}).get("mfma_issued", {}).get("frac")}

    cpu = None
    if not args.no_cpu_baseline and t128 is not None:
        log("timing the FP64 oracle on the host")
        mu_host = None
        if mu is not None:
            rows = min(max(args.cpu_samples, args.cpu_samples_1t), args.chunk)
            mu_host = mu[:rows].cpu().numpy().astype(np.complex128)
        cpu = cpu_baseline(t128, seed, min(args.cpu_samples, args.chunk), min(args.cpu_sites, M),
                           min(args.cpu_samples_1t, args.chunk), mu=mu_host)

    metric = METRIC if args.workload == "resident" else f"site-samples/s, {args.workload} chain"
    rec = {
        "metric": metric, "value": round(value, 1), "unit": "site-samples/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt / args.steps * 1e3, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": FORMS[args.precision]["dtype"],
        "data": "synthetic",
        "config": {"workload": wname + (f", per-sample displacement (complex Gaussian, scale {args.displace})"
                                        if args.displace > 0 else ""),
                   "sites": M, "d": (4 if args.workload != "uneven" else "2..6"),
                   "chi": int(max(chi)), "samples_per_step": args.chunk,
                   "precision": args.precision, "tensor_bytes": distinct_bytes(dev),
                   "displace_sigma": args.displace or None},
        "roofline": roof, "cpu_baseline": cpu,
    }
    if tuned:
        rec["config"]["autotune"] = tuned
    if tiles:
        rec["config"]["tiles"] = tiles
    if beside:
        rec["beside"] = beside
        if "fp32" in beside:
            rec["speedup_vs_fp32"] = round(value / beside["fp32"]["value"], 3)
    print(json.dumps(rec), flush=True)


def run_stream_bench(args):
    """64-site window at chi = 10^4 streamed from pinned host memory."""
    import torch
    from paper_2512_20064_amd import mps, synth

    M, chi_max, kind = args.sites, args.chi, args.storage
    dl = [4] * M
    t0 = time.time()
    sites, chi = synth.structured_chain(5, dl, chi_max, pool=args.pool, device="cuda")
    host = {}
    stored = []
    for A in sites:
        if id(A) not in host:
            b = synth.compress_site_torch(A, kind)
            h = torch.empty(b.numel(), dtype=torch.uint8, pin_memory=True)
            h.copy_(b)
            host[id(A)] = h
            del b
        stored.append(host[id(A)])
    shapes = [(chi[k], 4, chi[k + 1]) for k in range(M)]
    del sites
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    pinned = sum(h.numel() for h in host.values())
    log(f"window of {M} sites built and compressed ({kind}) in {time.time() - t0:.1f}s; "
        f"{pinned / 2**30:.1f} GiB pinned")
    N, seed = args.samples, 2024

    # plain host-to-device copy rate of the same pinned buffers
    big = max(host.values(), key=lambda h: h.numel())
    dst = torch.empty(big.numel(), dtype=torch.uint8, device="cuda")
    dst.copy_(big, non_blocking=True)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(3):
        dst.copy_(big, non_blocking=True)
    e1.record()
    torch.cuda.synchronize()
    copy_gbps = 3 * big.numel() / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del dst
    log(f"pinned H2D copy alone: {copy_gbps:.1f} GB/s")

    sampler = mps.Sampler(0, n_chunk=args.chunk, profile=True, precision=args.precision)
    # warm-up over the window's first plateau site (same scratch and staging sizes)
    first_plateau = next(k for k in range(M) if chi[k] == chi_max and chi[k + 1] == chi_max)
    sampler.sample_stored(stored[:first_plateau + 1], shapes[:first_plateau + 1], kind, N, seed)
    torch.cuda.synchronize()
    log("warm-up done")
    t0 = time.perf_counter()
    sampler.sample_stored(stored, shapes, kind, N, seed)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = sampler.stats
    sampler.close()
    main_ms = st.contract_ms + st.measure_ms + st.pack_ms + st.expand_ms
    copy_ms = st.h2d_ms
    overlap = None
    if copy_ms > 0:
        overlap = max(0.0, min(1.0, (main_ms + copy_ms - dt * 1e3) / copy_ms))
    rec = {
        "metric": "site-samples/s, streamed chi=10^4 window", "value": round(N * M / dt, 1),
        "unit": "site-samples/s", "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": round(dt * 1e3, 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": FORMS[args.precision]["dtype"], "data": "synthetic",
        "config": {"workload": f"streamed window M={M} d=4 chi={chi_max} structured right-canonical, "
                               f"{kind} in pinned host memory (pool of {args.pool} plateau tensors, every "
                               f"site copied separately), N={N} in chunks of {args.chunk}",
                   "sites": M, "chi": chi_max, "storage": kind, "samples": N, "precision": args.precision},
        "stream": {
            "per_site_ms": round(dt * 1e3 / M, 2),
            "h2d_bytes": st.h2d_bytes,
            "h2d_gbps_in_sweep": round(st.h2d_bytes / (copy_ms * 1e-3) / 1e9, 2) if copy_ms > 0 else None,
            "h2d_gbps_copy_alone": round(copy_gbps, 2),
            "copy_ms": round(copy_ms, 1), "compute_stream_ms": round(main_ms, 1),
            "expand_ms": round(st.expand_ms, 1), "overlap": None if overlap is None else round(overlap, 4),
            "copy_share_of_wall": round(copy_ms / (dt * 1e3), 4),
        },
        # complex-fp16 sites, and complex-fp8 sites with power-of-two block
        # scales (the encoder's choice), expand to values exact in fp16: the
        # fp16 split form skips the product with the (zero) low parts
        "roofline": (roofline_of(args.precision, st.contract_flops, st.contract_launches, st.contract_ms,
                                 dt, st.measure_ms, st.pack_ms, args.chunk, args.chi,
                                 products=2 if (args.precision == "fp16x3" and kind in ("cf16", "cf8")) else None,
                                 m_bytes=st.measure_bytes, m_n=st.measure_launches)
                     if st.contract_ms > 0 else None),
        "cpu_baseline": None,
    }
    print(json.dumps(rec), flush=True)


def run_batch_bench(args):
    """256 independent chains in one batched call against one call per chain."""
    import torch
    from paper_2512_20064_amd import mps, synth

    t0 = time.time()
    chis = tuple(int(x) for x in args.ensemble_chis.split(",")) if args.ensemble_chis else (16, 32, 64, 128, 256)
    specs = synth.ensemble_specs(seed=2, B=args.chains, chis=chis)
    chains = []
    for b, (Mb, db, cb) in enumerate(specs):
        dl = [db] * Mb
        t128 = synth.random_mps(7, dl, synth.ramp_bonds(dl, cb), mps_id=b, pool=4)
        chains.append(upload(synth.to_c64(t128), share=True))
    N, seed = args.samples, 77
    tot_sites = sum(len(c) for c in chains)
    flops = sum(8.0 * N * t.shape[0] * t.shape[1] * t.shape[2] for c in chains for t in c)
    log(f"{len(chains)} chains, {tot_sites} sites, built in {time.time() - t0:.1f}s")

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / reps

    # chain descriptors (site pointers, bonds) are built once, like the upload
    prep = mps.prepare_batch(chains)
    res = {}
    tiles = {}
    for form in [args.precision] + [f for f in args.beside.split(",") if f and f != args.precision]:
        sb = mps.Sampler(0, n_chunk=args.chunk, precision=form, fused_small=bool(args.fused_small))
        choice = []
        if args.tile_tune:
            t0 = time.perf_counter()
            choice = sb.autotune_tiles(prep, min(args.chunk, N))
            tiles[form] = tile_summary(choice, chains, time.perf_counter() - t0)
            log(f"{form} tiles: {tiles[form]['narrow']} of {tiles[form]['shapes']} shapes narrow")
        t_batch = timed(lambda: sb.sample_batch(prep, N, seed), args.steps)
        log(f"{form} batched: {t_batch * 1e3:.1f} ms")
        singles = [mps.Sampler(0, n_chunk=args.chunk, precision=form, mps_id=b, fused_small=bool(args.fused_small))
                   for b in range(len(chains))]
        for s_ in singles:  # the same tile per shape as the batched call
            s_.set_tiles(choice)

        def loop():
            for b, c in enumerate(chains):
                singles[b].sample(c, N, seed)

        t_loop = timed(loop, args.steps)
        log(f"{form} one call per chain: {t_loop * 1e3:.1f} ms")
        for s_ in singles:
            s_.close()
        sb.close()
        res[form] = {"batched": N * tot_sites / t_batch, "per_chain_calls": N * tot_sites / t_loop,
                     "batched_ms": t_batch * 1e3, "per_chain_ms": t_loop * 1e3,
                     "alg_tflops_batched": flops / t_batch / 1e12}
    main = res[args.precision]
    rec = {
        "metric": "site-samples/s, batched ensemble", "value": round(main["batched"], 1), "unit": "site-samples/s",
        "n_gpus": 1, "steps": args.steps, "warmup": 1, "ms_per_step": round(main["batched_ms"], 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": FORMS[args.precision]["dtype"],
        "data": "synthetic",
        "config": {"workload": f"{len(chains)} random right-canonical chains, M~U[32,512], chi in "
                               f"{set(chis)}, d in {{2,3,4}}, complex64, N={N} each",
                   "chains": len(chains), "total_sites": tot_sites, "samples": N, "precision": args.precision,
                   "fused_small": args.fused_small},
        "batch": {f: {k: round(v, 3) for k, v in r.items()} for f, r in res.items()},
        "speedup_batched_vs_per_chain": round(main["batched"] / main["per_chain_calls"], 3),
        "roofline": None, "cpu_baseline": None,
    }
    if tiles:
        rec["config"]["tiles"] = tiles
    print(json.dumps(rec), flush=True)


WORKLOAD_DEFAULTS = {
    "resident": {"sites": 1024, "chi": 1024, "pool": 16, "chunk": 65536, "precision": "fp16f6",
                 "beside": "fp16f8,bf16x3,fp32"},
    "small": {"sites": 32, "chi": 32, "pool": 1, "chunk": 4096, "precision": "fp32", "beside": ""},
    "uneven": {"sites": 2048, "chi": 4096, "pool": 2, "chunk": 8192, "precision": "bf16x3", "beside": ""},
    # N = 2^20 as configured; 24 sites (7 ramp, 17 plateau) keep one call,
    # which prints nothing until it returns, near 90 s; per-site figures are
    # those of a 64-site window
    "stream": {"sites": 24, "chi": 10000, "pool": 4, "chunk": 65536, "samples": 1 << 20, "precision": "fp16x3",
               "beside": ""},
    "batch": {"chunk": 8192, "samples": 8192, "precision": "fp32", "beside": "bf16x3"},
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="resident", choices=sorted(WORKLOAD_DEFAULTS))
    ap.add_argument("--sites", type=int, default=None)
    ap.add_argument("--chi", type=int, default=None)
    ap.add_argument("--pool", type=int, default=None)
    ap.add_argument("--chunk", type=int, default=None)
    ap.add_argument("--samples", type=int, default=None, help="samples per call (stream, batch)")
    ap.add_argument("--chains", type=int, default=256, help="chains in the batch workload")
    ap.add_argument("--ensemble-chis", default="", help="bond caps drawn for the batch workload (comma list)")
    ap.add_argument("--fused-small", type=int, default=1, help="persistent kernel for chains with bonds <= 32 (FP32)")
    ap.add_argument("--storage", default="cf16", choices=["c64", "cf16", "cf8"], help="stream workload storage")
    ap.add_argument("--precision", default=None, choices=sorted(FORMS))
    ap.add_argument("--graph", type=int, default=0, help="replay one captured chunk graph per chunk")
    ap.add_argument("--autotune", type=int, default=1, help="pick the tile order with mps_autotune first")
    ap.add_argument("--tile-tune", type=int, default=1, help="pick the tile shape per site shape first")
    ap.add_argument("--beside", default=None, help="comma-separated forms also timed ('' for none)")
    ap.add_argument("--beside-steps", type=int, default=1)
    ap.add_argument("--displace", type=float, default=0.0, metavar="SIGMA",
                    help="chain workloads: per-sample complex Gaussian displacements of scale SIGMA (GBS)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-samples", type=int, default=4096, help="oracle samples, all BLAS threads")
    ap.add_argument("--cpu-samples-1t", type=int, default=256, help="oracle samples, one BLAS thread")
    ap.add_argument("--cpu-sites", type=int, default=128, help="first sites of the chain the oracle takes")
    ap.add_argument("--no-profile", action="store_true", help="do not event-time each launch")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="also run one plain device copy of this many MiB (reference for HBM counters)")
    args = ap.parse_args()
    for k, v in WORKLOAD_DEFAULTS[args.workload].items():
        if getattr(args, k) is None:
            setattr(args, k, v)
    check_one_gpu(args)

    import torch
    from paper_2512_20064_amd import mps

    if not torch.cuda.is_available():
        raise SystemExit("bench needs a GPU")
    mps.load()
    if args.workload == "stream":
        run_stream_bench(args)
    elif args.workload == "batch":
        run_batch_bench(args)
    else:
        run_chain_bench(args)


if __name__ == "__main__":
    main()
