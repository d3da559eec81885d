#!/usr/bin/env python3
"""Throughput of SFFT image subtraction on one MI355X.

One step = the whole subtraction (build the normal system from FFT
correlations, FP64 Cholesky solve with refinement, convolve-and-subtract) of
a batch of B distinct synthetic 4088x4088 Roman-detector-like pairs in one
batched run (the factorisation launches serve all pairs at once).  Inputs are resident in device memory before the
timed region; the value is pairs per second over the K timed steps.

Also reported, on the same JSON line:
  * roofline   -- the dominant stage's algorithmic bytes (or flops) per
                  launch over its average device time, taken live from HIP
                  events recorded on the stream that launches it;
  * cpu_baseline -- the CPU FP64 oracle (scipy FFTs + LAPACK Cholesky) timed
                  on this host on one pair of the same workload;
  * accuracy   -- relative errors of pair 0's coefficients and difference
                  image against that oracle.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "4088^2 image pairs/sec subtracted at <=1e-5 rel err vs FP64 oracle"
HBM_PEAK_GBS = 8000.0
FP64_VECTOR_PEAK_TFLOPS = 78.6

WORKLOADS = {
    "c3": dict(n=4088, w=9, dk=2, db=2, seed0=3000,
               label="4088x4088 Roman-detector pair, 19x19 delta kernel (w=9), DK=2, DB=2, "
                     "~40000 stars, bright-star + transient masks"),
    "c2": dict(n=1024, w=9, dk=2, db=2, seed0=1002,
               label="1024x1024 pair, 19x19 delta kernel, DK=2, DB=2, 3000 stars, 5% saturation mask"),
    "c1": dict(n=256, w=5, dk=1, db=1, seed0=1001,
               label="256x256 pair, 11x11 delta kernel, DK=1, DB=1, ~400 stars"),
}


def _gen(args):
    name, seed = args
    import synth
    if name == "c3":
        p = synth.pair_c3(seed=seed)
    elif name == "c2":
        p = synth.pair_c2(seed=seed)
    else:
        p = synth.pair_c1(seed=seed)
    return p


def kernel_source_hash():
    h = hashlib.sha256()
    cdir = os.path.join(ROOT, "paper_2509_18544_amd", "csrc")
    for f in sorted(os.listdir(cdir)):
        with open(os.path.join(cdir, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


STAGE_KERNEL = {"corr": "corr_kernel", "col_fwd": "col_fwd_kernel", "row_fwd": "row_fwd_kernel",
                "subtract": "sub_conv_kernel", "moments": "moments_kernel", "row_win": "row_win_kernel"}


def measured_traffic(stage, mode, src):
    """HBM bytes per launch of the stage's kernel from the committed rocprofv3 counter
    summaries (profiles/*.md lines 'traffic: kernel=K mode=M src=H bytes_per_launch=N'),
    or None when none was taken for the current kernel sources."""
    import glob
    import re
    kern = STAGE_KERNEL.get(stage)
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        for line in open(path):
            m = re.match(r"traffic: kernel=(\S+) mode=(\S+) src=(\S+) bytes_per_launch=(\d+)", line.strip())
            if m and m.group(1) == kern and m.group(2) == mode and m.group(3) == src:
                return int(m.group(4))
    return None


def stage_cost(stage, D, mode_f64):
    """Algorithmic amount of one launch of a stage for one pair: ("hbm", bytes) or ("alu", FP64 flops).

    Bytes count each algorithmic read or write once.  The correlation stage
    is priced in flops: per lag-window pair and residue k1, the P2 = 16
    spectral products (6 flops each), one 16-point inverse DFT (168 flops) and
    8 flops per lag row kept; the pair count and lag rows follow the fit.
    """
    n, P, H, planes, vrows = D["N"], D["P"], D["P"] // 2, D["nplanes"], D["vrows"]
    s = 8 if mode_f64 else 4
    cs = 2 * s
    nk, nb, w, L = D["nk"], D["nb"], D["w"], 2 * D["w"] + 1
    nbase = D["nbase"]
    if stage == "row_fwd":
        return "hbm", n * n * (2 * s + 1) + nbase * n * H * cs
    if stage == "col_fwd":
        return "hbm", nbase * H * n * cs + planes * (H + 1) * P * cs
    if stage == "moments":
        return "hbm", n * n * (2 * s + 1)
    if stage == "corr":
        residues = P // 16
        kk = nk * (nk + 1) // 2
        per_res = kk * (96 + 168 + 8 * (4 * w + 1)) + (nk * nb + nk) * (96 + 168 + 8 * (2 * w + 1))
        return "alu", float(per_res) * residues * (H + 1)
    if stage == "subtract":
        return "hbm", 3 * n * n * s
    if stage == "factor":
        m = D["ncoef"]
        return "alu", m ** 3 / 3.0
    return None, None


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--batch", type=int, default=32, help="distinct pairs per step (one batched run)")
    ap.add_argument("--mode", choices=["f32c", "f64"], default="f32c")
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="c3")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default correlation chunk")
    ap.add_argument("--graph", action="store_true",
                    help="also time K graph replays of the batch run (reported as graph_pairs_per_s)")
    ap.add_argument("--quiet", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build runs each pair on a single MI355X "
              "(pairs are independent; see the sharding notes in the design document). "
              "Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    wl = WORKLOADS[args.workload]
    log = (lambda *a: None) if args.quiet else (lambda *a: print(*a, file=sys.stderr, flush=True))

    # ---- synthetic inputs (CPU, before any GPU use) ----
    t0 = time.perf_counter()
    seeds = [wl["seed0"] + i for i in range(args.batch)]
    workers = max(1, min(args.batch, 16, len(os.sched_getaffinity(0))))
    with cf.ProcessPoolExecutor(max_workers=workers) as ex:
        pairs = list(ex.map(_gen, [(args.workload, s) for s in seeds]))
    log(f"[bench] generated {len(pairs)} {args.workload} pairs in {time.perf_counter() - t0:.1f}s")

    import numpy as np
    import torch
    from paper_2509_18544_amd import binding as B

    mode = B.SFFT_MODE_F64 if args.mode == "f64" else B.SFFT_MODE_F32C
    dt = torch.float64 if mode == B.SFFT_MODE_F64 else torch.float32
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.Stream(device=dev)
    descs = [B.make_desc(p.sci.shape[0], p.sci.shape[1], p.w, p.dk, p.db, mode) for p in pairs]
    handle = B.sfft_batch_plan(descs, stream)
    S = [torch.from_numpy(p.sci).to(dev, dt) for p in pairs]
    R = [torch.from_numpy(p.tmpl).to(dev, dt) for p in pairs]
    M = [torch.from_numpy(p.mask).to(dev) for p in pairs]
    Dd = [torch.empty_like(x) for x in S]
    C = [torch.zeros(B.sfft_num_coeffs(d), dtype=torch.float64, device=dev) for d in descs]
    info = torch.zeros(len(pairs), dtype=torch.int32, device=dev)
    lds = [x.stride(0) for x in S]
    torch.cuda.synchronize()

    tuned = None
    if not args.no_autotune:
        # plan-time tuning on pair 0 (outside the timed region)
        tuned = B.sfft_autotune(handle, S[0], R[0], M[0], lds[0])
        log("[bench] autotune (chunk, ms): " + ", ".join(f"({c}, {t:.3f})" for c, t in tuned))

    def step():
        B.sfft_batch_run(handle, S, R, M, lds, C, Dd, info)

    graph_value = None
    if args.graph:
        # the same batch run captured once and replayed as one graph launch per step
        B.sfft_batch_capture(handle, S, R, M, lds, C, Dd, info)
        for _ in range(args.warmup):
            B.sfft_batch_launch(handle)
        torch.cuda.synchronize()
        tg = time.perf_counter()
        for _ in range(args.steps):
            B.sfft_batch_launch(handle)
        torch.cuda.synchronize()
        graph_value = args.batch * args.steps / (time.perf_counter() - tg)
        log(f"[bench] graph replay: {graph_value:.2f} pairs/s")

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    B.sfft_timing_read(handle)          # drop warm-up counters
    B.sfft_timing_enable(handle, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    stage_tot = B.sfft_timing_read(handle)
    B.sfft_timing_enable(handle, False)
    st, inf, nf = B.sfft_status(handle)
    if st != B.SFFT_OK:
        raise RuntimeError(f"device status {B.strerror(st)} (info={inf}, nonfinite={nf})")
    ms_per_step = 1000.0 * elapsed / args.steps
    value = args.batch * args.steps / elapsed
    # per pair: the batched factor/solve stages run once per step for all pairs
    per_pair = {}
    for k, (ms, c) in stage_tot.items():
        per_pair[k] = ms / (args.steps * args.batch) if c else 0.0
    stages_avg = {k: (ms / c if c else 0.0) for k, (ms, c) in stage_tot.items()}
    log("[bench] stage device ms per pair: " + ", ".join(f"{k}={v:.3f}" for k, v in per_pair.items()))

    # ---- roofline of the dominant stage ----
    n_px = pairs[0].sci.shape[0]
    P = 1 << max(6, (n_px - 1).bit_length())
    nk = (pairs[0].dk + 1) * (pairs[0].dk + 2) // 2
    nb = (pairs[0].db + 1) * (pairs[0].db + 2) // 2
    w = pairs[0].w
    vrows = (nk * (nk + 1) // 2) * (4 * w + 1) + (nk * nb + nk) * (2 * w + 1)
    ncoef = B.sfft_num_coeffs(descs[0])
    Dinfo = dict(N=n_px, P=P, nplanes=nk + nb + 1, vrows=vrows, nk=nk, nb=nb, w=w, ncoef=ncoef,
                 nbase=pairs[0].dk + pairs[0].db + 3)
    # dominant kernel: among the stages that are one kernel per pair (the factor/solve
    # stages are batched launches of many kernels, the subtraction is six kernels)
    dom = max((k for k in stages_avg if k in STAGE_KERNEL and k != "subtract"), key=lambda k: per_pair[k])
    def roof_of(stage):
        bound, amount = stage_cost(stage, Dinfo, mode == B.SFFT_MODE_F64)
        # batched stages run once per step for all pairs: price them per pair
        ms = per_pair.get(stage, 0.0) if stage in ("factor", "solve") else stages_avg.get(stage, 0.0)
        if bound is None or ms <= 0:
            return None
        sec = ms / 1000.0
        if bound == "hbm":
            ach = amount / sec / 1e9
            return dict(bound="hbm", achieved=round(ach, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                        frac=round(ach / HBM_PEAK_GBS, 4), per_launch=amount, avg_ms=round(ms, 4))
        ach = amount / sec / 1e12
        return dict(bound="alu", achieved=round(ach, 2), peak=FP64_VECTOR_PEAK_TFLOPS, unit="TFLOP/s",
                    frac=round(ach / FP64_VECTOR_PEAK_TFLOPS, 4), per_launch=amount, avg_ms=round(ms, 4))

    roof = roof_of(dom)
    if roof is not None:
        src = kernel_source_hash()
        roof.update(kernel=dom, traffic=measured_traffic(dom, args.mode, src), src=src)
    stage_roofs = {k: roof_of(k) for k in stages_avg if roof_of(k) is not None}

    # ---- accuracy of pair 0 and the CPU baseline (the oracle itself) ----
    theta_gpu = C[0].cpu().numpy()
    diff_gpu = Dd[0].cpu().numpy().astype(np.float64)
    cpu = None
    acc = None
    if not args.no_cpu_baseline:
        import oracle
        cores = len(os.sched_getaffinity(0))
        p = pairs[0]
        # the oracle sees exactly the values the GPU saw (float32 inputs upcast in FP32C mode)
        s_in = S[0].cpu().numpy().astype(np.float64)
        r_in = R[0].cpu().numpy().astype(np.float64)
        t1 = time.perf_counter()
        ref = oracle.fit(s_in, r_in, p.mask, p.w, p.dk, p.db, mode="fft")
        cpu_s = time.perf_counter() - t1
        cpu = dict(value=round(1.0 / cpu_s, 5), unit="pairs/s", cores=cores, kind="oracle",
                   sample=f"1 pair of the workload (seed {seeds[0]}): FP64 scipy.fft correlations + "
                          f"LAPACK Cholesky + FFT difference image, {cpu_s:.1f} s")
        acc = dict(e_theta=oracle.rel_err(theta_gpu, ref["theta"]),
                   e_diff=oracle.rel_err(diff_gpu, ref["diff"]))
        acc["within_1e-5"] = bool(acc["e_theta"] <= 1e-5 and acc["e_diff"] <= 1e-5)
        log(f"[bench] oracle {cpu_s:.1f}s on {cores} cores; e_theta={acc['e_theta']:.2e} "
            f"e_diff={acc['e_diff']:.2e}")

    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if mode == B.SFFT_MODE_F64 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": wl["label"] + f"; {args.mode.upper()} mode; batch of {args.batch} "
                                             f"distinct pairs per step (one batched run)",
                   "global_batch": args.batch, "frame": n_px, "fft_size": P, "coefficients": ncoef,
                   "corr_chunk_autotune": tuned},
        "roofline": roof,
        "cpu_baseline": cpu,
        "accuracy": acc,
        "stages_ms_per_pair": {k: round(v, 4) for k, v in per_pair.items()},
        "graph_pairs_per_s": None if graph_value is None else round(graph_value, 3),
        "stage_rooflines": {k: {"bound": v["bound"], "frac": v["frac"], "achieved": v["achieved"],
                                "unit": v["unit"]} for k, v in stage_roofs.items()},
    }
    print(json.dumps(out), flush=True)
    B.sfft_destroy(handle)


if __name__ == "__main__":
    main()
