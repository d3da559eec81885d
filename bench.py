#!/usr/bin/env python3
"""Throughput of SFFT image subtraction on one MI355X.

One step = the whole subtraction (build the normal system from FFT
correlations, FP64 Cholesky solve with refinement, convolve-and-subtract) of
a batch of B distinct synthetic pairs in one batched run (the factorisation
launches serve all pairs at once).  Inputs are resident in device memory
before the timed region; `value` is pairs per second over the K timed steps
of the headline form (FP32C: FP32 transforms, FP64 products, lag sums,
Cholesky and refinement), with per-stage event timing off except around the
dominant kernel.

The same JSON line also carries:
  * step_ms        -- median, p10 and p90 of the per-step device times;
  * graph          -- the same batch captured once and replayed as one graph
                      launch per step;
  * fp64           -- the plain FP64 GPU form on the same pairs;
  * roofline       -- the dominant kernel's algorithmic flops per launch over
                      its average device time (HIP events on the stream that
                      launches it, over the timed region), plus the whole
                      path against the HBM roofline and against the
                      bandwidth a plain device copy attains on this GPU;
  * cpu_baseline   -- the CPU FP64 oracle timed on this host (median of 3) on
                      one pair of the workload, and on the 256^2 and 1024^2
                      pairs, with the core count and CPU model;
  * assembly_routes -- pair 0 assembled by each route (FFT transforms, direct
                      lag sums where allowed, FP64 matrix-core products):
                      sfft_autotune_route's build times and the route it keeps,
                      and the matrix-core kernel's executed FP64 TFLOP/s
                      against the 78.6 TFLOP/s peak;
  * accuracy       -- e_theta and e_D of EVERY timed pair against the oracle
                      (theta* stored by tests/golden/make_golden.py or solved
                      live, D* computed by the oracle from theta*), with the
                      maximum over pairs; `value` is null unless every pair
                      meets the bar (1e-5 FP32C, 1e-9 FP64).
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
BAR = {"f32c": 1e-5, "f64": 1e-9}
GOLDEN = os.path.join(ROOT, "tests", "golden")

WORKLOADS = {
    "c3": dict(seed0=3000, label="4088x4088 Roman-detector pairs, 19x19 delta kernel (w=9), DK=2, DB=2, "
                                 "~40000 stars, bright-star + transient masks"),
    "c2": dict(seed0=1002, label="1024x1024 pairs, 19x19 delta kernel, DK=2, DB=2, 3000 stars, 5% saturation mask"),
    "c1": dict(seed0=1001, label="256x256 pairs, 11x11 delta kernel, DK=1, DB=1, ~400 stars"),
    "c4": dict(seed0=4000, label="S x T = 8 x 16 uneven cutouts, N in {512,1024,2048}, w in 5..9, DK in {1,2}, DB=DK"),
    "st": dict(seed0=6000, label="S x T template groups: 16 science epochs per 4088x4088 template and mask "
                                 "(19x19 delta kernel, w=9, DK=2, DB=2), the template spectra, normal matrix, "
                                 "factor and template row spectra shared within a group"),
}
ST_EPOCHS = 16   # science epochs per template in the template-group workload


# ---------------------------------------------------------------------------
# synthetic inputs (CPU worker processes, created before the GPU is touched)
# ---------------------------------------------------------------------------

def _generate(workload, i):
    import synth
    seed0 = WORKLOADS[workload]["seed0"]
    if workload == "c3":
        return synth.pair_c3(seed=seed0 + i)
    if workload == "c2":
        return synth.pair_c2(seed=seed0 + i)
    if workload == "c1":
        return synth.pair_c1(seed=seed0 + i)
    if workload == "st":
        return synth.template_group_pair(seed0 + i // ST_EPOCHS, 4088, i % ST_EPOCHS, ST_EPOCHS)
    return synth.pair_c4(synth.batch_c4_descriptors()[i])



def _pin_worker(cores, counter):
    """Pool initializer: one host core per worker process (the oracle then uses one thread)."""
    with counter.get_lock():
        k = counter.value
        counter.value += 1
    os.sched_setaffinity(0, {cores[k % len(cores)]})


# ---------------------------------------------------------------------------
# CPU-baseline leg: everything that runs the oracle (timing and references)
# ---------------------------------------------------------------------------

def _oracle_reference(workload, i, pair, tags):
    """theta* and D* of one pair for each input precision in `tags` (f32in / f64),
    from the oracle: theta* stored by the golden script (4088^2 benchmark pairs)
    or solved live, D* = the oracle's difference image from theta*."""
    import numpy as np
    import oracle
    out = {}
    for tag in tags:
        cast = np.float32 if tag == "f32in" else np.float64
        s_in = pair.sci.astype(cast).astype(np.float64)
        r_in = pair.tmpl.astype(cast).astype(np.float64)
        theta = None
        gpath = os.path.join(GOLDEN, f"bench_c3_theta_{tag}.npy")
        if workload == "c3" and WORKLOADS["c3"]["seed0"] == 3000 and os.path.exists(gpath):
            g = np.load(gpath)
            if i < g.shape[0]:
                theta = g[i]
        if theta is None:
            theta = oracle.fit(s_in, r_in, pair.mask, pair.w, pair.dk, pair.db, mode="fft")["theta"]
        dstar = oracle.difference(s_in, r_in, theta, pair.w, pair.dk, pair.db, mode="fft")
        out[tag] = (theta, dstar)
    return out


def _prepare(job):
    workload, i, tags = job
    p = _generate(workload, i)
    ref = _oracle_reference(workload, i, p, tags) if tags else None
    return p, ref


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline_leg(pairs, workload, log):
    """The oracle as it stands, timed on this host's cores: median of 3 runs
    on pair 0 of the workload, on the 256^2 pair (FFT and direct routes) and
    on the 1024^2 pair; plus cond(Omega) of pair 0."""
    import numpy as np
    import scipy
    import oracle
    import synth

    cores = len(os.sched_getaffinity(0))

    def med3(fn):
        ts = []
        for _ in range(3):
            t = time.perf_counter()
            r = fn()
            ts.append(time.perf_counter() - t)
        return float(np.median(ts)), ts, r

    p = pairs[0]
    s_in = p.sci.astype(np.float32).astype(np.float64)
    r_in = p.tmpl.astype(np.float32).astype(np.float64)
    t_med, ts, ref = med3(lambda: oracle.fit(s_in, r_in, p.mask, p.w, p.dk, p.db, mode="fft"))
    log(f"[bench] oracle on pair 0: median {t_med:.2f}s of {[round(x, 2) for x in ts]} on {cores} cores")
    t = time.perf_counter()
    cond = oracle.cond_number(ref["omega"])
    log(f"[bench] cond(Omega) of pair 0 = {cond:.3e} ({time.perf_counter() - t:.1f}s)")
    by = {}
    for name, gen, mode in (("256x256 (fft route)", synth.pair_c1, "fft"), ("256x256 (direct route)", synth.pair_c1, "direct"),
                            ("1024x1024 (fft route)", synth.pair_c2, "fft")):
        q = gen()
        tm, tq, _ = med3(lambda: oracle.fit(q.sci, q.tmpl, q.mask, q.w, q.dk, q.db, mode=mode))
        by[name] = dict(value=round(1.0 / tm, 4), unit="pairs/s", median_s=round(tm, 4),
                        runs_s=[round(x, 4) for x in tq])
        log(f"[bench] oracle {name}: median {tm:.3f}s")
    n = p.sci.shape[0]
    cpu = dict(value=round(1.0 / t_med, 5), unit="pairs/s", cores=cores, kind="oracle",
               sample=f"1 pair of the workload ({n}x{n}, seed {WORKLOADS[workload]['seed0']}, float32-rounded inputs): "
                      f"FP64 scipy.fft correlations + LAPACK Cholesky + FFT difference image; median of 3 runs",
               median_of=3, runs_s=[round(x, 3) for x in ts], cpu_model=cpu_model(),
               versions=dict(numpy=np.__version__, scipy=scipy.__version__), by_config=by)
    return cpu, ref, cond


def accuracy_of(outputs, refs, tag, bar):
    """Relative errors of every pair's theta and D against the oracle's."""
    import numpy as np
    et, ed, eb = [], [], []
    for (theta, diff), ref in zip(outputs, refs):
        th_ref, d_ref = ref[tag]
        et.append(float(np.linalg.norm(theta - th_ref) / np.linalg.norm(th_ref)))
        dd = diff.astype(np.float64)
        ed.append(float(np.linalg.norm(dd - d_ref) / np.linalg.norm(d_ref)))
        eb.append(float(np.abs(dd - d_ref).max() / np.abs(d_ref).max()))
    return dict(pairs=len(et), e_theta_max=max(et), e_diff_max=max(ed), e_diff_inf_max=max(eb),
                e_theta_median=float(np.median(et)), e_diff_median=float(np.median(ed)),
                bar=bar, all_within=bool(max(et) <= bar and max(ed) <= bar))


# ---------------------------------------------------------------------------
# the GPU legs
# ---------------------------------------------------------------------------

# what the correlation kernel is compiled from: its header, the shared
# device helpers and the build flags (the committed traffic figures are valid
# while these are unchanged)
CORR_SOURCES = ("paper_2509_18544_amd/csrc/assemble.hpp", "paper_2509_18544_amd/csrc/common.hpp",
                "paper_2509_18544_amd/build.py")


def kernel_source_hash():
    h = hashlib.sha256()
    for f in CORR_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


STAGE_KERNEL = {"corr": "corr_kernel", "col_fwd": "col_fwd_kernel", "row_fwd": "row_fwd_kernel",
                "moments": "moments_kernel", "row_win": "row_win_kernel"}


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


def shape_info(p):
    n = p.sci.shape[0]
    P = 1 << max(6, (n - 1).bit_length())
    nk = (p.dk + 1) * (p.dk + 2) // 2
    nb = (p.db + 1) * (p.db + 2) // 2
    L = 2 * p.w + 1
    # the transform route: bases xh^p G_R R (p <= DK) and G S; planes A_a and S_m
    return dict(N=n, P=P, nk=nk, nb=nb, w=p.w, ncoef=L * L * nk + nb, nbase=p.dk + 2,
                nplanes=nk + 1)


def stage_cost(stage, D, mode_f64):
    """Algorithmic amount of one launch of a stage for one pair: ("hbm", bytes) or ("alu", FP64 flops).

    Bytes count each algorithmic read or write once.  The correlation stage
    is priced in flops: per lag-window pair and residue k1, the P2 = 16
    spectral products (6 flops each), one 16-point inverse DFT (168 flops) and
    8 flops per lag row kept; the pairs are the template-template windows
    (|d| <= 2w) and the template-science windows (|d| <= w) -- the
    template-background block is formed from moments, not correlations.
    """
    n, P, H, planes = D["N"], D["P"], D["P"] // 2, D["nplanes"]
    s = 8 if mode_f64 else 4
    cs = 2 * s
    nk, nb, w = D["nk"], D["nb"], D["w"]
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
        per_res = kk * (96 + 168 + 8 * (4 * w + 1)) + nk * (96 + 168 + 8 * (2 * w + 1))
        return "alu", float(per_res) * residues * (H + 1)
    if stage == "subtract":
        return "hbm", 3 * n * n * s
    if stage == "factor":
        m = D["ncoef"]
        return "alu", m ** 3 / 3.0
    return None, None


def path_bytes(D, mode_f64):
    """Algorithmic HBM bytes of one whole pair: inputs read once and D written once,
    every spectrum (the nK + 1 forward planes plus the apply's one) written and
    read once, Omega gathered, factored and read."""
    n, P = D["N"], D["P"]
    s = 8 if mode_f64 else 4
    nplanes = D["nk"] + 2
    return 3 * n * n * s + n * n + 2 * nplanes * P * (P // 2 + 1) * 2 * s + 4 * D["ncoef"] ** 2 * 8


def copy_bandwidth(torch, dev, log, gib=2, reps=10):
    """HBM bandwidth a plain device copy attains: (read + write bytes) / time."""
    n = gib * (1 << 30) // 4
    a = torch.ones(n, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    gbs = 2 * n * 4 / (ms * 1e-3) / 1e9
    log(f"[bench] device copy of {gib} GiB: {ms:.3f} ms -> {gbs:.0f} GB/s (read + write)")
    del a, b
    return gbs


def run_leg(B, torch, pairs, mode_name, args, log, tmpl_of=None):
    """Time one precision mode on the batch; returns figures and the host copies of
    the outputs.  With tmpl_of, pair i uses pair tmpl_of[i]'s template and mask
    (a shared-template batch plan, one device copy of each template)."""
    import numpy as np
    mode = B.SFFT_MODE_F64 if mode_name == "f64" else B.SFFT_MODE_F32C
    dt = torch.float64 if mode == B.SFFT_MODE_F64 else torch.float32
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    descs = [B.make_desc(p.sci.shape[0], p.sci.shape[1], p.w, p.dk, p.db, mode) for p in pairs]
    handle = B.sfft_batch_plan(descs, stream) if tmpl_of is None else B.sfft_batch_plan_shared(descs, tmpl_of, stream)
    with torch.cuda.stream(stream):
        S = [torch.from_numpy(p.sci).to(dev, dt) for p in pairs]
        if tmpl_of is None:
            R = [torch.from_numpy(p.tmpl).to(dev, dt) for p in pairs]
            M = [torch.from_numpy(p.mask).to(dev) for p in pairs]
        else:
            R, M = [], []
            for i, p in enumerate(pairs):
                o = tmpl_of[i]
                if o == i:
                    R.append(torch.from_numpy(p.tmpl).to(dev, dt))
                    M.append(torch.from_numpy(p.mask).to(dev))
                else:
                    assert np.array_equal(p.tmpl, pairs[o].tmpl) and np.array_equal(p.mask, pairs[o].mask)
                    R.append(R[o])
                    M.append(M[o])
        Dd = [torch.empty_like(x) for x in S]
        C = [torch.zeros(B.sfft_num_coeffs(d), dtype=torch.float64, device=dev) for d in descs]
        info = torch.zeros(len(pairs), dtype=torch.int32, device=dev)
    lds = [x.stride(0) for x in S]
    stream.synchronize()
    out = dict(mode=mode_name)
    tuned = None
    if not args.no_autotune:
        tuned = B.sfft_autotune(handle, S[0], R[0], M[0], lds[0])     # plan time, outside the timed region
        log(f"[bench] {mode_name} autotune (chunk, ms): " + ", ".join(f"({c}, {t:.3f})" for c, t in tuned))
    out["corr_chunk_autotune"] = tuned

    def step():
        B.sfft_batch_run(handle, S, R, M, lds, C, Dd, info)

    # timed region: events around the correlation kernel only, the event pool made before
    B.sfft_timing_enable(handle, ["corr"])
    for _ in range(args.warmup):
        step()
    B.sfft_timing_read(handle)                          # synchronises; drops the warm-up counts
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ev[k].record(stream)
        step()
    ev[args.steps].record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    corr_tot = B.sfft_timing_read(handle)["corr"]
    B.sfft_timing_enable(handle, False)
    st, inf, nf = B.sfft_status(handle)
    if st != B.SFFT_OK:
        raise RuntimeError(f"device status {B.strerror(st)} (info={inf}, nonfinite={nf})")
    steps_ms = [ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)]
    out["value"] = len(pairs) * args.steps / elapsed
    out["ms_per_step"] = 1000.0 * elapsed / args.steps
    out["step_ms"] = dict(median=float(np.median(steps_ms)), p10=float(np.percentile(steps_ms, 10)),
                          p90=float(np.percentile(steps_ms, 90)), min=float(min(steps_ms)), max=float(max(steps_ms)))
    out["corr_ms_per_launch"] = corr_tot[0] / corr_tot[1] if corr_tot[1] else None
    out["corr_launches"] = corr_tot[1]
    # a launch serves every pair of a group (same descriptor): pairs per launch
    out["corr_pairs_per_launch"] = len(pairs) * args.steps / corr_tot[1] if corr_tot[1] else None
    log(f"[bench] {mode_name}: {out['value']:.2f} pairs/s, {out['ms_per_step']:.2f} ms/step "
        f"(median {out['step_ms']['median']:.2f}), corr {out['corr_ms_per_launch']:.4f} ms x {corr_tot[1]}")

    # outputs of the last timed step, to the host for the accuracy check
    out["outputs"] = [(c.cpu().numpy(), d.cpu().numpy()) for c, d in zip(C, Dd)]
    out["info"] = info.cpu().tolist()

    # the same batch as one captured graph, replayed once per step
    out["graph"] = None
    if not args.no_graph:
        B.sfft_batch_capture(handle, S, R, M, lds, C, Dd, info)
        for _ in range(max(1, args.warmup)):
            B.sfft_batch_launch(handle)
        torch.cuda.synchronize()
        tg = time.perf_counter()
        for _ in range(args.steps):
            B.sfft_batch_launch(handle)
        torch.cuda.synchronize()
        gval = len(pairs) * args.steps / (time.perf_counter() - tg)
        # the replays recompute the same outputs: they must equal the eager ones bitwise
        same = all(np.array_equal(c.cpu().numpy(), o[0]) and np.array_equal(d.cpu().numpy(), o[1])
                   for c, d, o in zip(C, Dd, out["outputs"]))
        out["graph"] = dict(value=round(gval, 3), unit="pairs/s", outputs_equal_eager=bool(same))
        log(f"[bench] {mode_name} graph replay: {gval:.2f} pairs/s (outputs equal eager: {same})")

    # stage breakdown in a separate pass (every stage timed; not part of value)
    B.sfft_timing_enable(handle, True)
    for _ in range(2):
        step()
    tot = B.sfft_timing_read(handle)
    B.sfft_timing_enable(handle, False)
    out["stages_ms_per_pair"] = {k: (ms / (2 * len(pairs)) if c else 0.0) for k, (ms, c) in tot.items()}
    out["stages_avg_ms"] = {k: (ms / c if c else 0.0) for k, (ms, c) in tot.items()}
    B.sfft_destroy(handle)
    del S, R, M, Dd, C
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return out


MFMA_F64_PEAK_TFLOPS = 78.6
MFMA_XC = 256          # columns per block of the MFMA route's kernel


def mfma_flops(D):
    """(executed, useful) FP64 flops of one MFMA-route assembly: per (pair, 16-lag
    dy tile) block row, every source row of the frame runs 16 x 4 instructions
    of 16x16x4 (2048 flops) per dx tile over each 256-column chunk; the useful
    part is one multiply-add per pixel and window entry."""
    n, w, nk, nb = D["N"], D["w"], D["nk"], D["nb"]
    pairs = [2 * w] * (nk * (nk + 1) // 2) + [w] * (nk * nb + nk)   # lag half-widths: 2w (kernel x kernel), w
    nxc = -(-n // MFMA_XC)
    executed = useful = 0
    for hw in pairs:
        h = 2 * hw + 1
        tiles = -(-h // 16)
        executed += tiles * tiles * nxc * n * 64 * 2048
        useful += 2 * h * h * n * n
    return executed, useful


def route_leg(B, torch, p, mode_name, log):
    """Assembly routes on pair 0: sfft_autotune_route's build times (FFT, direct,
    MFMA) and the MFMA kernel's own device time with its matrix-core rate."""
    mode = B.SFFT_MODE_F64 if mode_name == "f64" else B.SFFT_MODE_F32C
    dt = torch.float64 if mode == B.SFFT_MODE_F64 else torch.float32
    S = torch.from_numpy(p.sci).to("cuda", dt)
    R = torch.from_numpy(p.tmpl).to("cuda", dt)
    M = torch.from_numpy(p.mask).cuda()
    n = p.sci.shape[0]
    out = {}
    plan = B.Plan(n, n, p.w, p.dk, p.db, mode=mode)
    try:
        ms, route = B.sfft_autotune_route(plan.handle, S, R, M, S.stride(0))
        out["build_ms"] = {k: (round(v, 3) if v is not None else None) for k, v in ms.items()}
        out["auto_route"] = route
    finally:
        plan.close()
    plan = B.Plan(n, n, p.w, p.dk, p.db, mode=mode, flags=B.SFFT_FLAG_ASSEMBLY_MFMA)
    try:
        plan.build(S, R, M)
        B.sfft_timing_enable(plan.handle, ["corr"])
        for _ in range(2):
            plan.build(S, R, M)
        t = B.sfft_timing_read(plan.handle)["corr"]
        B.sfft_timing_enable(plan.handle, False)
        kms = t[0] / t[1]
        ex, us = mfma_flops(shape_info(p))
        out["mfma_kernel"] = dict(avg_ms=round(kms, 3), executed_tflop=round(ex / 1e12, 3),
                                  useful_tflop=round(us / 1e12, 3),
                                  achieved_tflops=round(ex / (kms * 1e-3) / 1e12, 2), peak=MFMA_F64_PEAK_TFLOPS,
                                  utilisation=round(ex / (kms * 1e-3) / 1e12 / MFMA_F64_PEAK_TFLOPS, 4))
    finally:
        plan.close()
    log(f"[bench] assembly routes on pair 0 ({mode_name}): {out}")
    del S, R, M
    torch.cuda.empty_cache()
    return out


def next_leg(B, torch, p, mode_name, log, reps=10):
    """The pipeline steps around the subtraction on pair 0, each timed with HIP
    events on the stream it runs on (torch's current stream): alignment of the
    template and its mask (step 4) by a small rotation, scale and shift;
    cross-convolution of the science image with a PSF stamp (step 5); the
    constant-photometric-ratio solve against the free one; the decorrelation
    kernel and its application to the difference image (step 7).  Algorithmic
    bytes: alignment reads the template and mask and writes both (2 N^2 (e + 1),
    e the image element size); a convolution reads and writes one image
    (2 N^2 e)."""
    import math
    import synth
    mode = B.SFFT_MODE_F64 if mode_name == "f64" else B.SFFT_MODE_F32C
    dt = torch.float64 if mode == B.SFFT_MODE_F64 else torch.float32
    es = 8 if mode == B.SFFT_MODE_F64 else 4
    S = torch.from_numpy(p.sci).to("cuda", dt)
    R = torch.from_numpy(p.tmpl).to("cuda", dt)
    M = torch.from_numpy(p.mask).cuda()
    n = p.sci.shape[0]
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ev[0].record()
        for _ in range(reps):
            fn()
        ev[1].record()
        torch.cuda.synchronize()
        return ev[0].elapsed_time(ev[1]) / reps

    def hbm(ms, byt):
        g = byt / (ms * 1e-3) / 1e9
        return dict(bound="hbm", ms=round(ms, 4), bytes=int(byt), achieved_gbs=round(g, 1), peak=HBM_PEAK_GBS,
                    frac=round(g / HBM_PEAK_GBS, 4))

    out = {}
    th = 0.0015
    c, sn = math.cos(th), math.sin(th)
    pmap = B.make_map([n / 2 + 0.37, 1.0002 * c, -1.0002 * sn], [n / 2 - 0.21, 1.0002 * sn, 1.0002 * c],
                      (n / 2, n / 2))
    Ra, Ma = torch.empty_like(R), torch.empty_like(M)
    out["align"] = hbm(timed(lambda: B.sfft_align_image(pmap, mode, R, M, Ra, Ma)), 2 * n * n * (es + 1))
    out["align"]["kernel"] = "align_image_kernel"
    sp = 12
    pr = synth.psf_stamp(1.8, 3.0, half=sp)
    ps = synth.psf_stamp(2.2, 3.0, half=sp)
    prd, psd = torch.from_numpy(pr.ravel()).cuda(), torch.from_numpy(ps.ravel()).cuda()
    cplan = B.Plan(n, n, sp, 0, 0, mode=mode)
    try:
        Sx = torch.empty_like(S)
        out["cross_convolution"] = hbm(timed(lambda: cplan.apply_kernel(S, prd, Sx)), 2 * n * n * es)
        out["cross_convolution"]["stamp"] = 2 * sp + 1
    finally:
        cplan.close()
    solve_ms = {}
    for name, fl in (("free", 0), ("constrained", B.SFFT_FLAG_CONST_RATIO)):
        plan = B.Plan(n, n, p.w, p.dk, p.db, mode=mode, flags=fl)
        try:
            plan.build(S, R, M)
            coeffs = torch.zeros(plan.n, dtype=torch.float64, device="cuda")
            info = torch.zeros(1, dtype=torch.int32, device="cuda")
            solve_ms[name] = timed(lambda: plan.solve(coeffs, info))
            if fl:
                D = plan.subtract(S, R, coeffs)
                t = 12
                psi = torch.empty((2 * t + 1) ** 2, dtype=torch.float64, device="cuda")
                kms = timed(lambda: B.sfft_decorrelation_kernel(plan.handle, coeffs, psd, prd, sp, 32.0, 32.0, t, psi))
                dplan = B.Plan(n, n, t, 0, 0, mode=mode)
                try:
                    Dd = torch.empty_like(D)
                    app = hbm(timed(lambda: dplan.apply_kernel(D, psi, Dd)), 2 * n * n * es)
                finally:
                    dplan.close()
                out["decorrelation"] = dict(kernel_ms=round(kms, 4), grid=64, taps=2 * t + 1, apply=app)
        finally:
            plan.close()
    # output-masked fit: the rank-|M| correction of the kernel block on the
    # FP64 matrix cores, timed by the plan's stage events over `reps` builds
    plan = B.Plan(n, n, p.w, p.dk, p.db, mode=mode, flags=B.SFFT_FLAG_OUTPUT_MASK)
    try:
        plan.build(S, R, M)
        B.sfft_timing_enable(plan.handle, ["outmask"])
        for _ in range(3):
            plan.build(S, R, M)
        oms, cnt = B.sfft_timing_read(plan.handle)["outmask"]
        B.sfft_timing_enable(plan.handle, False)
        om_ms = oms / cnt
        nkk = (2 * p.w + 1) ** 2 * (p.dk + 1) * (p.dk + 2) // 2
        nexcl = int((p.mask != 0).sum())
        nt = -(-nkk // 64)
        executed = nt * (nt + 1) // 2 * 64 * 64 * 2 * (-(-nexcl // 64) * 64)
        useful = nkk * nkk * nexcl          # 2 flops per multiply-add over the symmetric half
        out["output_mask"] = dict(bound="mfma", kernel="om_syrk_kernel (+ planes, count, scan, list)", ms=round(om_ms, 3),
                                  excluded_pixels=nexcl, kernel_block=nkk, executed_tflop=round(executed / 1e12, 4),
                                  useful_tflop=round(useful / 1e12, 4),
                                  achieved_tflops=round(executed / (om_ms * 1e-3) / 1e12, 2),
                                  peak=MFMA_F64_PEAK_TFLOPS,
                                  frac=round(executed / (om_ms * 1e-3) / 1e12 / MFMA_F64_PEAK_TFLOPS, 4))
    finally:
        plan.close()
    out["const_ratio"] = dict(solve_ms_free=round(solve_ms["free"], 4),
                              solve_ms_constrained=round(solve_ms["constrained"], 4),
                              overhead_ms=round(solve_ms["constrained"] - solve_ms["free"], 4),
                              constraints=(p.dk + 1) * (p.dk + 2) // 2 - 1)
    log(f"[bench] pipeline steps 4-7 on pair 0 ({mode_name}): {out}")
    del S, R, M, Ra, Ma
    torch.cuda.empty_cache()
    return out


def roofline_of(stage, D, mode_f64, ms, pairs=1.0):
    """Algorithmic amount of `pairs` pairs over `ms` milliseconds against the peak."""
    bound, amount = stage_cost(stage, D, mode_f64)
    if bound is None or not ms:
        return None
    amount = amount * pairs
    sec = ms / 1000.0
    if bound == "hbm":
        ach = amount / sec / 1e9
        return dict(bound="hbm", achieved=round(ach, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(ach / HBM_PEAK_GBS, 4), per_launch=amount, avg_ms=round(ms, 4))
    ach = amount / sec / 1e12
    return dict(bound="alu", achieved=round(ach, 2), peak=FP64_VECTOR_PEAK_TFLOPS, unit="TFLOP/s",
                frac=round(ach / FP64_VECTOR_PEAK_TFLOPS, 4), per_launch=amount, avg_ms=round(ms, 4))


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--batch", type=int, default=32, help="distinct pairs per step (one batched run)")
    ap.add_argument("--mode", choices=["f32c", "f64"], default="f32c", help="the headline form")
    ap.add_argument("--no-f64", action="store_true", help="skip the plain FP64 comparison form")
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="c3")
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle (its timing and the accuracy check): value is then null")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default correlation chunk")
    ap.add_argument("--no-graph", action="store_true", help="skip the graph-replay timing")
    ap.add_argument("--no-routes", action="store_true", help="skip the assembly-route timings")
    ap.add_argument("--no-next", action="store_true",
                    help="skip the timings of the steps around the subtraction (alignment, cross-convolution, "
                         "constant ratio, decorrelation)")
    ap.add_argument("--quiet", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build runs each pair on a single MI355X "
              "(pairs are independent; see the sharding notes in the design document). "
              "Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    if args.workload == "c4":
        args.batch = min(args.batch, 128) if args.batch != 32 else 128
    if args.workload == "st":
        args.batch = max(ST_EPOCHS, (args.batch // ST_EPOCHS) * ST_EPOCHS)   # whole template groups
    log = (lambda *a: None) if args.quiet else (lambda *a: print(*a, file=sys.stderr, flush=True))
    wl = WORKLOADS[args.workload]
    legs = [args.mode] + ([] if args.no_f64 or args.mode == "f64" else ["f64"])
    tags = [] if args.no_cpu_baseline else [("f32in" if m == "f32c" else "f64") for m in legs]

    # ---- synthetic inputs and the oracle's references, in CPU worker processes
    # created before any GPU use (each worker pinned to one host core) ----
    import multiprocessing as mp
    t0 = time.perf_counter()
    cores = sorted(os.sched_getaffinity(0))
    nwork = max(1, min(args.batch, 16, len(cores)))
    ctx = mp.get_context("fork")
    counter = ctx.Value("i", 0)
    with cf.ProcessPoolExecutor(max_workers=nwork, mp_context=ctx, initializer=_pin_worker,
                                initargs=(cores, counter)) as ex:
        res = []
        for r in ex.map(_prepare, [(args.workload, i, tags) for i in range(args.batch)]):
            res.append(r)
            if len(res) % 4 == 0 or len(res) == args.batch:
                log(f"[bench] {len(res)}/{args.batch} pairs ready ({time.perf_counter() - t0:.0f}s)")
    pairs = [r[0] for r in res]
    refs = [r[1] for r in res]
    log(f"[bench] generated {len(pairs)} {args.workload} pairs"
        + (" with oracle references" if tags else "") + f" in {time.perf_counter() - t0:.1f}s")

    import numpy as np
    import torch
    from paper_2509_18544_amd import binding as B

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    copy_gbs = copy_bandwidth(torch, dev, log)
    tmpl_of = [ST_EPOCHS * (i // ST_EPOCHS) for i in range(len(pairs))] if args.workload == "st" else None
    results = {m: run_leg(B, torch, pairs, m, args, log, tmpl_of) for m in legs}
    unshared = None
    if tmpl_of is not None:
        # the same pairs with every template handled on its own, for comparison
        r = run_leg(B, torch, pairs, args.mode, args, log)
        unshared = dict(value=round(r["value"], 3), unit="pairs/s", ms_per_step=round(r["ms_per_step"], 3),
                        stages_ms_per_pair={k: round(v, 4) for k, v in r["stages_ms_per_pair"].items()})
        log(f"[bench] the same batch unshared: {r['value']:.2f} pairs/s")
    routes = None
    if not args.no_routes and len({(p.sci.shape, p.w, p.dk, p.db) for p in pairs}) == 1:
        routes = route_leg(B, torch, pairs[0], args.mode, log)
    steps = None
    if not args.no_next:
        steps = next_leg(B, torch, pairs[0], args.mode, log)

    # ---- CPU baseline and accuracy (the oracle) ----
    cpu = cond = None
    acc = {}
    if not args.no_cpu_baseline:
        cpu, ref0, cond = cpu_baseline_leg(pairs, args.workload, log)
        for m in legs:
            tag = "f32in" if m == "f32c" else "f64"
            acc[m] = accuracy_of(results[m]["outputs"], refs, tag, BAR[m])
            acc[m]["failed_pairs"] = [i for i, v in enumerate(results[m]["info"]) if v != 0]
            log(f"[bench] {m} accuracy over {acc[m]['pairs']} pairs: max e_theta={acc[m]['e_theta_max']:.2e} "
                f"max e_D={acc[m]['e_diff_max']:.2e} (bar {BAR[m]:g})")
        if "f32c" in legs and args.workload == "c3" and not args.no_cpu_baseline:
            # the stored theta* of pair 0 must be what the oracle computes now
            g = refs[0]["f32in"][0]
            acc["f32c"]["golden_vs_live_theta"] = float(np.linalg.norm(g - ref0["theta"]) / np.linalg.norm(ref0["theta"]))

    head = results[args.mode]
    D = shape_info(pairs[0])
    mode_f64 = args.mode == "f64"
    # per-launch flops and per-pair bytes depend on the pair's shape, and a
    # sharing pair does less than a full one: priced only for a uniform,
    # unshared batch
    same_shape = len({(p.sci.shape, p.w, p.dk, p.db) for p in pairs}) == 1
    uniform = same_shape and tmpl_of is None
    ppl = head["corr_pairs_per_launch"]
    roof = roofline_of("corr", D, mode_f64, head["corr_ms_per_launch"], ppl) if uniform else None
    src = kernel_source_hash()
    if roof is not None:
        roof.update(kernel="corr_kernel", traffic=measured_traffic("corr", args.mode, src), src=src,
                    launches_timed=head["corr_launches"], pairs_per_launch=ppl)
    value = head["value"]
    ok = (not args.no_cpu_baseline) and acc[args.mode]["all_within"] and not acc[args.mode]["failed_pairs"]
    path = None
    if uniform:
        bpp = path_bytes(D, mode_f64)
        path = dict(bytes_per_pair=bpp, roofline_pairs_per_s=round(HBM_PEAK_GBS * 1e9 / bpp, 1),
                    frac=round(value / (HBM_PEAK_GBS * 1e9 / bpp), 4),
                    attainable_gbs=round(copy_gbs, 1),
                    frac_of_attainable=round(value / (copy_gbs * 1e9 / bpp), 4))
    mpx = sum(p.sci.shape[0] * p.sci.shape[1] for p in pairs) / len(pairs) / 1e6
    fp64 = None
    if "f64" in results and args.mode != "f64":
        r = results["f64"]
        fp64 = dict(value=round(r["value"], 3) if (args.no_cpu_baseline or acc["f64"]["all_within"]) else None,
                    measured=round(r["value"], 3), unit="pairs/s", ms_per_step=round(r["ms_per_step"], 3),
                    step_ms={k: round(v, 3) for k, v in r["step_ms"].items()}, graph=r["graph"],
                    corr_ms_per_launch=r["corr_ms_per_launch"], accuracy=acc.get("f64"),
                    stages_ms_per_pair={k: round(v, 4) for k, v in r["stages_ms_per_pair"].items()})
        if uniform:
            bpp64 = path_bytes(D, True)
            fp64["path_roofline"] = dict(bytes_per_pair=bpp64, frac=round(r["value"] / (HBM_PEAK_GBS * 1e9 / bpp64), 4))
    stage_roofs = {}
    for k, per in head["stages_ms_per_pair"].items():
        rr = roofline_of(k, D, mode_f64, per) if uniform else None   # the per-pair share of device time
        if rr:
            stage_roofs[k] = {kk: rr[kk] for kk in ("bound", "frac", "achieved", "unit")}
    config = {"workload": wl["label"] + f"; {args.mode.upper()} mode; batch of {args.batch} distinct pairs per step "
                                       f"(one batched run)",
              "global_batch": args.batch, "frame": D["N"] if same_shape else "mixed",
              "fft_size": D["P"] if same_shape else "= N", "coefficients": D["ncoef"] if same_shape else "mixed",
              "corr_chunk_autotune": head["corr_chunk_autotune"]}
    out = {
        "metric": METRIC,
        "value": round(value, 3) if ok else None,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if mode_f64 else "f32+f64",
        "data": "synthetic",
        "config": config,
        "roofline": roof,
        "cpu_baseline": cpu,
        "measured_value": round(value, 3),
        "accuracy": acc.get(args.mode),
        "cond_omega_pair0": cond,
        "step_ms": {k: round(v, 3) for k, v in head["step_ms"].items()},
        "graph": head["graph"],
        "megapixels_per_s": round(value * mpx, 2),
        "path_roofline": path,
        "attainable_hbm_gbs": round(copy_gbs, 1),
        "fp64": fp64,
        "stages_ms_per_pair": {k: round(v, 4) for k, v in head["stages_ms_per_pair"].items()},
        "stage_rooflines": stage_roofs,
        "assembly_routes": routes,
        "pipeline_steps": steps,
    }
    if tmpl_of is not None:
        out["config"]["templates"] = len(set(tmpl_of))
        out["config"]["epochs_per_template"] = ST_EPOCHS
        out["unshared"] = unshared
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
