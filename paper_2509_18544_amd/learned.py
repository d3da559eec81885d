"""Learned warm start of the subtraction: dataset, GPU training, fallback policy.

A fully connected network (include/sfft_mlp.h; default widths 2180 -> 512 ->
512 -> 512 -> 2166) maps the science and template PSF stamps (33 x 33 each,
unit sum, taken at the frame centre) and the frame's focal-plane position
(X, Y) to the 2166 kernel coefficients of a w = 9, DK = 2 fit.  It is
trained on solutions that the library itself computes (FP64 solves with one
refinement step), by the library's own forward/backward/Adam kernels.

Policy for one pair (``WarmStart.subtract``): build the normal system, let
the network predict the kernel, complete it with the least-squares
background (sfft_fit_background) and judge it with
rho = ||beta - Omega theta|| / ||beta|| (sfft_residual).  If rho <= tau the
prediction is used; otherwise the plain Cholesky solve runs (the fallback).
Without the threshold test (``quick_look``) the prediction gives a
difference image with no solve at all.

Host-side work here is argument marshalling and bookkeeping only: feature
vectors are concatenations of the stamps and (X, Y), standardised with
per-feature statistics of the training set; every product of the network
and every step of the subtraction runs in the HIP library.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import binding as B

DIMS = (2180, 512, 512, 512, 2166)
STAMP = 33
W, DK, DB = 9, 2, 2


def features(stamp_s, stamp_t, X, Y) -> np.ndarray:
    """Network input: both stamps flattened, then (X, Y)."""
    return np.concatenate([np.asarray(stamp_s, np.float64).ravel(), np.asarray(stamp_t, np.float64).ravel(),
                           [float(X), float(Y)]])


def pair_features(pair) -> np.ndarray:
    t = pair.truth
    return features(t["stamp_s"], t["stamp_t"], t["X"], t["Y"])


class Standardizer:
    """Per-column affine map z = (v - mean) / std, std floored at `floor` * max std."""

    def __init__(self, mean, std):
        self.mean = np.asarray(mean, np.float64)
        self.std = np.asarray(std, np.float64)

    @classmethod
    def fit(cls, data, floor=1e-6):
        data = np.asarray(data, np.float64)
        mean = data.mean(axis=0)
        std = data.std(axis=0)
        std = np.maximum(std, floor * max(float(std.max()), 1e-300))
        return cls(mean, std)

    def apply(self, v):
        return (np.asarray(v, np.float64) - self.mean) / self.std

    def to_dict(self):
        return dict(mean=self.mean.tolist(), std=self.std.tolist())

    @classmethod
    def from_dict(cls, d):
        return cls(d["mean"], d["std"])


# ---------------------------------------------------------------- data from the method's own solves

def solve_pairs(pairs, mode=B.SFFT_MODE_F64, stream=None):
    """FP64 coefficient vectors of equally shaped pairs, one batched run."""
    import torch
    dt = torch.float64 if mode == B.SFFT_MODE_F64 else torch.float32
    descs = [B.make_desc(p.sci.shape[0], p.sci.shape[1], p.w, p.dk, p.db, mode) for p in pairs]
    h = B.sfft_batch_plan(descs, stream)
    try:
        S = [torch.from_numpy(p.sci).to("cuda", dt) for p in pairs]
        R = [torch.from_numpy(p.tmpl).to("cuda", dt) for p in pairs]
        M = [torch.from_numpy(p.mask).cuda() for p in pairs]
        n = B.sfft_num_coeffs(descs[0])
        C = torch.zeros((len(pairs), n), dtype=torch.float64, device="cuda")
        Dd = [torch.empty_like(s) for s in S]
        info = torch.zeros(len(pairs), dtype=torch.int32, device="cuda")
        B.sfft_batch_run(h, S, R, M, [s.stride(0) for s in S], list(C), Dd, info)
        torch.cuda.synchronize()
        return C.cpu().numpy(), info.cpu().numpy()
    finally:
        B.sfft_destroy(h)


def _render(args):
    import synth
    seed, n = args
    p = synth.pair_ws(seed, n=n, w=W, dk=DK, db=DB)
    return seed, p


def make_dataset(npairs, seed0, n=512, chunk=32, pool=None, log=None):
    """Render `npairs` frames (synth.pair_ws, seeds seed0..) and solve them.

    Returns (features [npairs, 2180] float64, theta [npairs, ncoef] float64,
    info [npairs]).  `pool` (an executor created before the GPU was touched)
    renders in parallel; without it frames are rendered in this process.
    """
    feats, thetas, infos, params = [], [], [], []
    seeds = [(seed0 + i, n) for i in range(npairs)]
    it = pool.map(_render, seeds, chunksize=4) if pool is not None else map(_render, seeds)
    buf = []
    t0 = time.perf_counter()
    for _, p in it:
        buf.append(p)
        if len(buf) == chunk or (len(feats) + len(buf)) == npairs:
            th, info = solve_pairs(buf)
            feats.extend(pair_features(q) for q in buf)
            params.extend([q.truth["X"], q.truth["Y"], q.truth["fwhm_s0"], q.truth["fwhm_t0"]] for q in buf)
            thetas.append(th)
            infos.append(info)
            buf = []
            if log:
                log(f"[learned] solved {len(feats)}/{npairs} pairs ({time.perf_counter() - t0:.1f}s)")
    make_dataset.last_params = np.asarray(params)     # (X, Y, FWHM_s0, FWHM_t0) per frame, for diagnostics
    return np.asarray(feats), np.concatenate(thetas), np.concatenate(infos)


# ---------------------------------------------------------------- 4088^2 frames rendered on the GPU

RT = 32   # catalogue tile side of the renderer (include/sfft_render.h)


def ws_frame_host(args):
    """Catalogue of one warm-start frame (synth.ws_catalog) in the renderer's tile
    order, for a host worker pool: returns (seed, catalogue, sorted arrays, tile_start)."""
    import synth
    seed, n = args
    cat = synth.ws_catalog(seed, n=n)
    nt = -(-n // RT)
    tx = np.clip(np.floor(cat["xs"] / RT), 0, nt - 1).astype(np.int64)
    ty = np.clip(np.floor(cat["ys"] / RT), 0, nt - 1).astype(np.int64)
    tile = ty * nt + tx
    order = np.argsort(tile, kind="stable")
    start = np.concatenate([[0], np.cumsum(np.bincount(tile, minlength=nt * nt))]).astype(np.int32)
    arrays = np.stack([cat[k][order] for k in ("xs", "ys", "flux", "fw_s", "fw_t", "mask_r")])
    small = {k: cat[k] for k in ("n", "X", "Y", "fwhm_s0", "fwhm_t0", "beta", "bc", "noise_seed", "stamp_s",
                                 "stamp_t")}
    return seed, small, arrays, start


class FrameRenderer:
    """Device buffers for `nbuf` frames of side n and the GPU rendering of catalogues into them."""

    def __init__(self, nbuf, n, stream=None):
        import torch
        self.n = n
        self.S = [torch.empty((n, n), dtype=torch.float64, device="cuda") for _ in range(nbuf)]
        self.R = [torch.empty_like(x) for x in self.S]
        self.M = [torch.empty((n, n), dtype=torch.uint8, device="cuda") for _ in range(nbuf)]
        self.overflow = torch.zeros(1, dtype=torch.int32, device="cuda")
        self.keep = []
        self.stream = stream

    def render(self, k, small, arrays, start):
        """Frame k <- the catalogue (host arrays from ws_frame_host)."""
        import torch
        A = torch.from_numpy(np.ascontiguousarray(arrays)).cuda()
        T = torch.from_numpy(start).cuda()
        norm = torch.empty(2 * max(1, arrays.shape[1]), dtype=torch.float64, device="cuda")
        f = B.sfft_ws_frame()
        f.n, f.nstar, f.beta = self.n, arrays.shape[1], small["beta"]
        for i in range(6):
            f.bc[i] = float(small["bc"][i])
        f.noise_seed = int(small["noise_seed"])
        f.xs, f.ys, f.flux, f.fw_s, f.fw_t, f.mask_r = (A[i].data_ptr() for i in range(6))
        f.tile_start = T.data_ptr()
        B.sfft_render_ws_frame(f, self.S[k], self.R[k], self.M[k], self.n, norm, self.overflow, self.stream)
        self.keep.append((A, T, norm))           # alive until the stream has run the kernels

    def settle(self):
        import torch
        torch.cuda.synchronize()
        self.keep = []
        if int(self.overflow.item()) != 0:
            raise RuntimeError("a render neighbourhood held more stars than the renderer stages")


def make_dataset_gpu(npairs, seed0, n=4088, chunk=32, pool=None, log=None):
    """`npairs` frames of side n rendered on the GPU from host catalogues (seeds
    seed0..) and solved in FP64 batches of `chunk` (one batch plan, reused).
    Returns (features, theta, info) like make_dataset; make_dataset_gpu.last_params
    holds (X, Y, FWHM_s0, FWHM_t0, beta) per frame."""
    import torch
    desc = B.make_desc(n, n, W, DK, DB, B.SFFT_MODE_F64)
    ncoef = B.sfft_num_coeffs(desc)
    rend = FrameRenderer(chunk, n)
    h = B.sfft_batch_plan([desc] * chunk)
    C = torch.zeros((chunk, ncoef), dtype=torch.float64, device="cuda")
    Dd = [torch.empty((n, n), dtype=torch.float64, device="cuda") for _ in range(chunk)]
    info = torch.zeros(chunk, dtype=torch.int32, device="cuda")
    feats, thetas, infos, params = [], [], [], []
    seeds = [(seed0 + i, n) for i in range(npairs)]
    chunks = [seeds[i:i + chunk] for i in range(0, npairs, chunk)]
    t0 = time.perf_counter()
    nxt = pool.map(ws_frame_host, chunks[0]) if pool is not None else map(ws_frame_host, chunks[0])
    try:
        for ci in range(len(chunks)):
            cur = list(nxt)
            if ci + 1 < len(chunks):   # the next catalogues are drawn while this batch runs
                nxt = pool.map(ws_frame_host, chunks[ci + 1]) if pool is not None else map(ws_frame_host, chunks[ci + 1])
            for k, (_, small, arrays, start) in enumerate(cur):
                rend.render(k, small, arrays, start)
            m = len(cur)
            if m == chunk:
                B.sfft_batch_run(h, rend.S, rend.R, rend.M, [n] * chunk, list(C), Dd, info)
                th, inf = C.cpu().numpy().copy(), info.cpu().numpy().copy()
            else:   # a short last batch: its own plan
                h2 = B.sfft_batch_plan([desc] * m)
                try:
                    B.sfft_batch_run(h2, rend.S[:m], rend.R[:m], rend.M[:m], [n] * m, list(C[:m]), Dd[:m], info[:m])
                    th, inf = C[:m].cpu().numpy().copy(), info[:m].cpu().numpy().copy()
                finally:
                    B.sfft_destroy(h2)
            rend.settle()
            for (_, small, _, _) in cur:
                feats.append(features(small["stamp_s"], small["stamp_t"], small["X"], small["Y"]))
                params.append([small["X"], small["Y"], small["fwhm_s0"], small["fwhm_t0"], small["beta"]])
            thetas.append(th)
            infos.append(inf)
            if log and (ci % 10 == 9 or ci == len(chunks) - 1):
                log(f"[learned] rendered and solved {len(feats)}/{npairs} frames of {n}^2 "
                    f"({time.perf_counter() - t0:.1f}s)")
    finally:
        B.sfft_destroy(h)
    make_dataset_gpu.last_params = np.asarray(params)
    return np.asarray(feats), np.concatenate(thetas), np.concatenate(infos)


# ---------------------------------------------------------------- the network

def he_uniform(dims, seed):
    """FP32 parameter vector: He-uniform weights, zero biases (packing of include/sfft_mlp.h)."""
    rng = np.random.default_rng(seed)
    parts = []
    for i in range(len(dims) - 1):
        lim = np.sqrt(6.0 / dims[i])
        parts.append(rng.uniform(-lim, lim, dims[i] * dims[i + 1]))
        parts.append(np.zeros(dims[i + 1]))
    return np.concatenate(parts).astype(np.float32)


class Net:
    """Network parameters, Adam state and standardisers, with the library handle."""

    def __init__(self, dims=DIMS, max_batch=256, seed=0, stream=None):
        import torch
        self.dims = tuple(int(d) for d in dims)
        self.max_batch = int(max_batch)
        self.handle = B.sfft_mlp_create(self.dims, self.max_batch, stream)
        n = B.sfft_mlp_param_count(self.handle)
        self.params = torch.from_numpy(he_uniform(self.dims, seed)).cuda()
        assert self.params.numel() == n
        self.m1 = torch.zeros_like(self.params)
        self.m2 = torch.zeros_like(self.params)
        self.step = 0
        self.xs = None      # input standardiser
        self.ys = None      # output standardiser
        self._bf16_step = -1
        self._scale = self._shift = None

    # ---- training (FP32 kernels)
    def train(self, feats, targets, epochs=30, batch=128, lr=1e-4, lr_final=1e-6, seed=0, log=None):
        """Adam on the MSE of standardised targets (cosine-decayed step size).  Returns the per-epoch
        mean losses.  The inputs are strongly collinear (stamp pixels), so steps much above 1e-4
        drive the network to the constant mean prediction."""
        import torch
        if self.xs is None:
            self.xs = Standardizer.fit(feats)
            self.ys = Standardizer.fit(targets)
        X = torch.from_numpy(self.xs.apply(feats).astype(np.float32)).cuda()
        T = torch.from_numpy(self.ys.apply(targets).astype(np.float32)).cuda()
        ns = X.shape[0]
        batch = min(batch, self.max_batch, ns)
        Y = torch.empty((batch, self.dims[-1]), device="cuda")
        dY = torch.empty_like(Y)
        G = torch.empty_like(self.params)
        loss = torch.zeros(1, dtype=torch.float64, device="cuda")
        rng = np.random.default_rng(seed)
        steps_total = epochs * (ns // batch)
        hist = []
        for ep in range(epochs):
            perm = torch.from_numpy(rng.permutation(ns)).cuda()
            acc = torch.zeros(1, dtype=torch.float64, device="cuda")
            nb = ns // batch
            for b in range(nb):
                idx = perm[b * batch:(b + 1) * batch]
                xb = X.index_select(0, idx)
                tb = T.index_select(0, idx)
                B.sfft_mlp_forward(self.handle, self.params, xb, batch, Y)
                B.sfft_mlp_mse(self.handle, Y, tb, batch, dY, loss)
                B.sfft_mlp_backward(self.handle, self.params, xb, dY, batch, G)
                self.step += 1
                # cosine decay from lr to lr_final over the run
                frac = min(1.0, (ep * nb + b) / max(1, steps_total - 1))
                lr_t = lr_final + 0.5 * (lr - lr_final) * (1.0 + np.cos(np.pi * frac))
                B.sfft_mlp_adam_step(self.handle, self.params, G, self.m1, self.m2, self.step, lr=lr_t)
                acc += loss
            hist.append(float(acc.item()) / nb)
            if log:
                log(f"[learned] epoch {ep + 1}/{epochs}: loss {hist[-1]:.4f}")
        return hist

    # ---- inference (BF16 kernels)
    def predict(self, feats, theta, ld):
        """Kernel coefficients of each row of `feats` into theta[i*ld : i*ld + dims[-1]] (device FP64)."""
        import torch
        if self._bf16_step != self.step:
            B.sfft_mlp_set_weights_bf16(self.handle, self.params)
            self._scale = torch.from_numpy(self.ys.std).cuda()
            self._shift = torch.from_numpy(self.ys.mean).cuda()
            self._bf16_step = self.step
        x = torch.from_numpy(self.xs.apply(np.atleast_2d(feats)).astype(np.float32)).cuda()
        nb = x.shape[0]
        for s in range(0, nb, self.max_batch):
            k = min(self.max_batch, nb - s)
            B.sfft_mlp_infer(self.handle, x[s:s + k], k, self._scale, self._shift,
                             theta.view(-1)[s * ld:], ld)
        return theta

    # ---- checkpoint: raw little-endian FP32 .bin + JSON header, resumable
    def save(self, path):
        blobs = [self.params, self.m1, self.m2]
        with open(path + ".bin", "wb") as f:
            for t in blobs:
                f.write(t.cpu().numpy().astype("<f4").tobytes())
        hdr = dict(format="sfft-mlp-1", dims=list(self.dims), step=self.step, count=int(self.params.numel()),
                   blobs=["params", "adam_m1", "adam_m2"], dtype="float32-le",
                   x_std=self.xs.to_dict(), y_std=self.ys.to_dict())
        with open(path + ".json", "w") as f:
            json.dump(hdr, f)

    @classmethod
    def load(cls, path, max_batch=256, stream=None):
        import torch
        hdr = json.load(open(path + ".json"))
        if hdr.get("format") != "sfft-mlp-1":
            raise ValueError(f"{path}.json is not a network checkpoint")
        net = cls(hdr["dims"], max_batch=max_batch, stream=stream)
        raw = np.fromfile(path + ".bin", dtype="<f4")
        n = hdr["count"]
        if raw.size != 3 * n or net.params.numel() != n:
            raise ValueError(f"{path}.bin holds {raw.size} values, expected {3 * n}")
        net.params = torch.from_numpy(raw[:n].copy()).cuda()
        net.m1 = torch.from_numpy(raw[n:2 * n].copy()).cuda()
        net.m2 = torch.from_numpy(raw[2 * n:].copy()).cuda()
        net.step = int(hdr["step"])
        net.xs = Standardizer.from_dict(hdr["x_std"])
        net.ys = Standardizer.from_dict(hdr["y_std"])
        return net

    def close(self):
        if getattr(self, "handle", None):
            B.sfft_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- warm start with fallback

class WarmStart:
    """Network guess judged by the method's own residual; the plain solve is the fallback."""

    def __init__(self, net, tau=1e-5):
        self.net = net
        self.tau = float(tau)
        self.calls = 0
        self.fallbacks = 0

    def coefficients(self, plan, feats, coeffs=None):
        """Predicted kernel + fitted background for a plan whose system is built.  Returns coeffs."""
        import torch
        if coeffs is None:
            coeffs = torch.zeros(plan.n, dtype=torch.float64, device="cuda")
        self.net.predict(feats, coeffs, plan.n)
        plan.fit_background(coeffs)
        return coeffs

    def subtract(self, plan, sci, tmpl, mask, feats, diff=None):
        """Returns (coeffs, diff, rho, used_guess).

        Raises SfftError (SFFT_ENOTSPD / SFFT_ENONFINITE) when the guess is
        rejected and the fallback solve fails too: the rejected guess is never
        used for the difference image."""
        plan.build(sci, tmpl, mask)
        coeffs = self.coefficients(plan, feats)
        rho = float(plan.residual(coeffs).item())        # synchronises
        self.calls += 1
        used = np.isfinite(rho) and rho <= self.tau
        if not used:
            self.fallbacks += 1
            plan.solve(coeffs)
            st, info, nonfinite = plan.status()          # synchronises
            if st != B.SFFT_OK:
                raise B.SfftError(st, f"fallback solve (info={info}, nonfinite={nonfinite})")
        diff = plan.subtract(sci, tmpl, coeffs, diff)
        return coeffs, diff, rho, used

    @property
    def fallback_rate(self):
        return self.fallbacks / max(1, self.calls)


# ---------------------------------------------------------------- command line: train and evaluate

def _cli(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--train-pairs", type=int, default=20000)
    ap.add_argument("--val-pairs", type=int, default=64)
    ap.add_argument("--frames", choices=["gpu", "host"], default="gpu",
                    help="gpu: frames rendered by the library's renderer (synth.ws_catalog recipe, any n); "
                         "host: synth.pair_ws rendered on the host (small n)")
    ap.add_argument("--n", type=int, default=4088, help="frame side of the training frames")
    ap.add_argument("--test-pairs", type=int, default=0, help="held-out frames for the evaluation (default val)")
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--lr", type=float, default=1e-4)
    ap.add_argument("--seed0", type=int, default=500000)
    ap.add_argument("--workers", type=int, default=16)
    ap.add_argument("--save", default=None, help="checkpoint path prefix (.bin + .json)")
    ap.add_argument("--report", default=None, help="write the evaluation as JSON here")
    ap.add_argument("--dump", default=None, help="also save the dataset (.npz) here")
    ap.add_argument("--dump-only", action="store_true", help="stop after building (and saving) the dataset")
    a = ap.parse_args(argv)
    log = lambda *m: print(*m, file=sys.stderr, flush=True)  # noqa: E731

    import concurrent.futures as cf
    import multiprocessing as mp
    # the host pool starts before anything touches the GPU
    pool = cf.ProcessPoolExecutor(max_workers=max(1, a.workers), mp_context=mp.get_context("spawn"))
    warm = ws_frame_host if a.frames == "gpu" else _render
    list(pool.map(warm, [(0, 64)] * max(1, a.workers)))

    import torch
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    build = make_dataset_gpu if a.frames == "gpu" else make_dataset
    Xtr, THtr, info = build(a.train_pairs, a.seed0, n=a.n, pool=pool, log=log)
    Ptr = build.last_params
    Xva, THva, info_v = build(a.val_pairs, a.seed0 + 10 ** 6, n=a.n, pool=pool, log=log)
    Pva = build.last_params
    pool.shutdown()
    t_data = time.perf_counter() - t0
    if a.dump:
        np.savez_compressed(a.dump, Xtr=Xtr.astype(np.float32), THtr=THtr, Ptr=Ptr, info=info,
                            Xva=Xva.astype(np.float32), THva=THva, Pva=Pva)
        log(f"[learned] wrote {a.dump}")
    if a.dump_only:
        return
    ok = info == 0
    log(f"[learned] dataset: {ok.sum()} usable of {len(ok)} ({time.perf_counter() - t0:.1f}s)")
    nk = DIMS[-1]
    net = Net(DIMS, max_batch=a.batch)
    t1 = time.perf_counter()
    hist = net.train(Xtr[ok], THtr[ok, :nk], epochs=a.epochs, batch=a.batch, lr=a.lr, log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    if a.save:
        net.save(a.save)
    ntest = a.test_pairs or a.val_pairs
    base = THtr[ok].mean(axis=0)
    if a.frames == "gpu":
        rep = evaluate_gpu(net, ntest, a.seed0 + 2 * 10 ** 6, n=a.n, base_mean=base, log=log)
    else:
        rep = evaluate(net, ntest, a.seed0 + 10 ** 6, n=a.n, theta_ref=THva, base_mean=base)
    # validation loss of the trained network on the held-out validation frames
    import torch as _t
    nv = min(len(Xva), net.max_batch)
    Yv = _t.empty((nv, net.dims[-1]), device="cuda")
    B.sfft_mlp_forward(net.handle, net.params, _t.from_numpy(net.xs.apply(Xva[:nv]).astype(np.float32)).cuda(), nv, Yv)
    resid = Yv.cpu().numpy() - net.ys.apply(THva[:nv, :nk])
    rep.update(train_pairs=int(ok.sum()), epochs=a.epochs, train_seconds=t_train, final_loss=hist[-1],
               loss_first=hist[0], frames=a.frames, data_seconds=t_data,
               val_loss=float(np.mean(resid ** 2)), val_explained=float(1.0 - np.mean(resid ** 2)))
    print(json.dumps(rep))
    if a.report:
        with open(a.report, "w") as f:
            json.dump(rep, f, indent=1)


def _eval_frame(plan, ws, S, R, M, f, base_mean, nk, ev):
    """One held-out frame: the full solve path and the quick look (both timed
    after a warm-up), rho of the guess, the policy, and the mean-kernel baseline.
    Returns (e_kernel_net, e_kernel_mean, e_diff_net, e_diff_mean, rho, ms_full,
    ms_quick, ms_policy)."""
    import torch
    for _ in range(2):                     # first pass warms up, second is timed
        ev[0].record()
        plan.build(S, R, M)
        c_full, _ = plan.solve()
        d_full = plan.subtract(S, R, c_full)
        ev[1].record()
        torch.cuda.synchronize()
    t_full = ev[0].elapsed_time(ev[1])
    for _ in range(2):
        ev[0].record()
        plan.build(S, R, M)
        c_q = ws.coefficients(plan, f)
        d_q = plan.subtract(S, R, c_q)
        ev[1].record()
        torch.cuda.synchronize()
    t_quick = ev[0].elapsed_time(ev[1])
    rho = float(plan.residual(c_q).item())
    t = time.perf_counter()
    ws.subtract(plan, S, R, M, f)
    torch.cuda.synchronize()
    t_policy = 1e3 * (time.perf_counter() - t)
    c_b = torch.from_numpy(np.asarray(base_mean, np.float64).copy()).cuda()
    plan.fit_background(c_b)
    d_b = plan.subtract(S, R, c_b)
    ref = c_full.cpu().numpy()
    cq, cb = c_q.cpu().numpy(), c_b.cpu().numpy()
    df = d_full.cpu().numpy()
    return (np.linalg.norm(cq[:nk] - ref[:nk]) / np.linalg.norm(ref[:nk]),
            np.linalg.norm(cb[:nk] - ref[:nk]) / np.linalg.norm(ref[:nk]),
            np.linalg.norm(d_q.cpu().numpy() - df) / np.linalg.norm(df),
            np.linalg.norm(d_b.cpu().numpy() - df) / np.linalg.norm(df), rho, t_full, t_quick, t_policy)


def _report(rows, ws, npairs, n, tau):
    r = np.asarray(rows, np.float64)
    med = lambda k: float(np.median(r[:, k]))  # noqa: E731
    return dict(val_pairs=npairs, n=n, tau=tau,
                e_kernel_net=med(0), e_kernel_mean=med(1),
                e_diff_quicklook_net=med(2), e_diff_quicklook_mean=med(3),
                rho_median=med(4), rho_min=float(r[:, 4].min()), fallback_rate=ws.fallback_rate,
                ms_full=med(5), ms_quicklook=med(6), ms_policy=med(7),
                pairs_per_s_full=1e3 / med(5), pairs_per_s_quicklook=1e3 / med(6))


def evaluate(net, npairs, seed0, n=512, theta_ref=None, base_mean=None, tau=1e-5, log=None):
    """Gain of the network on held-out frames (synth.pair_ws, host-rendered):
    coefficient and quick-look errors against the full solve, rho and fallback
    rate, and per-pair times."""
    import torch
    import synth
    ws = WarmStart(net, tau)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    rows = []
    plan = B.Plan(n, n, W, DK, DB, mode=B.SFFT_MODE_F64)
    try:
        for i in range(npairs):
            p = synth.pair_ws(seed0 + i, n=n, w=W, dk=DK, db=DB)
            S = torch.from_numpy(p.sci).cuda()
            R = torch.from_numpy(p.tmpl).cuda()
            M = torch.from_numpy(p.mask).cuda()
            rows.append(_eval_frame(plan, ws, S, R, M, pair_features(p), base_mean, net.dims[-1], ev))
    finally:
        plan.close()
    return _report(rows, ws, npairs, n, tau)


def evaluate_gpu(net, npairs, seed0, n=4088, base_mean=None, tau=1e-5, log=None):
    """The same evaluation on frames rendered on the GPU (synth.ws_catalog recipe)."""
    import torch
    ws = WarmStart(net, tau)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    rows = []
    rend = FrameRenderer(1, n)
    plan = B.Plan(n, n, W, DK, DB, mode=B.SFFT_MODE_F64)
    try:
        for i in range(npairs):
            _, small, arrays, start = ws_frame_host((seed0 + i, n))
            rend.render(0, small, arrays, start)
            rend.settle()
            f = features(small["stamp_s"], small["stamp_t"], small["X"], small["Y"])
            rows.append(_eval_frame(plan, ws, rend.S[0], rend.R[0], rend.M[0], f, base_mean, net.dims[-1], ev))
            if log and i % 16 == 15:
                log(f"[learned] evaluated {i + 1}/{npairs}")
    finally:
        plan.close()
    return _report(rows, ws, npairs, n, tau)


if __name__ == "__main__":
    _cli(sys.argv[1:])
