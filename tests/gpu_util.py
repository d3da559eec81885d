"""Helpers for the GPU tests: run one pair through the C ABI with torch buffers."""
from __future__ import annotations

import numpy as np

from paper_2509_18544_amd import binding as B


def to_dev(a, dtype, pitch=None):
    import torch
    a = np.ascontiguousarray(a)
    ny, nx = a.shape
    if pitch is None or pitch == nx:
        return torch.from_numpy(a).to(device="cuda", dtype=dtype)
    full = torch.zeros((ny, pitch), dtype=dtype, device="cuda")
    full[:, :nx] = torch.from_numpy(a).to(device="cuda", dtype=dtype)
    return full[:, :nx]


def run_pair(sci, tmpl, mask, w, dk, db, mode=B.SFFT_MODE_F64, pitch=None, refine_steps=-1,
             theta_in=None, want_system=True, flags=0):
    """Build, solve and subtract one pair on cuda:0.  Returns host numpy results."""
    import torch
    ny, nx = sci.shape
    dt = torch.float64 if mode == B.SFFT_MODE_F64 else torch.float32
    S = to_dev(sci, dt, pitch)
    R = to_dev(tmpl, dt, pitch)
    M = None if mask is None else to_dev(mask.astype(np.uint8), torch.uint8, pitch)
    ld = S.stride(0)
    plan = B.Plan(ny, nx, w, dk, db, mode=mode, refine_steps=refine_steps, flags=flags)
    try:
        plan.build(S, R, M)
        out = {}
        if want_system:
            om, be = plan.system()
            out["omega"], out["beta"] = om, be
        coeffs, info = plan.solve()
        theta_used = coeffs if theta_in is None else torch.from_numpy(np.asarray(theta_in, np.float64)).cuda()
        diff = torch.full_like(S, float("nan")) if pitch is None else to_dev(np.zeros_like(sci), dt, pitch)
        B.sfft_subtract(plan.handle, S, R, theta_used, diff, ld)
        rho = plan.residual(coeffs)
        st, inf, nf = plan.status()
        torch.cuda.synchronize()
        res = {k: v.cpu().numpy().astype(np.float64) for k, v in out.items()}
        res.update(theta=coeffs.cpu().numpy(), diff=diff.cpu().numpy().astype(np.float64),
                   info=int(info.cpu().item()), status=st, info_flag=inf, nonfinite=nf,
                   rho=float(rho.cpu().item()))
        return res
    finally:
        plan.close()


def oracle_reference(args):
    """(theta*, D*) of one pair from the CPU oracle, for a process pool:
    args = (sci, tmpl, mask, w, dk, db, input dtype name)."""
    import oracle
    sci, tmpl, mask, w, dk, db, cast = args
    s_in = sci.astype(cast).astype(np.float64)
    r_in = tmpl.astype(cast).astype(np.float64)
    ref = oracle.fit(s_in, r_in, mask, w, dk, db, mode="fft")
    return ref["theta"], ref["diff"]


def pin_worker(cores, counter):
    """Pool initializer: one host core per worker process, so that the oracle
    (whose FFT thread count follows the affinity mask) runs single-threaded."""
    import os
    with counter.get_lock():
        k = counter.value
        counter.value += 1
    os.sched_setaffinity(0, {cores[k % len(cores)]})
