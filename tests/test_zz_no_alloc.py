"""The no-allocation entry point (sfft_subtract_pair_noalloc) through the C ABI.

Its result must equal the plan path (sfft_plan with its own workspace +
sfft_build_system + sfft_solve + sfft_subtract) bit for bit -- the same
kernels run on the static scratch -- and meet the oracle bar (FP64 <= 1e-9,
FP32C <= 1e-5 relative 2-norm on theta and D).  Two calls in a row on one
GPU, the second with a smaller pair, so that the second runs on the scratch
the first left behind.  A pair too large for the scratch is rejected with
SFFT_ETOOBIG and leaves the outputs untouched.
"""
import numpy as np
import pytest

import oracle
import synth
from paper_2509_18544_amd import binding as B

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

F64, F32C = B.SFFT_MODE_F64, B.SFFT_MODE_F32C
BAR = {F64: 1e-9, F32C: 1e-5}

# (ny, nx, w, dk, db, mask_frac, seed): the second pair is smaller than the first
PAIRS = [(160, 144, 4, 2, 1, 0.10, 11), (96, 80, 3, 1, 2, 0.05, 12)]


def _dev(a, dt):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dt)


def _plan_path(p, mode, S, R, M):
    plan = B.Plan(p.sci.shape[0], p.sci.shape[1], p.w, p.dk, p.db, mode=mode)
    try:
        plan.build(S, R, M)
        coeffs, info = plan.solve()
        diff = plan.subtract(S, R, coeffs)
        st, _, _ = plan.status()
        assert st == B.SFFT_OK, B.strerror(st)
        return coeffs.clone(), diff.clone(), int(info.item())
    finally:
        plan.close()


@pytest.mark.parametrize("mode", [F64, F32C])
def test_noalloc_equals_plan_path_twice(mode):
    dt = torch.float64 if mode == F64 else torch.float32
    for (ny, nx, w, dk, db, frac, seed) in PAIRS:
        print(f"noalloc pair {ny}x{nx} w={w} dk={dk} db={db} mode={mode}", flush=True)
        p = synth.random_pair(seed, ny, nx, w, dk, db, mask_frac=frac, stars=True)
        S, R, M = _dev(p.sci, dt), _dev(p.tmpl, dt), _dev(p.mask, torch.uint8)
        desc = B.make_desc(ny, nx, w, dk, db, mode)
        n = B.sfft_num_coeffs(desc)
        coeffs = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
        diff = torch.full_like(S, float("nan"))
        info = torch.full((1,), -99, dtype=torch.int32, device="cuda")
        B.sfft_subtract_pair_noalloc(desc, S, R, M, S.stride(0), coeffs, diff, info)
        torch.cuda.synchronize()
        c_ref, d_ref, i_ref = _plan_path(p, mode, S, R, M)
        assert int(info.item()) == 0 and i_ref == 0
        assert torch.equal(coeffs, c_ref), "coefficients differ from the plan path"
        assert torch.equal(diff, d_ref), "difference image differs from the plan path"
        cast = np.float32 if mode == F32C else np.float64   # the images as the GPU path receives them
        s_in = p.sci.astype(cast).astype(np.float64)
        r_in = p.tmpl.astype(cast).astype(np.float64)
        ref = oracle.fit(s_in, r_in, p.mask, w, dk, db)
        et = oracle.rel_err(coeffs.cpu().numpy(), ref["theta"])
        ed = oracle.rel_err(diff.cpu().numpy().astype(np.float64), ref["diff"])
        assert et <= BAR[mode] and ed <= BAR[mode], (et, ed)


def test_noalloc_rejects_a_pair_larger_than_the_scratch():
    n = 2048
    desc = B.make_desc(n, n, 9, 2, 2, F64)
    assert B.sfft_workspace_bytes(desc) > B.SFFT_NOALLOC_SCRATCH_BYTES
    # real buffers of the full size, so that nothing could read out of bounds
    S = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    R = torch.zeros_like(S)
    D = torch.full_like(S, 7.0)
    coeffs = torch.full((B.sfft_num_coeffs(desc),), 3.0, dtype=torch.float64, device="cuda")
    with pytest.raises(B.SfftError) as ei:
        B.sfft_subtract_pair_noalloc(desc, S, R, None, n, coeffs, D, None)
    assert ei.value.status == B.SFFT_ETOOBIG
    torch.cuda.synchronize()
    assert bool((D == 7.0).all()) and bool((coeffs == 3.0).all())
    # a fitting pair still runs after the rejection
    ny, nx, w, dk, db, frac, seed = PAIRS[1]
    p = synth.random_pair(seed, ny, nx, w, dk, db, mask_frac=frac, stars=True)
    S2, R2, M2 = _dev(p.sci, torch.float64), _dev(p.tmpl, torch.float64), _dev(p.mask, torch.uint8)
    d2 = B.make_desc(ny, nx, w, dk, db, F64)
    c2 = torch.zeros((B.sfft_num_coeffs(d2),), dtype=torch.float64, device="cuda")
    D2 = torch.empty_like(S2)
    B.sfft_subtract_pair_noalloc(d2, S2, R2, M2, S2.stride(0), c2, D2, None)
    c_ref, d_ref, _ = _plan_path(p, F64, S2, R2, M2)
    assert torch.equal(c2, c_ref) and torch.equal(D2, d_ref)
