"""Cross-convolution (pipeline step 5) and kernel application on the GPU
through the C ABI (sfft_apply_kernel) against the CPU FP64 oracle.

Bars (relative 2-norm error against the oracle on the same inputs): FP64
<= 1e-12; FP32C <= 1e-6 (the output is rounded to float32 once, 6e-8
relative per pixel; the arithmetic is FP64).  At 4088 x 4088 the oracle runs
on crops: the four corners (which carry the zero boundary) and the centre,
each with an s-wide margin on the inner sides.
"""
import numpy as np
import pytest

import oracle
import synth
from paper_2509_18544_amd import binding as B

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

F64, F32C = B.SFFT_MODE_F64, B.SFFT_MODE_F32C
BAR = {F64: 1e-12, F32C: 1e-6}


def _apply(img, kcoef, w, dk, mode):
    dt = torch.float64 if mode == F64 else torch.float32
    X = torch.from_numpy(np.ascontiguousarray(img)).to("cuda", dt)
    K = torch.from_numpy(np.asarray(kcoef, np.float64)).cuda()
    plan = B.Plan(img.shape[0], img.shape[1], w, dk, 0, mode=mode)
    try:
        out = plan.apply_kernel(X, K)
        torch.cuda.synchronize()
        return out.cpu().numpy().astype(np.float64)
    finally:
        plan.close()


def _as_seen(img, mode):
    return img.astype(np.float32).astype(np.float64) if mode == F32C else img


@pytest.mark.parametrize("mode", [F64, F32C])
@pytest.mark.parametrize("shape,s", [((64, 64), 2), ((100, 90), 5), ((130, 129), 9), ((96, 128), 15),
                                     ((37, 41), 1), ((70, 66), 0)])
def test_psf_convolution(shape, s, mode):
    p = synth.random_pair(400 + s, shape[0], shape[1], s, 0, 0, mask_frac=0.0, stars=True)
    stamp = synth.psf_stamp(2.2, 3.0, half=s) if s > 0 else np.array([[1.7]])
    got = _apply(p.sci, stamp.ravel(), s, 0, mode)
    ref = oracle.convolve(_as_seen(p.sci, mode), stamp)
    e = oracle.rel_err(got, ref)
    print(f"{shape} s={s} mode={mode}: e={e:.2e}")
    assert e <= BAR[mode]


@pytest.mark.parametrize("mode", [F64, F32C])
@pytest.mark.parametrize("w,dk", [(3, 1), (4, 2), (2, 4)])
def test_spatially_varying_kernel(w, dk, mode):
    p = synth.random_pair(500 + dk, 120, 110, w, dk, 0, mask_frac=0.0, stars=True)
    L = 2 * w + 1
    kc = np.random.default_rng(dk).normal(size=oracle.num_basis(dk) * L * L)
    got = _apply(p.tmpl, kc, w, dk, mode)
    ref = oracle.apply_kernel(_as_seen(p.tmpl, mode), kc, w, dk)
    e = oracle.rel_err(got, ref)
    print(f"w={w} dk={dk} mode={mode}: e={e:.2e}")
    assert e <= BAR[mode]


@pytest.mark.parametrize("mode", [F32C, F64])
def test_cross_convolution_4088(mode):
    """S' = P_T * S and R' = P_S * R of a 4088^2 Roman-like pair with 31 x 31 Moffat
    stamps of the two PSFs (FWHM 1.8 template, 2.2 science, beta 3)."""
    p = synth.pair_c3(seed=1003)
    s = 15
    pt = synth.psf_stamp(1.8, 3.0, half=s)
    ps = synth.psf_stamp(2.2, 3.0, half=s)
    S2 = _apply(p.sci, pt.ravel(), s, 0, mode)
    R2 = _apply(p.tmpl, ps.ravel(), s, 0, mode)
    n = p.sci.shape[0]
    c = 128
    worst = 0.0
    for (y0, x0) in ((0, 0), (0, n - c), (n - c, 0), (n - c, n - c), (n // 2, n // 2)):
        ya, xa = max(0, y0 - s), max(0, x0 - s)
        yb, xb = min(n, y0 + c + s), min(n, x0 + c + s)
        for img, stamp, got in ((p.sci, pt, S2), (p.tmpl, ps, R2)):
            crop = oracle.convolve(_as_seen(img[ya:yb, xa:xb], mode), stamp)
            ref = crop[y0 - ya:y0 - ya + c, x0 - xa:x0 - xa + c]
            e = oracle.rel_err(got[y0:y0 + c, x0:x0 + c], ref)
            worst = max(worst, e)
            assert e <= BAR[mode], ((y0, x0), e)
    print(f"4088 cross-convolution mode={mode}: worst crop e={worst:.2e}")


def test_apply_kernel_rejects_in_place():
    plan = B.Plan(64, 64, 2, 0, 0, mode=F64)
    try:
        X = torch.zeros((64, 64), dtype=torch.float64, device="cuda")
        K = torch.zeros(25, dtype=torch.float64, device="cuda")
        with pytest.raises(B.SfftError) as e:
            B.sfft_apply_kernel(plan.handle, X, K, X, 64)
        assert e.value.status == B.SFFT_EINVAL
    finally:
        plan.close()
