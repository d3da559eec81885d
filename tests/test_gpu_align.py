"""Template alignment on the GPU (sfft_align_image, sfft_align_psf) against the
CPU oracle (oracle.align_oracle).

Images: element by element within 1e-12 of the largest output value in FP64
(the same normalised Lanczos-3 sums in another order, the weights from
sincos recurrences instead of numpy's sinc), within 1e-6 in FP32C (float
template as the oracle sees it, float output); masks bit for bit; the
identity map and integer translations bit for bit in FP64.  Maps: identity,
integer shift, rotation + scale + shift, and second- and third-degree
distortions, on ragged template and output shapes, with and without a mask;
at 4088^2, windows of the full frame (corners and centre) against the
oracle on the same windows.  PSF stamps to 1e-13.  Degenerate maps: every
pixel outside the template, and a NaN coefficient, give an all-masked zero
image."""
import math

import numpy as np
import pytest

from oracle import align_oracle as A
from paper_2509_18544_amd import binding as B

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

F64, F32C = B.SFFT_MODE_F64, B.SFFT_MODE_F32C


def _rot(theta, scale, tx, ty):
    c, s = math.cos(theta), math.sin(theta)
    return [tx, scale * c, -scale * s], [ty, scale * s, scale * c]


MAPS = {
    "identity": ([0.0, 1.0, 0.0], [0.0, 0.0, 1.0], (0.0, 0.0)),
    "shift": ([3.0, 1.0, 0.0], [-2.0, 0.0, 1.0], (0.0, 0.0)),
    "rotate": (*_rot(0.21, 0.98, 70.3, 64.8), (60.0, 55.0)),
    "deg2": ([70.1, 1.01, 0.05, 2e-4, -1e-4, 3e-4], [63.7, -0.04, 0.99, 1e-4, 2e-4, -2e-4], (60.0, 55.0)),
    "deg3": ([70.1, 1.01, 0.05, 2e-4, -1e-4, 3e-4, 1e-6, -2e-6, 1e-6, 3e-7],
             [63.7, -0.04, 0.99, 1e-4, 2e-4, -2e-4, -1e-6, 1e-6, 2e-6, -1e-6], (60.0, 55.0)),
}


def _run(img, msk, cx, cy, ref, ny, nx, mode, pitch=None):
    dt = torch.float64 if mode == F64 else torch.float32
    T = torch.from_numpy(np.ascontiguousarray(img)).to("cuda", dt)
    Mk = None if msk is None else torch.from_numpy(np.ascontiguousarray(msk)).cuda()
    if pitch is None:
        out = torch.full((ny, nx), float("nan"), dtype=dt, device="cuda")
        om = torch.full((ny, nx), 7, dtype=torch.uint8, device="cuda")
    else:
        out = torch.full((ny, pitch), float("nan"), dtype=dt, device="cuda")[:, :nx]
        om = torch.full((ny, pitch), 7, dtype=torch.uint8, device="cuda")[:, :nx]
    B.sfft_align_image(B.make_map(cx, cy, ref), mode, T, Mk, out, om)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64), om.cpu().numpy()


def _template(seed, ny, nx, mask_frac=0.02):
    rng = np.random.default_rng(seed)
    yy, xx = np.mgrid[0:ny, 0:nx].astype(np.float64)
    img = 100.0 * np.exp(-((xx - 0.4 * nx) ** 2 + (yy - 0.6 * ny) ** 2) / 50.0) + rng.normal(0, 1, (ny, nx))
    msk = (rng.random((ny, nx)) < mask_frac).astype(np.uint8)
    return img, msk


@pytest.mark.parametrize("mode", [F64, F32C])
@pytest.mark.parametrize("name", list(MAPS))
def test_align_matches_oracle(name, mode):
    cx, cy, ref = MAPS[name]
    img, msk = _template(5, 150, 137)
    seen = img if mode == F64 else img.astype(np.float32).astype(np.float64)
    out, om = _run(img, msk, cx, cy, ref, 130, 121, mode, pitch=128)
    ref_img, ref_m = A.resample(seen, msk, cx, cy, ref, 130, 121)
    np.testing.assert_array_equal(om, ref_m)
    scale = np.abs(ref_img).max()
    err = np.abs(out - ref_img).max() / scale
    print(f"{name} mode {mode}: max error {err:.2e}, masked {int(om.sum())}")
    assert err <= (1e-12 if mode == F64 else 1e-6)
    if name in ("identity", "shift") and mode == F64:
        np.testing.assert_array_equal(out, ref_img)


def test_no_mask_and_degenerate_maps():
    img, _ = _template(7, 64, 64)
    out, om = _run(img, None, [0.0, 1.0, 0.0], [0.0, 0.0, 1.0], (0.0, 0.0), 64, 64, F64)
    inner = np.s_[2:61, 2:61]
    np.testing.assert_array_equal(out[inner], img[inner])
    assert om[inner].sum() == 0 and om.sum() == 64 * 64 - 59 * 59
    for cx, cy in (([1e4, 1.0, 0.0], [0.0, 0.0, 1.0]), ([float("nan"), 1.0, 0.0], [0.0, 0.0, 1.0])):
        out, om = _run(img, None, cx, cy, (0.0, 0.0), 40, 40, F64)
        assert (om == 1).all() and (out == 0.0).all()


@pytest.mark.parametrize("mode", [F64, F32C])
def test_full_frame_windows(mode):
    n = 4088
    rng = np.random.default_rng(9)
    img = rng.normal(0, 10, (n, n))
    msk = (rng.random((n, n)) < 0.01).astype(np.uint8)
    cx, cy = _rot(0.0015, 1.0002, 2044.3, 2043.6)
    ref = (2044.0, 2044.0)
    out, om = _run(img, msk, cx, cy, ref, n, n, mode)
    seen = img if mode == F64 else img.astype(np.float32).astype(np.float64)
    for (y0, x0) in [(0, 0), (0, n - 128), (2000, 2000), (n - 128, 17), (n - 128, n - 128)]:
        # the oracle on the window: shift the reference point into window coordinates
        r_img, r_m = A.resample(seen, msk, cx, cy, (ref[0] - x0, ref[1] - y0), 128, 128)
        np.testing.assert_array_equal(om[y0:y0 + 128, x0:x0 + 128], r_m)
        err = np.abs(out[y0:y0 + 128, x0:x0 + 128] - r_img).max() / np.abs(seen).max()
        assert err <= (1e-12 if mode == F64 else 1e-6), (y0, x0, err)


@pytest.mark.parametrize("name", ["identity", "rotate", "deg3"])
def test_align_psf_matches_oracle(name):
    cx, cy, ref = MAPS[name]
    v, u = np.mgrid[-15:16, -15:16].astype(np.float64)
    p = np.exp(-(u ** 2 + 0.8 * v ** 2 + 0.3 * u * v) / 8.0)
    p /= p.sum()
    x0, y0 = 61.5, 57.25
    J = A.map_jacobian(cx, cy, ref, x0, y0)
    for s in (12, 15, 20):
        want = A.align_psf(p, s, J)
        got = torch.zeros((2 * s + 1, 2 * s + 1), dtype=torch.float64, device="cuda")
        B.sfft_align_psf(B.make_map(cx, cy, ref), x0, y0, torch.from_numpy(p).cuda(), got)
        torch.cuda.synchronize()
        g = got.cpu().numpy()
        assert np.abs(g - want).max() <= 1e-13 * np.abs(want).max(), (name, s)
        assert abs(g.sum() - 1.0) < 1e-13
