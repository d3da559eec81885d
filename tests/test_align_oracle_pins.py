"""Pins of the alignment oracle (oracle.align_oracle) against facts fixed by
the mathematics, not by its own code:

  * the Lanczos-3 kernel's closed-form values, zeros and symmetry;
  * the map's Jacobian against central finite differences, and the affine
    map written out by hand;
  * the identity map and integer translations copy the template exactly,
    with the frame border (taps outside the template) masked where the
    6 x 6 tap window says;
  * one masked template pixel masks exactly the 6 x 6 block of outputs
    whose taps contain it (identity map);
  * constants survive any map exactly (normalised weights);
  * a band-limited image under rotation, scale and shift matches the
    analytic function at the mapped coordinates within the bound that the
    kernel's own 1-D transfer function sets (and nearly reaches it);
  * the aligned PSF: identity returns the stamp, a rotation of a Gaussian
    matches the rotated Gaussian within the kernel's first-order sub-pixel
    bias, and a scale J = 0.5 doubles its width (second moment x 4)."""
import math

import numpy as np
import pytest

from oracle import align_oracle as A


def test_lanczos3_values():
    assert A.lanczos3(0.0) == 1.0
    for k in (1.0, 2.0, -1.0, -2.0):
        assert abs(A.lanczos3(k)) < 1e-15
    assert A.lanczos3(3.0) == 0.0 and A.lanczos3(-3.2) == 0.0
    assert abs(A.lanczos3(0.5) - 6.0 / math.pi ** 2) < 1e-15                  # 3 sin(pi/2) sin(pi/6) / (pi^2 / 4)
    assert abs(A.lanczos3(1.5) + 3.0 / (2.25 * math.pi ** 2)) < 1e-15         # sin(3pi/2) sin(pi/2) 3 / (2.25 pi^2)
    t = np.linspace(-2.9, 2.9, 57)
    assert np.array_equal(A.lanczos3(t), A.lanczos3(-t))


def test_map_and_jacobian():
    rng = np.random.default_rng(3)
    cx = rng.normal(0, 1, 10) * np.array([5, 1, 0.1, 1e-3, 1e-3, 1e-3, 1e-6, 1e-6, 1e-6, 1e-6])
    cy = rng.normal(0, 1, 10) * np.array([5, 0.1, 1, 1e-3, 1e-3, 1e-3, 1e-6, 1e-6, 1e-6, 1e-6])
    ref = (100.0, 80.0)
    x0, y0, h = 137.3, 41.9, 1e-4
    J = A.map_jacobian(cx, cy, ref, x0, y0)
    fx = [A.apply_map(cx, cy, ref, x0 + s * h, y0) for s in (1, -1)]
    fy = [A.apply_map(cx, cy, ref, x0, y0 + s * h) for s in (1, -1)]
    num = np.array([[(fx[0][0] - fx[1][0]) / (2 * h), (fy[0][0] - fy[1][0]) / (2 * h)],
                    [(fx[0][1] - fx[1][1]) / (2 * h), (fy[0][1] - fy[1][1]) / (2 * h)]])
    assert np.allclose(J, num, rtol=1e-7, atol=1e-9)
    # affine written out
    xt, yt = A.apply_map([1.5, 0.9, -0.2], [-3.0, 0.1, 1.1], (10.0, 20.0), 14.0, 27.0)
    assert abs(xt - (1.5 + 0.9 * 4.0 - 0.2 * 7.0)) < 1e-14 and abs(yt - (-3.0 + 0.1 * 4.0 + 1.1 * 7.0)) < 1e-14


def test_identity_and_integer_shift_copy():
    rng = np.random.default_rng(5)
    img = rng.normal(size=(40, 50))
    out, m = A.resample(img, None, [0.0, 1.0, 0.0], [0.0, 0.0, 1.0], (0.0, 0.0), 40, 50)
    inner = np.s_[2:40 - 3, 2:50 - 3]
    assert np.array_equal(out[inner], img[inner])
    want = np.ones((40, 50), np.uint8)
    want[inner] = 0
    assert np.array_equal(m, want)
    # x_t = x + 3, y_t = y - 2 (ref (0, 0)), onto a 30 x 30 grid
    out, m = A.resample(img, None, [3.0, 1.0, 0.0], [-2.0, 0.0, 1.0], (0.0, 0.0), 30, 30)
    for y in range(30):
        for x in range(30):
            xt, yt = x + 3, y - 2
            ok = 2 <= xt <= 50 - 4 and 2 <= yt <= 40 - 4
            assert m[y, x] == (0 if ok else 1)
            assert out[y, x] == (img[yt, xt] if ok else 0.0)


def test_one_masked_pixel_masks_a_6x6_block():
    img = np.zeros((30, 30))
    msk = np.zeros((30, 30), np.uint8)
    msk[14, 17] = 1
    _, m = A.resample(img, msk, [0.0, 1.0, 0.0], [0.0, 0.0, 1.0], (0.0, 0.0), 30, 30)
    border = np.ones((30, 30), bool)
    border[2:27, 2:27] = False
    block = np.zeros((30, 30), bool)
    block[14 - 3:14 + 3, 17 - 3:17 + 3] = True         # x - 2 <= 17 <= x + 3
    assert np.array_equal(m.astype(bool), border | block)


def _rot(theta, scale, tx, ty, ref):
    c, s = math.cos(theta), math.sin(theta)
    return [tx, scale * c, -scale * s], [ty, scale * s, scale * c], ref


def test_constant_kept_exactly():
    cx, cy, ref = _rot(0.3, 1.07, 40.0, 35.0, (32.0, 32.0))
    out, m = A.resample(np.full((80, 80), 2.5), None, cx, cy, ref, 64, 64)
    ok = m == 0
    assert ok.sum() > 3000 and np.abs(out[ok] - 2.5).max() < 1e-14


def _response_error(nu):
    """Worst |H(nu) - 1| over sub-pixel offsets of the normalised 6-tap Lanczos-3
    interpolator for the plane wave exp(2 pi i nu t) (its 1-D transfer function)."""
    k = np.arange(-2, 4)
    worst = 0.0
    for f in np.linspace(0.0, 1.0, 401)[:-1]:
        w = np.sinc(f - k) * np.sinc((f - k) / 3.0)
        worst = max(worst, abs((w * np.exp(2j * np.pi * nu * (k - f))).sum() / w.sum() - 1.0))
    return worst


def test_band_limited_image_under_rotation():
    # two plane waves; separable interpolation of a wave (a, b) errs by at most
    # |H(a) H(b) - 1| <= e(a) + e(b) + e(a) e(b) of its amplitude
    def f(x, y):
        return np.cos(2 * np.pi * (0.05 * x + 0.03 * y)) + 0.5 * np.sin(2 * np.pi * 0.04 * y + 0.3)
    yy, xx = np.mgrid[0:120, 0:120].astype(np.float64)
    img = f(xx, yy)
    cx, cy, ref = _rot(0.12, 0.97, 60.0, 58.0, (50.0, 50.0))
    out, m = A.resample(img, None, cx, cy, ref, 100, 100)
    gy, gx = np.mgrid[0:100, 0:100].astype(np.float64)
    xt, yt = A.apply_map(cx, cy, ref, gx, gy)
    ok = m == 0
    assert ok.sum() > 8000
    e05, e03, e04 = _response_error(0.05), _response_error(0.03), _response_error(0.04)
    bound = (e05 + e03 + e05 * e03) + 0.5 * e04
    err = np.abs(out[ok] - f(xt, yt)[ok]).max()
    assert err <= 1.02 * bound
    assert err >= 0.5 * bound          # the bound is nearly reached: the taps and weights are the kernel's


def _gauss_stamp(s, sig, J=None):
    """exp(-|r|^2 / 2 sig^2) on the (2s+1)^2 grid at r = J (u, v), and |dg/dx| + |dg/dy| there."""
    v, u = np.mgrid[-s:s + 1, -s:s + 1].astype(np.float64)
    if J is not None:
        x = J[0, 0] * u + J[0, 1] * v
        y = J[1, 0] * u + J[1, 1] * v
        u, v = x, y
    g = np.exp(-(u ** 2 + v ** 2) / (2 * sig ** 2))
    return g, (np.abs(u) + np.abs(v)) / sig ** 2 * g


def test_align_psf():
    p, _ = _gauss_stamp(12, 1.8)
    c = p.sum()
    p /= c
    out = A.align_psf(p, 12, np.eye(2))
    assert np.abs(out - p).max() < 1e-15
    # a rotation: the normalised 6-tap Lanczos-3 weights reproduce a linear
    # function up to a sub-pixel bias of at most delta per axis, so the sampled
    # rotated Gaussian differs by at most delta (|dg/dx| + |dg/dy|) (first order)
    k = np.arange(-2, 4)
    delta = 0.0
    for f in np.linspace(0.0, 1.0, 401)[:-1]:
        w = np.sinc(f - k) * np.sinc((f - k) / 3.0)
        delta = max(delta, abs((w * (k - f)).sum() / w.sum()))
    th = 0.4
    J = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    q = A.align_psf(p, 12, J)
    want, grad = _gauss_stamp(12, 1.8, J)
    want /= c
    grad /= c
    assert np.abs(q - want).max() <= delta * grad.max()
    assert abs(q.sum() - 1.0) < 1e-14
    # J = 0.5 I: a science offset of 2 px is 1 template px, the width doubles
    w = A.align_psf(p, 15, 0.5 * np.eye(2))
    v, u = np.mgrid[-15:16, -15:16].astype(np.float64)
    var = (w * u ** 2).sum() / w.sum()
    assert abs(var - 4 * 1.8 ** 2) < 0.02 * 4 * 1.8 ** 2
    assert abs(w.sum() - p.sum()) < 1e-14
