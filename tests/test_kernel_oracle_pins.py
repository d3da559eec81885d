"""Pins of the kernel-application oracle (cross-convolution, pipeline step 5)
against statements other than itself: brute-force loops, a library routine
(scipy.signal.convolve2d, 'same' output, zero fill), special cases (a delta
stamp, a shifted delta), flux conservation, and the subtraction's model."""
import numpy as np
import pytest
import scipy.signal

import oracle
import synth


def brute_convolve(img, stamp):
    ny, nx = img.shape
    s = stamp.shape[0] // 2
    out = np.zeros((ny, nx))
    for y in range(ny):
        for x in range(nx):
            acc = 0.0
            for uy in range(-s, s + 1):
                for ux in range(-s, s + 1):
                    sy, sx = y - uy, x - ux
                    if 0 <= sy < ny and 0 <= sx < nx:
                        acc += stamp[uy + s, ux + s] * img[sy, sx]
            out[y, x] = acc
    return out


def test_convolve_brute_force():
    rng = np.random.default_rng(1)
    img = rng.normal(size=(9, 11))
    stamp = rng.normal(size=(5, 5))
    assert np.abs(oracle.convolve(img, stamp) - brute_convolve(img, stamp)).max() < 1e-13


@pytest.mark.parametrize("shape,L", [((40, 33), 7), ((64, 64), 31), ((17, 50), 1)])
def test_convolve_is_scipy_same_mode(shape, L):
    rng = np.random.default_rng(L)
    img = rng.normal(size=shape)
    stamp = rng.normal(size=(L, L))
    ref = scipy.signal.convolve2d(img, stamp, mode="same", boundary="fill", fillvalue=0.0)
    assert np.abs(oracle.convolve(img, stamp) - ref).max() <= 1e-12 * np.abs(ref).max()


def test_delta_stamps():
    rng = np.random.default_rng(2)
    img = rng.normal(size=(20, 24))
    d = np.zeros((5, 5))
    d[2, 2] = 1.0
    assert np.array_equal(oracle.convolve(img, d), img)
    # a delta at u = (1, -2): content moves one row down and two columns left
    d = np.zeros((5, 5))
    d[2 + 1, 2 - 2] = 1.0
    out = oracle.convolve(img, d)
    assert np.array_equal(out[1:, :-2], img[:-1, 2:])
    assert not out[0].any() and not out[:, -2:].any()


def test_flux_conservation():
    """An image that vanishes within s of the edges keeps sum(img) * sum(stamp)."""
    p = synth.random_pair(3, 48, 52, 4, 0, 0, mask_frac=0.0, stars=True)
    img = np.zeros_like(p.tmpl)
    img[6:-6, 6:-6] = p.tmpl[6:-6, 6:-6]
    stamp = synth.psf_stamp(2.2, 3.0, half=5)
    out = oracle.convolve(img, stamp)
    assert abs(out.sum() - img.sum() * stamp.sum()) <= 1e-12 * abs(img).sum()


def test_apply_kernel_reduces_to_convolve_at_degree_zero():
    rng = np.random.default_rng(4)
    img = rng.normal(size=(30, 28))
    k = rng.normal(size=(7, 7))
    assert np.abs(oracle.apply_kernel(img, k.ravel(), 3, 0) - oracle.convolve(img, k)).max() < 1e-13


def test_apply_kernel_brute_force_degree_one():
    """Monomials written out by hand: m = 1, xh, yh on the source pixel."""
    rng = np.random.default_rng(5)
    ny, nx, w = 8, 10, 1
    img = rng.normal(size=(ny, nx))
    L = 2 * w + 1
    kc = rng.normal(size=3 * L * L)
    out = np.zeros((ny, nx))
    for y in range(ny):
        for x in range(nx):
            acc = 0.0
            for a in range(3):
                for uy in range(-w, w + 1):
                    for ux in range(-w, w + 1):
                        sy, sx = y - uy, x - ux
                        if 0 <= sy < ny and 0 <= sx < nx:
                            xh = 2.0 * sx / (nx - 1) - 1.0
                            yh = 2.0 * sy / (ny - 1) - 1.0
                            mono = (1.0, xh, yh)[a]
                            acc += kc[a * L * L + (uy + w) * L + (ux + w)] * mono * img[sy, sx]
            out[y, x] = acc
    assert np.abs(oracle.apply_kernel(img, kc, w, 1) - out).max() < 1e-13


def test_apply_kernel_is_the_subtraction_model():
    """D = S - (K * R) - background, with D from the subtraction's own oracle route."""
    p = synth.random_pair(6, 40, 36, 3, 2, 1, mask_frac=0.1, stars=True)
    n = oracle.num_coeffs(p.w, p.dk, p.db)
    theta = np.random.default_rng(7).normal(size=n)
    d = oracle.difference_direct(p.sci, p.tmpl, theta, p.w, p.dk, p.db)
    nkk = (2 * p.w + 1) ** 2 * oracle.num_basis(p.dk)
    bg = np.tensordot(theta[nkk:], oracle.monomials(*p.sci.shape, p.db), axes=(0, 0))
    model = oracle.apply_kernel(p.tmpl, theta[:nkk], p.w, p.dk)
    assert np.abs((p.sci - model - bg) - d).max() <= 1e-12 * np.abs(d).max()
