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


# ---------------------------------------------------------------------------
# decorrelation kernel (pipeline step 7)
# ---------------------------------------------------------------------------

def _gauss(sig, s):
    u = np.arange(-s, s + 1, dtype=np.float64)
    g = np.exp(-0.5 * (u[:, None] ** 2 + u[None, :] ** 2) / sig ** 2)
    return g / g.sum()


def test_decorrelation_identity():
    """Delta PSFs and a delta kernel leave white noise white: Psi is a delta."""
    d = np.zeros((3, 3))
    d[1, 1] = 1.0
    kc = np.zeros(9)
    kc[4] = 1.0
    psi = oracle.decorrelation_kernel(kc, 1, 0, 100, 100, d, d, 3.0, 5.0, 4)
    ref = np.zeros((9, 9))
    ref[4, 4] = 1.0
    assert np.abs(psi - ref).max() < 1e-14


def test_decorrelation_spectrum_gaussian_closed_form():
    """Gaussian PSFs and kernel: N(f) in closed form from the Gaussians' transforms."""
    sr, ss, sk, alpha = 1.4, 1.6, 1.2, 1.3
    pr, ps, kc = _gauss(sr, 12), _gauss(ss, 12), alpha * _gauss(sk, 9)
    sig_s, sig_r = 7.0, 4.0
    spec = oracle.decorrelation_spectrum(kc, ps, pr, sig_s, sig_r)
    nd = oracle.DECORR_GRID
    f = np.fft.fftfreq(nd)
    f2 = f[:, None] ** 2 + f[None, :] ** 2
    g = lambda s2: np.exp(-2.0 * np.pi ** 2 * s2 * f2)  # noqa: E731  (FT of a unit Gaussian, squared width s2)
    noise = sig_s ** 2 * g(sr ** 2) ** 2 + sig_r ** 2 * alpha ** 2 * g(sk ** 2) ** 2 * g(ss ** 2) ** 2
    ref = np.sqrt((sig_s ** 2 + sig_r ** 2) / noise)
    low = f2 <= 0.1 ** 2
    assert np.abs(spec[low] / ref[low] - 1.0).max() < 1e-4


def test_centre_kernel_is_the_local_kernel_at_the_centre():
    """For an odd frame the centre pixel has xh = yh = 0: applying the spatially
    varying kernel there equals convolving with K_c at that pixel."""
    rng = np.random.default_rng(8)
    ny = nx = 41
    w, dk = 3, 2
    img = rng.normal(size=(ny, nx))
    kc = rng.normal(size=oracle.num_basis(dk) * (2 * w + 1) ** 2)
    full = oracle.apply_kernel(img, kc, w, dk)
    loc = oracle.convolve(img, oracle.centre_kernel(kc, w, dk, ny, nx))
    assert abs(full[20, 20] - loc[20, 20]) < 1e-12 * np.abs(full).max()


def test_decorrelation_whitens_the_difference_noise():
    """Monte Carlo: D = P_R * n_s - K_c * P_S * n_r is strongly correlated between
    neighbouring pixels; Psi * D is white with variance sigma_s^2 + sigma_r^2."""
    rng = np.random.default_rng(9)
    n, sig_s, sig_r = 320, 6.0, 3.0
    pr, ps = synth.psf_stamp(2.0, 3.0, half=10), synth.psf_stamp(2.4, 3.0, half=10)
    kc = 0.9 * _gauss(1.0, 6)
    ns, nr = rng.normal(0.0, sig_s, (n, n)), rng.normal(0.0, sig_r, (n, n))
    d = oracle.convolve(ns, pr) - oracle.convolve(oracle.convolve(nr, ps), kc)
    psi = oracle.decorrelation_kernel(kc.ravel(), 6, 0, n, n, ps, pr, sig_s, sig_r, 31)
    e = oracle.convolve(d, psi)
    inner = slice(60, n - 60)

    def corr(x, dy, dx):
        a = x[inner, inner]
        b = np.roll(np.roll(x, -dy, 0), -dx, 1)[inner, inner]
        return float((a * b).mean() / (a * a).mean())

    assert corr(d, 0, 1) > 0.5 and corr(d, 1, 0) > 0.5
    for lag in ((0, 1), (1, 0), (1, 1), (0, 2)):
        assert abs(corr(e, *lag)) < 0.03, lag
    var = float(e[inner, inner].var())
    assert abs(var / (sig_s ** 2 + sig_r ** 2) - 1.0) < 0.05
