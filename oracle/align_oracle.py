"""Plain CPU FP64 oracle of the alignment of the template to the science frame.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.

Pipeline step 4 ("Pipeline steps") aligns the reference image, its PSF and its
detection mask to the science image before cross-convolution; the paper names
image alignment and resampling as the part its authors worked hardest to
accelerate ("GPU acceleration and performance") but gives neither the
coordinate model nor the interpolation.  The reading fixed here:

  * geometry: a polynomial pixel map from science to template pixel
    coordinates (a first-order WCS is the affine case; degree up to 3 covers a
    SIP-style distortion):
        u = x - x_ref,  v = y - y_ref,
        x_t = sum_j cx_j u^p_j v^q_j,   y_t = sum_j cy_j u^p_j v^q_j,
    monomials graded by d = p + q, then q ascending: 1; u, v; u^2, u v, v^2;
    u^3, u^2 v, u v^2, v^3 (the subtraction's own monomial order);
  * interpolation: Lanczos-3, L(t) = sinc(t) sinc(t / 3) for |t| < 3, else 0,
    sinc(t) = sin(pi t) / (pi t); with i0 = floor(x_t), j0 = floor(y_t) the
    36 taps are i = i0-2..i0+3, j = j0-2..j0+3 and
        out(y, x) = sum_{j,i} L(y_t - j) L(x_t - i) R[j, i]
                    / ((sum_j L(y_t - j)) (sum_i L(x_t - i)))
    (normalised weights, so constants are kept exactly);
  * validity and mask: an output pixel is valid when all 36 taps lie in the
    template frame; it is masked (1) when it is not valid or when any of its 36
    tap pixels is masked in the template mask; an invalid pixel's value is 0;
  * PSF: the aligned PSF stamp (side 2s+1) samples the template PSF stamp
    (side 2s_t+1, centre tap at index s_t, zero outside the stamp) at the
    template offsets J (u, v), J the Jacobian of the map at a science-frame
    point (x0, y0), with the same Lanczos-3 interpolation, and is scaled to
    the template stamp's sum.
"""
from __future__ import annotations

import numpy as np

__all__ = ["map_monomials", "apply_map", "map_jacobian", "lanczos3", "resample", "align_psf", "MAP_MAX_DEG"]

MAP_MAX_DEG = 3


def map_monomials(deg):
    """(p, q) exponents of the map's monomials in order."""
    return [(d - q, q) for d in range(deg + 1) for q in range(d + 1)]


def apply_map(cx, cy, ref, x, y):
    """Template coordinates (x_t, y_t) of science pixel coordinates (x, y)."""
    cx = np.asarray(cx, np.float64)
    cy = np.asarray(cy, np.float64)
    deg = {1: 0, 3: 1, 6: 2, 10: 3}[len(cx)]
    u = np.asarray(x, np.float64) - ref[0]
    v = np.asarray(y, np.float64) - ref[1]
    xt = np.zeros(np.broadcast(u, v).shape)
    yt = np.zeros_like(xt)
    for j, (p, q) in enumerate(map_monomials(deg)):
        m = u ** p * v ** q
        xt = xt + cx[j] * m
        yt = yt + cy[j] * m
    return xt, yt


def map_jacobian(cx, cy, ref, x0, y0):
    """[[dx_t/dx, dx_t/dy], [dy_t/dx, dy_t/dy]] at (x0, y0)."""
    deg = {1: 0, 3: 1, 6: 2, 10: 3}[len(cx)]
    u, v = x0 - ref[0], y0 - ref[1]
    J = np.zeros((2, 2))
    for j, (p, q) in enumerate(map_monomials(deg)):
        du = p * u ** (p - 1) * v ** q if p > 0 else 0.0
        dv = q * u ** p * v ** (q - 1) if q > 0 else 0.0
        J[0, 0] += cx[j] * du
        J[0, 1] += cx[j] * dv
        J[1, 0] += cy[j] * du
        J[1, 1] += cy[j] * dv
    return J


def lanczos3(t):
    """L(t) = sinc(t) sinc(t/3) on |t| < 3, else 0 (numpy's normalised sinc); exactly
    1 at 0 and 0 at the other integers, where sin(pi t) vanishes."""
    t = np.asarray(t, np.float64)
    v = np.where(np.abs(t) < 3.0, np.sinc(t) * np.sinc(t / 3.0), 0.0)
    return np.where(t == np.floor(t), (t == 0.0).astype(np.float64), v)


def resample(img, mask, cx, cy, ref, ny, nx):
    """(out, out_mask) on the ny x nx science grid from the template image and mask."""
    img = np.asarray(img, np.float64)
    nyt, nxt = img.shape
    tm = np.zeros(img.shape, bool) if mask is None else (np.asarray(mask) != 0)
    yy, xx = np.mgrid[0:ny, 0:nx].astype(np.float64)
    xt, yt = apply_map(cx, cy, ref, xx, yy)
    i0 = np.floor(xt).astype(np.int64)
    j0 = np.floor(yt).astype(np.int64)
    valid = (i0 - 2 >= 0) & (i0 + 3 <= nxt - 1) & (j0 - 2 >= 0) & (j0 + 3 <= nyt - 1)
    acc = np.zeros((ny, nx))
    wsx = np.zeros((ny, nx))
    wsy = np.zeros((ny, nx))
    masked = ~valid
    for k in range(-2, 4):
        wsx += lanczos3(xt - (i0 + k))
        wsy += lanczos3(yt - (j0 + k))
    for dj in range(-2, 4):
        jj = np.clip(j0 + dj, 0, nyt - 1)
        wy = lanczos3(yt - (j0 + dj))
        for di in range(-2, 4):
            ii = np.clip(i0 + di, 0, nxt - 1)
            wx = lanczos3(xt - (i0 + di))
            acc += wy * wx * img[jj, ii]
            masked |= tm[jj, ii] & valid
    out = np.where(valid, acc / (wsx * wsy), 0.0)
    return out, masked.astype(np.uint8)


def align_psf(psf_t, s, J):
    """Aligned PSF stamp (2s+1 square) from the template stamp psf_t by the Jacobian J."""
    psf_t = np.asarray(psf_t, np.float64)
    st = psf_t.shape[0] // 2
    out = np.zeros((2 * s + 1, 2 * s + 1))
    for v in range(-s, s + 1):
        for u in range(-s, s + 1):
            xt = st + J[0, 0] * u + J[0, 1] * v
            yt = st + J[1, 0] * u + J[1, 1] * v
            i0, j0 = int(np.floor(xt)), int(np.floor(yt))
            num = 0.0
            wsx = sum(lanczos3(xt - (i0 + k)) for k in range(-2, 4))
            wsy = sum(lanczos3(yt - (j0 + k)) for k in range(-2, 4))
            for dj in range(-2, 4):
                for di in range(-2, 4):
                    j, i = j0 + dj, i0 + di
                    if 0 <= j < psf_t.shape[0] and 0 <= i < psf_t.shape[1]:
                        num += lanczos3(yt - j) * lanczos3(xt - i) * psf_t[j, i]
            out[v + s, u + s] = num / (wsx * wsy)
    tot = out.sum()
    return out * (psf_t.sum() / tot) if tot != 0.0 else out
