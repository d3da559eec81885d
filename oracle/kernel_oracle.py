"""Plain CPU FP64 oracle of the kernel applications around the subtraction.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.

Cross-convolution is pipeline step 5 of the paper's "Pipeline steps" list: the
template PSF is convolved with the science image and the science PSF with the
template, so that both images carry the same effective PSF before the
subtraction (step 6).  The paper gives no formula; the reading fixed here is
the plain one:

  * a PSF stamp P is an odd (2s+1) x (2s+1) array centred on its middle pixel;
  * the convolution is linear, zero outside the frame, and returns an image of
    the frame's size (the same boundary as the subtraction's kernel):
        (P * X)(y, x) = sum_{|u_y|, |u_x| <= s} P[u_y + s, u_x + s] X(y - u_y, x - u_x).

A spatially varying kernel in the subtraction's coefficient layout (the
polynomial acts on the source pixels, before the shift) applies the same way:

        (K * X)(y, x) = sum_{a < nK} sum_u k_{a,u} (m_a X)(y - u_y, x - u_x),
        k_{a,u} = kcoef[a L^2 + (u_y + w) L + (u_x + w)],  L = 2w + 1,

which is the kernel part of the subtraction's model, so that
D = S - (K * R) - background.
"""
from __future__ import annotations

import numpy as np

from .sfft_oracle import _shift, monomials, num_basis

__all__ = ["convolve", "apply_kernel"]


def convolve(img, stamp):
    """P * X by explicit shifted sums over the stamp's taps (FP64)."""
    img = np.asarray(img, dtype=np.float64)
    stamp = np.asarray(stamp, dtype=np.float64)
    L = stamp.shape[0]
    if stamp.ndim != 2 or stamp.shape[1] != L or L % 2 != 1:
        raise ValueError("the stamp must be square with an odd side")
    s = L // 2
    out = np.zeros_like(img)
    for uy in range(-s, s + 1):
        for ux in range(-s, s + 1):
            k = stamp[uy + s, ux + s]
            if k != 0.0:
                out += k * _shift(img, uy, ux)
    return out


def apply_kernel(img, kcoef, w, dk):
    """K * X for a kernel of half-width w and spatial degree dk (FP64)."""
    img = np.asarray(img, dtype=np.float64)
    ny, nx = img.shape
    L = 2 * w + 1
    nk = num_basis(dk)
    k = np.asarray(kcoef, dtype=np.float64)[:nk * L * L].reshape(nk, L, L)
    m = monomials(ny, nx, dk)
    out = np.zeros_like(img)
    for a in range(nk):
        out += convolve(m[a] * img, k[a])
    return out
