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

from .sfft_oracle import _shift, monomial_exponents, monomials, num_basis

__all__ = ["convolve", "apply_kernel", "centre_kernel", "decorrelation_spectrum", "decorrelation_kernel",
           "DECORR_GRID"]


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


# ---------------------------------------------------------------------------
# decorrelation kernel (pipeline step 7)
# ---------------------------------------------------------------------------
# Step 7 fits a decorrelation kernel to the difference image and applies it
# to the difference image, the science PSF and the cross-convolved science
# image.  The paper gives no formula; the reading fixed here:
#   * the inputs carry independent white noise of standard deviations
#     sigma_s (science) and sigma_r (template);
#   * after cross-convolution S' = P_R * S and R' = P_S * R (P_R the
#     template PSF, P_S the science PSF) and the subtraction
#     D = S' - K * R' - background, the noise of D has the power spectrum
#         N(f) = sigma_s^2 |P_R^(f)|^2 + sigma_r^2 |K_c^(f)|^2 |P_S^(f)|^2,
#     with K_c the matching kernel at the frame centre (xh = yh = 0):
#         K_c(u) = sum_a k_{a,u} (-u_x sx)^p_a (-u_y sy)^q_a,
#     sx = 2/(nx-1), sy = 2/(ny-1) (the source-pixel weights m_a(z - u) at z
#     with xh = yh = 0);
#   * the kernel Psi^(f) = sqrt((sigma_s^2 + sigma_r^2) / N(f)) makes that
#     noise white with variance sigma_s^2 + sigma_r^2;
#   * spectra are the DFTs on an nd x nd grid (nd = 64) of the stamps placed
#     with their centre tap at index (0, 0) (negative offsets wrap); Psi is
#     the real part of the inverse DFT of Psi^, cropped to its (2t+1)^2
#     central taps (offsets |u| <= t), stamp[u_y + t, u_x + t].

DECORR_GRID = 64


def centre_kernel(kcoef, w, dk, ny, nx):
    """K_c(u) as an L x L stamp, L = 2w + 1."""
    L = 2 * w + 1
    nk = num_basis(dk)
    k = np.asarray(kcoef, dtype=np.float64)[:nk * L * L].reshape(nk, L, L)
    sx, sy = 2.0 / (nx - 1), 2.0 / (ny - 1)
    u = np.arange(-w, w + 1, dtype=np.float64)
    out = np.zeros((L, L))
    for a, (p, q) in enumerate(monomial_exponents(dk)):
        out += k[a] * np.outer((-u * sy) ** q, (-u * sx) ** p)
    return out


def _on_grid(stamp, nd):
    L = stamp.shape[0]
    s = L // 2
    g = np.zeros((nd, nd))
    for uy in range(-s, s + 1):
        for ux in range(-s, s + 1):
            g[uy % nd, ux % nd] += stamp[uy + s, ux + s]
    return g


def decorrelation_spectrum(kc, psf_sci, psf_tmpl, sigma_sci, sigma_tmpl, nd=DECORR_GRID):
    """Psi^ on the nd x nd grid of frequencies (f_y, f_x) = (j_y, j_x) / nd."""
    pr = np.fft.fft2(_on_grid(np.asarray(psf_tmpl, np.float64), nd))
    ps = np.fft.fft2(_on_grid(np.asarray(psf_sci, np.float64), nd))
    kk = np.fft.fft2(_on_grid(np.asarray(kc, np.float64), nd))
    noise = sigma_sci ** 2 * np.abs(pr) ** 2 + sigma_tmpl ** 2 * np.abs(kk) ** 2 * np.abs(ps) ** 2
    return np.sqrt((sigma_sci ** 2 + sigma_tmpl ** 2) / noise)


def decorrelation_kernel(kcoef, w, dk, ny, nx, psf_sci, psf_tmpl, sigma_sci, sigma_tmpl, t, nd=DECORR_GRID):
    """Psi cropped to (2t+1) x (2t+1) taps."""
    spec = decorrelation_spectrum(centre_kernel(kcoef, w, dk, ny, nx), psf_sci, psf_tmpl, sigma_sci,
                                  sigma_tmpl, nd)
    psi = np.real(np.fft.ifft2(spec))
    out = np.empty((2 * t + 1, 2 * t + 1))
    for uy in range(-t, t + 1):
        for ux in range(-t, t + 1):
            out[uy + t, ux + t] = psi[uy % nd, ux % nd]
    return out
