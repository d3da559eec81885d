"""Plain CPU FP64 oracle of the output-masked fit (an SFFT variant).

TEST INFRASTRUCTURE ONLY: imported by the tests and the benchmark's
CPU-baseline leg, never by the product path.

The default fit (sfft_oracle) zero-fills the excluded pixels: the masked
science pixels enter the least squares as equations "0 = model", which is
what makes every normal-matrix entry a correlation.  The paper's pipeline
masks bad pixels before subtraction ("Pipeline steps") and leaves the
method's options to the method papers; this module takes the other common
reading of a mask, as weights on the output pixels:

  theta* = argmin  sum_{z in F, G(z) = 1} ( S(z) - sum_{a,u} k_{a,u} (T_u A_a)(z) - sum_b c_b m_b(z) )^2

with A_a = m_a * G_R * R exactly as in the default fit (the template side is
unchanged: excluded template pixels and the w-wide strip stay zero-filled).
The normal equations are Omega = Phi^T diag(G) Phi and beta =
Phi^T diag(G) S_m, Phi and S_m the default design matrix and target.

Two routes to the same numbers:
  * direct -- the definition: Phi built explicitly and its excluded rows
              dropped (small frames);
  * fft    -- the default (zero-filled) system minus the excluded rows:
              Omega = Omega_zf - Phi_M^T Phi_M, with Phi_M the rows of Phi at
              the excluded pixels.  Those rows vanish in the background
              columns (G m_b = 0 there) and in the target (S_m = G S = 0),
              so only the kernel block changes and beta is beta_zf.
Both solve with LAPACK Cholesky.  The difference image is the default one,
D = S - K (x) R - background, with the unmasked R.
"""
from __future__ import annotations

import numpy as np

from . import sfft_oracle as so

__all__ = ["normal_system_outmask_direct", "masked_rows", "normal_system_outmask_fft",
           "normal_system_outmask", "fit_outmask"]


def normal_system_outmask_direct(sci, tmpl, mask, w, dk, db):
    """Omega = Phi_G^T Phi_G, beta = Phi_G^T S_G over the good output pixels only."""
    phi, sm = so.design_matrix(sci, tmpl, mask, w, dk, db)
    ny, nx = np.shape(sci)
    g, _ = so.good_masks(mask, ny, nx, w)
    keep = g.ravel() > 0
    pg = phi[keep]
    return pg.T @ pg, pg.T @ sm[keep]


def masked_rows(tmpl, mask, w, dk):
    """Kernel part of the design-matrix rows at the excluded pixels, in row-major
    pixel order: [count, L^2 nK] with entry (a, u) = A_a(z - u), zero outside F."""
    tmpl = np.asarray(tmpl, dtype=np.float64)
    ny, nx = tmpl.shape
    g, gr = so.good_masks(mask, ny, nx, w)
    mk = so.monomials(ny, nx, dk)
    L = 2 * w + 1
    nk = mk.shape[0]
    ys, xs = np.nonzero(g == 0)
    rows = np.zeros((ys.size, L * L * nk), dtype=np.float64)
    for a in range(nk):
        aa = mk[a] * gr * tmpl
        for uy in range(-w, w + 1):
            for ux in range(-w, w + 1):
                yy, xx = ys - uy, xs - ux
                ok = (yy >= 0) & (yy < ny) & (xx >= 0) & (xx < nx)
                v = np.zeros(ys.size, dtype=np.float64)
                v[ok] = aa[yy[ok], xx[ok]]
                rows[:, so.theta_index(a, uy, ux, w)] = v
    return rows


def normal_system_outmask_fft(sci, tmpl, mask, w, dk, db):
    """The zero-filled system (FFT correlations) minus the excluded pixels' rows."""
    omega, beta = so.normal_system_fft(sci, tmpl, mask, w, dk, db)
    pm = masked_rows(tmpl, mask, w, dk)
    nkk = pm.shape[1]
    omega = omega.copy()
    omega[:nkk, :nkk] -= pm.T @ pm
    return omega, beta


def normal_system_outmask(sci, tmpl, mask, w, dk, db, mode="auto"):
    if mode == "auto":
        ny, nx = np.shape(sci)
        mode = "direct" if ny * nx * so.num_coeffs(w, dk, db) <= 4_000_000 else "fft"
    if mode == "direct":
        return normal_system_outmask_direct(sci, tmpl, mask, w, dk, db)
    if mode == "fft":
        return normal_system_outmask_fft(sci, tmpl, mask, w, dk, db)
    raise ValueError(mode)


def fit_outmask(sci, tmpl, mask, w, dk, db, mode="auto"):
    """Output-masked fit: normal system, Cholesky solve, difference image."""
    omega, beta = normal_system_outmask(sci, tmpl, mask, w, dk, db, mode=mode)
    theta = so.solve(omega, beta)
    dmode = mode if mode in ("direct", "fft") else "auto"
    d = so.difference(sci, tmpl, theta, w, dk, db, mode=dmode)
    return dict(omega=omega, beta=beta, theta=theta, diff=d)
