"""Plain CPU FP64 oracle of SFFT image subtraction.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.

What is computed (pipeline step 6 of the paper's "Pipeline steps" list: SFFT
subtraction of a science/template pair producing a difference image; the
method fits a delta-basis matching kernel that can follow a spatially varying
PSF, "Statement of need", by solving a large linear system, "Future
development").  The paper does not print the equations; the readings below
are the contract this project fixes, each one listed with its reason in the
design notes:

  Frame F = {0..ny-1} x {0..nx-1}, pixel (y, x), arrays row-major [y][x].
  G    = 1 - [mask != 0]                          good pixels (science side, background)
  G_R  = G * [w <= y < ny-w] * [w <= x < nx-w]    template side: w-wide border strip excluded
  xh   = 2x/(nx-1) - 1,  yh = 2y/(ny-1) - 1       frame-centred coordinates in [-1, 1]
  m_j  = xh^p yh^q, graded by d = p+q, then q ascending: 1; xh, yh; xh^2, xh yh, yh^2; ...
  A_a  = m_a * G_R * R      (a < nK = (DK+1)(DK+2)/2)  polynomial-weighted masked template
  S_m  = G * S
  (T_u X)(y, x) = X(y - u_y, x - u_x) inside F, else 0;  u in {-w..w}^2
  columns of the design matrix Phi: T_u A_a (kernel), G * m_b (background, b < nB)
  theta index: kernel (a, u) -> a*L^2 + (u_y+w)*L + (u_x+w), L = 2w+1;
               background b  -> nK*L^2 + b
  theta* = argmin || S_m - Phi theta ||^2 = Omega^{-1} beta,
           Omega = Phi^T Phi,  beta = Phi^T S_m            (Cholesky, FP64)
  D = S - sum_{a,u} k_{a,u} T_u(m_a * R) - sum_b c_b m_b    (unmasked R, whole frame)

Two routes to the same numbers:
  * direct  -- builds Phi explicitly (the definition itself); small frames.
  * fft     -- the normal-equation entries as zero-padded linear cross-
               correlations of the polynomial-weighted images (scipy.fft,
               FP64), windowed to the lags the entries need; any size.
Both solve with LAPACK Cholesky (scipy.linalg.cho_factor / cho_solve).
"""
from __future__ import annotations

import os

import numpy as np
import scipy.fft
import scipy.linalg

__all__ = [
    "num_basis", "num_coeffs", "monomial_exponents", "frame_coords", "monomials",
    "good_masks", "design_matrix", "normal_system_direct", "normal_system_fft",
    "normal_system", "solve", "difference_direct", "difference_fft", "difference",
    "fit", "rel_err", "theta_index", "cond_number", "omega_entries", "beta_entries",
    "difference_at", "fit_background", "residual_ratio",
]

_WORKERS = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()


# ---------------------------------------------------------------------------
# basis bookkeeping
# ---------------------------------------------------------------------------

def num_basis(deg: int) -> int:
    """Number of monomials of total degree <= deg in two variables."""
    return (deg + 1) * (deg + 2) // 2


def num_coeffs(w: int, dk: int, db: int) -> int:
    """n = (2w+1)^2 * nK + nB."""
    return (2 * w + 1) ** 2 * num_basis(dk) + num_basis(db)


def monomial_exponents(deg: int):
    """[(p, q)] for m = xh^p yh^q, ordered by degree d = p + q, then q ascending."""
    return [(d - q, q) for d in range(deg + 1) for q in range(d + 1)]


def frame_coords(ny: int, nx: int):
    """Frame-centred coordinates xh[x], yh[y] in [-1, 1] (float64 1-D arrays)."""
    xh = 2.0 * np.arange(nx, dtype=np.float64) / (nx - 1) - 1.0
    yh = 2.0 * np.arange(ny, dtype=np.float64) / (ny - 1) - 1.0
    return xh, yh


def monomials(ny: int, nx: int, deg: int) -> np.ndarray:
    """Stack [num_basis(deg), ny, nx] of the monomial images m_j(y, x)."""
    xh, yh = frame_coords(ny, nx)
    out = np.empty((num_basis(deg), ny, nx), dtype=np.float64)
    for j, (p, q) in enumerate(monomial_exponents(deg)):
        out[j] = np.outer(yh ** q, xh ** p)
    return out


def theta_index(a: int, uy: int, ux: int, w: int) -> int:
    L = 2 * w + 1
    return a * L * L + (uy + w) * L + (ux + w)


def good_masks(mask, ny: int, nx: int, w: int):
    """(G, G_R): good-pixel indicator and its template-side version with the w-strip removed."""
    if mask is None:
        g = np.ones((ny, nx), dtype=np.float64)
    else:
        g = (np.asarray(mask) == 0).astype(np.float64)
    gr = np.zeros_like(g)
    gr[w:ny - w, w:nx - w] = g[w:ny - w, w:nx - w]
    return g, gr


def _check(sci, tmpl, w, dk, db):
    sci = np.asarray(sci, dtype=np.float64)
    tmpl = np.asarray(tmpl, dtype=np.float64)
    if sci.shape != tmpl.shape or sci.ndim != 2:
        raise ValueError("science and template must be 2-D arrays of one shape")
    ny, nx = sci.shape
    if w < 0 or dk < 0 or db < 0:
        raise ValueError("w, DK and DB must be non-negative")
    if ny < 4 * w + 2 or nx < 4 * w + 2:
        raise ValueError("frame must be at least 4w+2 pixels on each side")
    return sci, tmpl, ny, nx


def _shift(x: np.ndarray, uy: int, ux: int) -> np.ndarray:
    """(T_u X)(y, x) = X(y - uy, x - ux) inside the frame, zero elsewhere."""
    ny, nx = x.shape
    out = np.zeros_like(x)
    ys, yd = (slice(0, ny - uy), slice(uy, ny)) if uy >= 0 else (slice(-uy, ny), slice(0, ny + uy))
    xs, xd = (slice(0, nx - ux), slice(ux, nx)) if ux >= 0 else (slice(-ux, nx), slice(0, nx + ux))
    out[yd, xd] = x[ys, xs]
    return out


# ---------------------------------------------------------------------------
# route (i): the definition, with an explicit design matrix
# ---------------------------------------------------------------------------

def design_matrix(sci, tmpl, mask, w, dk, db):
    """Explicit Phi [ny*nx, n] and target S_m [ny*nx] (small frames only)."""
    sci, tmpl, ny, nx = _check(sci, tmpl, w, dk, db)
    g, gr = good_masks(mask, ny, nx, w)
    mk = monomials(ny, nx, dk)
    mb = monomials(ny, nx, db)
    L = 2 * w + 1
    nk, nb = mk.shape[0], mb.shape[0]
    n = L * L * nk + nb
    phi = np.empty((ny * nx, n), dtype=np.float64)
    for a in range(nk):
        aa = mk[a] * gr * tmpl
        for uy in range(-w, w + 1):
            for ux in range(-w, w + 1):
                phi[:, theta_index(a, uy, ux, w)] = _shift(aa, uy, ux).ravel()
    for b in range(nb):
        phi[:, nk * L * L + b] = (g * mb[b]).ravel()
    return phi, (g * sci).ravel()


def normal_system_direct(sci, tmpl, mask, w, dk, db):
    """Omega = Phi^T Phi, beta = Phi^T S_m from the explicit design matrix."""
    phi, sm = design_matrix(sci, tmpl, mask, w, dk, db)
    return phi.T @ phi, phi.T @ sm


# ---------------------------------------------------------------------------
# route (ii): entries as windows of zero-padded linear cross-correlations
# ---------------------------------------------------------------------------

def _window(spec_l, spec_r, lag, shape):
    """c(d) = sum_z l(z) * r(z + d) for |d_y|, |d_x| <= lag from the two rfft2 spectra.

    With zero padding to Q >= n + lag on each axis the circular correlation
    irfft2(conj(L) * R) equals the linear one on the requested lags.
    Returns [2lag+1, 2lag+1] indexed [d_y + lag, d_x + lag].
    """
    qy, qx = shape
    c = scipy.fft.irfft2(np.conj(spec_l) * spec_r, s=(qy, qx), workers=_WORKERS)
    idx_y = np.arange(-lag, lag + 1) % qy
    idx_x = np.arange(-lag, lag + 1) % qx
    return c[np.ix_(idx_y, idx_x)]


def normal_system_fft(sci, tmpl, mask, w, dk, db):
    """Omega and beta from the correlation identities (exact given the w-strip).

    Omega[(a,u),(b,v)] = C_ab(u - v),   C_ab(d) = sum_z A_a(z) A_b(z + d),  |d| <= 2w
    Omega[(a,u), b']   = sum_z A_a(z) (G m_b')(z + u)
    beta[(a,u)]        = sum_z A_a(z) S_m(z + u)
    Omega[b, b']       = sum_z G m_b m_b',   beta[b] = sum_z G m_b S
    """
    sci, tmpl, ny, nx = _check(sci, tmpl, w, dk, db)
    g, gr = good_masks(mask, ny, nx, w)
    mk = monomials(ny, nx, dk)
    mb = monomials(ny, nx, db)
    L = 2 * w + 1
    nk, nb = mk.shape[0], mb.shape[0]
    nkk = L * L * nk
    n = nkk + nb
    qy = scipy.fft.next_fast_len(ny + 2 * w + 1, real=True)
    qx = scipy.fft.next_fast_len(nx + 2 * w + 1, real=True)
    A = [mk[a] * gr * tmpl for a in range(nk)]
    GB = [g * mb[b] for b in range(nb)]
    sm = g * sci
    rf = lambda x: scipy.fft.rfft2(x, s=(qy, qx), workers=_WORKERS)  # noqa: E731
    FA = [rf(x) for x in A]
    FG = [rf(x) for x in GB]
    FS = rf(sm)
    omega = np.zeros((n, n), dtype=np.float64)
    beta = np.zeros(n, dtype=np.float64)
    uy_arr = np.repeat(np.arange(-w, w + 1), L)   # u index order: u_y major, then u_x
    ux_arr = np.tile(np.arange(-w, w + 1), L)
    dyy = uy_arr[:, None] - uy_arr[None, :]       # rows (a, u), columns (b, v): lag u - v
    dxx = ux_arr[:, None] - ux_arr[None, :]
    for a in range(nk):
        ra = slice(a * L * L, (a + 1) * L * L)
        for b in range(nk):
            cab = _window(FA[a], FA[b], 2 * w, (qy, qx))
            omega[ra, b * L * L:(b + 1) * L * L] = cab[dyy + 2 * w, dxx + 2 * w]
        for b in range(nb):
            col = _window(FA[a], FG[b], w, (qy, qx))[uy_arr + w, ux_arr + w]
            omega[ra, nkk + b] = col
            omega[nkk + b, ra] = col
        beta[ra] = _window(FA[a], FS, w, (qy, qx))[uy_arr + w, ux_arr + w]
    for b in range(nb):
        for c in range(nb):
            omega[nkk + b, nkk + c] = np.sum(GB[b] * mb[c])
        beta[nkk + b] = np.sum(GB[b] * sci)
    return omega, beta


def normal_system(sci, tmpl, mask, w, dk, db, mode="auto"):
    if mode == "auto":
        ny, nx = np.shape(sci)
        mode = "direct" if ny * nx * num_coeffs(w, dk, db) <= 4_000_000 else "fft"
    if mode == "direct":
        return normal_system_direct(sci, tmpl, mask, w, dk, db)
    if mode == "fft":
        return normal_system_fft(sci, tmpl, mask, w, dk, db)
    raise ValueError(mode)


# ---------------------------------------------------------------------------
# solve and difference image
# ---------------------------------------------------------------------------

def solve(omega, beta):
    """theta = Omega^{-1} beta by LAPACK Cholesky (FP64).  Raises LinAlgError if not SPD."""
    cf = scipy.linalg.cho_factor(omega, lower=True, check_finite=True)
    return scipy.linalg.cho_solve(cf, beta)


def cond_number(omega):
    """2-norm condition number of the symmetric matrix Omega (from eigvalsh)."""
    ev = np.linalg.eigvalsh(omega)
    return float(ev[-1] / ev[0]) if ev[0] > 0 else float("inf")


def _split_theta(theta, w, dk, db):
    L = 2 * w + 1
    nk = num_basis(dk)
    k = np.asarray(theta[:nk * L * L], dtype=np.float64).reshape(nk, L, L)  # [a, uy+w, ux+w]
    c = np.asarray(theta[nk * L * L:], dtype=np.float64)
    return k, c


def difference_direct(sci, tmpl, theta, w, dk, db):
    """D = S - sum_{a,u} k_{a,u} T_u(m_a R) - sum_b c_b m_b, by explicit shifted sums."""
    sci, tmpl, ny, nx = _check(sci, tmpl, w, dk, db)
    k, c = _split_theta(theta, w, dk, db)
    mk = monomials(ny, nx, dk)
    mb = monomials(ny, nx, db)
    model = np.zeros((ny, nx), dtype=np.float64)
    for a in range(mk.shape[0]):
        wr = mk[a] * tmpl
        for uy in range(-w, w + 1):
            for ux in range(-w, w + 1):
                model += k[a, uy + w, ux + w] * _shift(wr, uy, ux)
    for b in range(mb.shape[0]):
        model += c[b] * mb[b]
    return sci - model


def difference_fft(sci, tmpl, theta, w, dk, db):
    """Same D with each kernel applied as a zero-padded linear convolution (scipy.fft, FP64)."""
    sci, tmpl, ny, nx = _check(sci, tmpl, w, dk, db)
    k, c = _split_theta(theta, w, dk, db)
    mk = monomials(ny, nx, dk)
    mb = monomials(ny, nx, db)
    qy = scipy.fft.next_fast_len(ny + w + 1, real=True)
    qx = scipy.fft.next_fast_len(nx + w + 1, real=True)
    acc = np.zeros((qy, qx // 2 + 1), dtype=np.complex128)
    for a in range(mk.shape[0]):
        kp = np.zeros((qy, qx), dtype=np.float64)
        for uy in range(-w, w + 1):
            for ux in range(-w, w + 1):
                kp[uy % qy, ux % qx] = k[a, uy + w, ux + w]
        acc += (scipy.fft.rfft2(mk[a] * tmpl, s=(qy, qx), workers=_WORKERS)
                * scipy.fft.rfft2(kp, workers=_WORKERS))
    conv = scipy.fft.irfft2(acc, s=(qy, qx), workers=_WORKERS)[:ny, :nx]
    model = conv + np.tensordot(c, mb, axes=(0, 0))
    return sci - model


def difference(sci, tmpl, theta, w, dk, db, mode="auto"):
    if mode == "auto":
        ny, nx = np.shape(sci)
        mode = "direct" if ny * nx * num_coeffs(w, dk, db) <= 50_000_000 else "fft"
    if mode == "direct":
        return difference_direct(sci, tmpl, theta, w, dk, db)
    if mode == "fft":
        return difference_fft(sci, tmpl, theta, w, dk, db)
    raise ValueError(mode)


def fit(sci, tmpl, mask, w, dk, db, mode="auto", with_cond=False):
    """Whole subtraction: normal system, Cholesky solve, difference image."""
    omega, beta = normal_system(sci, tmpl, mask, w, dk, db, mode=mode)
    theta = solve(omega, beta)
    dmode = mode if mode in ("direct", "fft") else "auto"
    d = difference(sci, tmpl, theta, w, dk, db, mode=dmode)
    out = dict(omega=omega, beta=beta, theta=theta, diff=d)
    if with_cond:
        out["cond"] = cond_number(omega)
    return out


def rel_err(x, ref):
    """||x - ref||_2 / ||ref||_2 over the whole array."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.linalg.norm(ref.ravel())
    return float(np.linalg.norm((x - ref).ravel()) / (den if den > 0 else 1.0))


# ---------------------------------------------------------------------------
# single entries and single pixels, straight from the definition (for
# sampled checks at sizes where the full system is too large to rebuild)
# ---------------------------------------------------------------------------

def _column(sci, tmpl, mask, w, dk, db, idx):
    """Column idx of Phi as an image (T_u A_a, or G m_b), and S_m."""
    sci, tmpl, ny, nx = _check(sci, tmpl, w, dk, db)
    g, gr = good_masks(mask, ny, nx, w)
    L = 2 * w + 1
    nk = num_basis(dk)
    xh, yh = frame_coords(ny, nx)
    if idx < nk * L * L:
        a, u = divmod(idx, L * L)
        uy, ux = divmod(u, L)
        p, q = monomial_exponents(dk)[a]
        aa = np.outer(yh ** q, xh ** p) * gr * tmpl
        return _shift(aa, uy - w, ux - w)
    p, q = monomial_exponents(db)[idx - nk * L * L]
    return g * np.outer(yh ** q, xh ** p)


def omega_entries(sci, tmpl, mask, w, dk, db, pairs):
    """[Omega[r, c] for (r, c) in pairs] as full-frame dot products of two Phi columns."""
    cache = {}

    def col(i):
        if i not in cache:
            cache[i] = _column(sci, tmpl, mask, w, dk, db, i)
        return cache[i]
    return np.array([float(np.sum(col(r) * col(c))) for r, c in pairs])


def beta_entries(sci, tmpl, mask, w, dk, db, rows):
    """[beta[r] for r in rows] = column r of Phi dotted with S_m."""
    sci = np.asarray(sci, dtype=np.float64)
    g, _ = good_masks(mask, sci.shape[0], sci.shape[1], w)
    sm = g * sci
    return np.array([float(np.sum(_column(sci, tmpl, mask, w, dk, db, r) * sm)) for r in rows])


def difference_at(sci, tmpl, theta, w, dk, db, ys, xs):
    """D at the pixels (ys[i], xs[i]) by the explicit sum over kernel taps and background terms.

    Per pixel z: D(z) = S(z) - sum_{a,u} k_{a,u} m_a(z - u) R(z - u) - sum_b c_b m_b(z), the sum
    running over the taps whose source pixel z - u lies in the frame (the sum over taps of one
    pixel is done with numpy on the L x L source window, flipped so that tap u meets z - u).
    """
    sci = np.asarray(sci, dtype=np.float64)
    tmpl = np.asarray(tmpl, dtype=np.float64)
    ny, nx = sci.shape
    k, c = _split_theta(theta, w, dk, db)
    xh, yh = frame_coords(ny, nx)
    kexp = monomial_exponents(dk)
    bexp = monomial_exponents(db)
    out = []
    for y, x in zip(ys, xs):
        y, x = int(y), int(x)
        # taps u with 0 <= y - u_y < ny and 0 <= x - u_x < nx
        uy_lo, uy_hi = max(-w, y - ny + 1), min(w, y)
        ux_lo, ux_hi = max(-w, x - nx + 1), min(w, x)
        acc = 0.0
        if uy_lo <= uy_hi and ux_lo <= ux_hi:
            sy = y - np.arange(uy_lo, uy_hi + 1)          # source rows, one per tap u_y
            sx = x - np.arange(ux_lo, ux_hi + 1)
            rwin = tmpl[np.ix_(sy, sx)]
            for a, (p, q) in enumerate(kexp):
                wgt = np.outer(yh[sy] ** q, xh[sx] ** p)
                ka = k[a, uy_lo + w:uy_hi + w + 1, ux_lo + w:ux_hi + w + 1]
                acc += float(np.sum(ka * wgt * rwin))
        for b, (p, q) in enumerate(bexp):
            acc += c[b] * xh[x] ** p * yh[y] ** q
        out.append(sci[y, x] - acc)
    return np.array(out)


def fit_background(omega, beta, theta, nkk):
    """Least-squares background for the fixed kernel theta[:nkk]: the normal
    equations restricted to the background columns, Omega_BB c = beta_B -
    Omega_BK k (the quantity a predicted kernel is completed with before
    its residual is judged).  Returns theta with its background replaced."""
    omega = np.asarray(omega, dtype=np.float64)
    beta = np.asarray(beta, dtype=np.float64)
    k = np.asarray(theta, dtype=np.float64)[:nkk]
    rhs = beta[nkk:] - omega[nkk:, :nkk] @ k
    c = scipy.linalg.solve(omega[nkk:, nkk:], rhs, assume_a="pos")
    return np.concatenate([k, c])


def residual_ratio(omega, beta, theta):
    """rho = ||beta - Omega theta|| / ||beta||: how far theta is from solving the normal equations."""
    r = np.asarray(beta, dtype=np.float64) - np.asarray(omega, dtype=np.float64) @ np.asarray(theta, dtype=np.float64)
    return float(np.linalg.norm(r) / np.linalg.norm(beta))
