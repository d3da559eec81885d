"""Seeded synthetic star-field pairs shaped like Roman detector images.

This module only *renders data*: star catalogues with power-law fluxes,
point-spread functions (Gaussian or Moffat, evaluated at pixel centres and
normalised to unit sum) whose width varies across the frame, sky, noise and
masks.  It contains none of the subtraction method's arithmetic (no basis,
no normal equations, no solve, no kernel application), so both the CPU
oracle and the GPU path can take their inputs from it.

Every generator takes an explicit seed and uses numpy's PCG64
(``numpy.random.default_rng``), so the same seed gives the same images on
any machine with the same numpy.

The workloads stand in for the OpenUniverse 2024 Roman simulations that the
pipeline paper tests on (Summary / Statement of need); that data set is not
available here.  The shapes follow the paper: full 4088x4088 detector frames
and cutouts down to about 1000x1000 (GPU acceleration section), with a
spatially varying PSF (Statement of need).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

FWHM_PER_SIGMA = 2.0 * math.sqrt(2.0 * math.log(2.0))  # 2.3548...
STAMP_HALF = 20  # PSF stamps are 41 x 41 pixels


# ---------------------------------------------------------------------------
# small helpers
# ---------------------------------------------------------------------------

def _norm_coords(x, n):
    """Map pixel index 0..n-1 to [-1, 1] (the frame-centred coordinate)."""
    return 2.0 * np.asarray(x, dtype=np.float64) / (n - 1) - 1.0


def powerlaw_fluxes(rng, count, fmin, fmax, slope=-1.5):
    """Draw fluxes with p(F) ~ F**slope on [fmin, fmax] by inverse CDF."""
    u = rng.random(count)
    g = slope + 1.0
    if abs(g) < 1e-12:
        return fmin * (fmax / fmin) ** u
    a, b = fmin ** g, fmax ** g
    return (a + u * (b - a)) ** (1.0 / g)


def gaussian_stamp(dx, dy, sigma):
    """Unit-sum Gaussian sampled at integer offsets (dx, dy) from the star.

    ``dx``/``dy`` broadcast against the per-star ``sigma`` (shape [k,1,1]).
    """
    r2 = dx * dx + dy * dy
    img = np.exp(-0.5 * r2 / (sigma * sigma))
    return img / img.sum(axis=(-2, -1), keepdims=True)


def moffat_alpha(fwhm, beta):
    return fwhm / (2.0 * np.sqrt(2.0 ** (1.0 / beta) - 1.0))


def moffat_stamp(dx, dy, fwhm, beta):
    """Unit-sum Moffat profile (1 + r^2/alpha^2)^-beta at integer offsets."""
    alpha = moffat_alpha(fwhm, beta)
    r2 = dx * dx + dy * dy
    img = (1.0 + r2 / (alpha * alpha)) ** (-beta)
    return img / img.sum(axis=(-2, -1), keepdims=True)


def render_stars(ny, nx, xs, ys, fluxes, stamp_fn, chunk=4096, half=STAMP_HALF):
    """Add ``fluxes[i] * stamp_fn(...)`` centred at (xs[i], ys[i]) into an image.

    ``stamp_fn(dx, dy, idx)`` returns unit-sum stamps for the star indices
    ``idx``; dx, dy are the pixel-centre offsets from the (sub-pixel) star
    position.  Parts of a stamp that fall off the frame are dropped.
    """
    img = np.zeros(ny * nx, dtype=np.float64)
    off = np.arange(-half, half + 1)
    for s in range(0, len(xs), chunk):
        idx = np.arange(s, min(s + chunk, len(xs)))
        cx = np.floor(xs[idx] + 0.5).astype(np.int64)
        cy = np.floor(ys[idx] + 0.5).astype(np.int64)
        px = cx[:, None, None] + off[None, None, :]
        py = cy[:, None, None] + off[None, :, None]
        dx = px - xs[idx][:, None, None]
        dy = py - ys[idx][:, None, None]
        st = stamp_fn(dx, dy, idx) * fluxes[idx][:, None, None]
        px = np.broadcast_to(px, st.shape)
        py = np.broadcast_to(py, st.shape)
        ok = (px >= 0) & (px < nx) & (py >= 0) & (py < ny)
        img +=np.bincount((py[ok] * nx + px[ok]).ravel(), weights=st[ok].ravel(),
                           minlength=ny * nx)
    return img.reshape(ny, nx)


def disk_mask(ny, nx, xs, ys, radii):
    """Boolean mask of the union of disks (x - xs)^2 + (y - ys)^2 <= r^2."""
    m = np.zeros((ny, nx), dtype=bool)
    for x0, y0, r in zip(np.atleast_1d(xs), np.atleast_1d(ys), np.atleast_1d(radii)):
        r = float(r)
        x_lo, x_hi = max(int(math.floor(x0 - r)), 0), min(int(math.ceil(x0 + r)), nx - 1)
        y_lo, y_hi = max(int(math.floor(y0 - r)), 0), min(int(math.ceil(y0 + r)), ny - 1)
        if x_lo > x_hi or y_lo > y_hi:
            continue
        yy, xx = np.mgrid[y_lo:y_hi + 1, x_lo:x_hi + 1]
        m[y_lo:y_hi + 1, x_lo:x_hi + 1] |= (xx - x0) ** 2 + (yy - y0) ** 2 <= r * r
    return m


@dataclasses.dataclass
class Pair:
    """One science/template pair plus what the generator knows about it."""
    sci: np.ndarray          # float64 [ny, nx]
    tmpl: np.ndarray         # float64 [ny, nx]
    mask: np.ndarray         # uint8  [ny, nx], nonzero = excluded pixel
    w: int
    dk: int
    db: int
    truth: dict


# ---------------------------------------------------------------------------
# configurations
# ---------------------------------------------------------------------------

def pair_c1(seed=1001):
    """256x256 FP64 pair: ~400 Gaussian stars (FWHM 2.0), flat sky 100, Poisson.

    The science image is the template convolved with a Gaussian matching
    kernel (sigma ~0.7 px) whose amplitude and width vary linearly across the
    frame (DK=1 in the fit), plus a linear (DB=1) background plane and one
    injected point source of known flux.  Because a Gaussian convolved with a
    Gaussian is a Gaussian, the science stars are rendered directly with
    sigma_S^2 = sigma_T^2 + sigma_k(x, y)^2 and flux scaled by a(x, y); the
    sky is scaled by the same a(x, y).  The sky is left in (not subtracted),
    so the background terms have a pedestal to absorb.
    """
    rng = np.random.default_rng(seed)
    n = 256
    nstar = 400
    xs = rng.uniform(-5.0, n + 4.0, nstar)
    ys = rng.uniform(-5.0, n + 4.0, nstar)
    flux = powerlaw_fluxes(rng, nstar, 2e2, 2e5)
    sig_t = 2.0 / FWHM_PER_SIGMA
    xh, yh = _norm_coords(xs, n), _norm_coords(ys, n)
    amp = 1.0 + 0.04 * xh - 0.03 * yh
    sig_k = 0.7 * (1.0 + 0.10 * xh + 0.06 * yh)
    sig_s = np.sqrt(sig_t ** 2 + sig_k ** 2)
    sky = 100.0
    tmodel = render_stars(n, n, xs, ys, flux,
                          lambda dx, dy, i: gaussian_stamp(dx, dy, sig_t)) + sky
    gx = _norm_coords(np.arange(n), n)[None, :]
    gy = _norm_coords(np.arange(n), n)[:, None]
    amp_img = 1.0 + 0.04 * gx - 0.03 * gy
    bg = 3.0 + 2.0 * gx - 1.5 * gy
    smodel = render_stars(n, n, xs, ys, flux * amp,
                          lambda dx, dy, i: gaussian_stamp(dx, dy, sig_s[i][:, None, None]))
    tr_x, tr_y, tr_flux = 150.3, 97.6, 1.0e5
    tr_sig = math.sqrt(sig_t ** 2 + (0.7 * (1.0 + 0.10 * _norm_coords(tr_x, n)
                                              + 0.06 * _norm_coords(tr_y, n))) ** 2)
    transient = render_stars(n, n, np.array([tr_x]), np.array([tr_y]), np.array([tr_flux]),
                             lambda dx, dy, i: gaussian_stamp(dx, dy, tr_sig))
    smodel = smodel + sky * amp_img + bg + transient
    tmpl = rng.poisson(tmodel).astype(np.float64)
    sci = rng.poisson(smodel).astype(np.float64)
    mask = np.zeros((n, n), dtype=np.uint8)
    return Pair(sci, tmpl, mask, w=5, dk=1, db=1,
                truth=dict(transient_xy=(tr_x, tr_y), transient_flux=tr_flux,
                           transient_sigma=tr_sig, sky=sky, name="C1"))


def _roman_like(rng, ny, nx, nstar, fwhm_s, fwhm_t, beta=3.0, sky=1000.0, read_noise=8.0,
                fmin=5e2, fmax=5e6, bg_amp=0.0, transient=None, psf_var=0.05):
    """Sky-subtracted Moffat star-field pair with quadratic PSF-width variation.

    FWHM(x, y) = FWHM0 * (1 + psf_var * (xh^2 + yh^2)) for each image.
    Returns (sci, tmpl, star catalogue dict).
    """
    xs = rng.uniform(-5.0, nx + 4.0, nstar)
    ys = rng.uniform(-5.0, ny + 4.0, nstar)
    flux = powerlaw_fluxes(rng, nstar, fmin, fmax)
    vary = 1.0 + psf_var * (_norm_coords(xs, nx) ** 2 + _norm_coords(ys, ny) ** 2)
    fw_t = fwhm_t * vary
    fw_s = fwhm_s * vary
    tmodel = render_stars(ny, nx, xs, ys, flux,
                          lambda dx, dy, i: moffat_stamp(dx, dy, fw_t[i][:, None, None], beta))
    smodel = render_stars(ny, nx, xs, ys, flux,
                          lambda dx, dy, i: moffat_stamp(dx, dy, fw_s[i][:, None, None], beta))
    if bg_amp:
        gx = _norm_coords(np.arange(nx), nx)[None, :]
        gy = _norm_coords(np.arange(ny), ny)[:, None]
        smodel = smodel + bg_amp * (0.6 + 0.5 * gx - 0.4 * gy + 0.3 * gx * gx
                                    - 0.2 * gx * gy + 0.25 * gy * gy)
    if transient is not None:
        tx, ty, tf = transient
        tv = 1.0 + psf_var * (_norm_coords(tx, nx) ** 2 + _norm_coords(ty, ny) ** 2)
        smodel = smodel + render_stars(
            ny, nx, np.array([tx]), np.array([ty]), np.array([tf]),
            lambda dx, dy, i: moffat_stamp(dx, dy, fwhm_s * tv, beta))
    tmpl = rng.poisson(tmodel + sky).astype(np.float64) + rng.normal(0.0, read_noise, (ny, nx)) - sky
    sci = rng.poisson(smodel + sky).astype(np.float64) + rng.normal(0.0, read_noise, (ny, nx)) - sky
    cat = dict(xs=xs, ys=ys, flux=flux, fwhm_t=fw_t, fwhm_s=fw_s, beta=beta)
    return sci, tmpl, cat


def pair_c2(seed=1002):
    """1024x1024 pair, w=9, DK=DB=2; Moffat beta=3, FWHM 2.2 (sci) / 1.8 (tmpl).

    3000 stars; sky 1000 e- and read noise 8 e-, then sky-subtracted.  A 5%
    saturation mask: the pixels above the 95th percentile of max(S, R) are
    masked and both images are clipped to that level there.
    """
    rng = np.random.default_rng(seed)
    n = 1024
    sci, tmpl, cat = _roman_like(rng, n, n, 3000, 2.2, 1.8)
    mx = np.maximum(sci, tmpl)
    level = np.percentile(mx, 95.0)
    sat = mx > level
    sci = np.where(sat, np.minimum(sci, level), sci)
    tmpl = np.where(sat, np.minimum(tmpl, level), tmpl)
    return Pair(sci, tmpl, sat.astype(np.uint8), w=9, dk=2, db=2,
                truth=dict(name="C2", saturation_level=float(level), **{"nstar": 3000}))


def pair_c3(seed=1003, n=4088):
    """Roman-detector-sized pair: 4088x4088, w=9, DK=DB=2.

    About 40000 stars (2.39e-3 per pixel^2); PSFs as in the 1024 pair; sky
    1000 e- with Poisson noise, read noise 8 e-, sky-subtracted; a DB=2
    background of amplitude ~5 e- in the science image.  Masks: a disk of
    radius 3*FWHM around every star whose template peak exceeds 5e4 e-, and
    one of the same radius at the injected transient.
    """
    rng = np.random.default_rng(seed)
    nstar = int(round(2.39e-3 * n * n))
    tr = (0.61 * n + 0.3, 0.37 * n + 0.6, 2.0e5)
    sci, tmpl, cat = _roman_like(rng, n, n, nstar, 2.2, 1.8, bg_amp=5.0, transient=tr)
    # peak of a unit-flux Moffat at its centre pixel ~ 1/(pi alpha^2/(beta-1))
    alpha = moffat_alpha(cat["fwhm_t"], cat["beta"])
    peak = cat["flux"] * (cat["beta"] - 1.0) / (math.pi * alpha * alpha)
    bright = peak > 5e4
    m = disk_mask(n, n, cat["xs"][bright], cat["ys"][bright], 3.0 * cat["fwhm_s"][bright])
    m |= disk_mask(n, n, [tr[0]], [tr[1]], [3.0 * 2.2])
    return Pair(sci, tmpl, m.astype(np.uint8), w=9, dk=2, db=2,
                truth=dict(name="C3", transient_xy=tr[:2], transient_flux=tr[2],
                           nbright=int(bright.sum())))


def batch_c4_descriptors(npairs=128, seed0=4000):
    """Per-pair shapes of the batched workload (science s = i // 16, template t = i % 16).

    N uniform on {512, 1024, 2048}; w uniform on 5..9; DK uniform on {1, 2}; DB = DK.
    """
    out = []
    for i in range(npairs):
        rng = np.random.default_rng(seed0 + i)
        n = int(rng.choice([512, 1024, 2048]))
        w = int(rng.integers(5, 10))
        dk = int(rng.integers(1, 3))
        out.append(dict(index=i, s=i // 16, t=i % 16, n=n, w=w, dk=dk, db=dk, seed=seed0 + i))
    return out


def pair_c4(desc):
    """Render one pair of the batched workload from its descriptor."""
    rng = np.random.default_rng(desc["seed"] + 100000)
    n = desc["n"]
    nstar = int(round(2.39e-3 * n * n))
    sci, tmpl, cat = _roman_like(rng, n, n, nstar, 2.2, 1.8, bg_amp=5.0)
    alpha = moffat_alpha(cat["fwhm_t"], cat["beta"])
    peak = cat["flux"] * (cat["beta"] - 1.0) / (math.pi * alpha * alpha)
    bright = peak > 5e4
    m = disk_mask(n, n, cat["xs"][bright], cat["ys"][bright], 3.0 * cat["fwhm_s"][bright])
    return Pair(sci, tmpl, m.astype(np.uint8), w=desc["w"], dk=desc["dk"], db=desc["db"],
                truth=dict(name="C4", **desc))


def template_frame(seed, n, nstar=None):
    """The template of a template group and its mask (see template_group)."""
    rng = np.random.default_rng([seed, 0])
    if nstar is None:
        nstar = int(round(2.39e-3 * n * n))
    beta, sky, rn, psf_var, fwhm_t = 3.0, 1000.0, 8.0, 0.05, 1.8
    xs = rng.uniform(-5.0, n + 4.0, nstar)
    ys = rng.uniform(-5.0, n + 4.0, nstar)
    flux = powerlaw_fluxes(rng, nstar, 5e2, 5e6)
    vary = 1.0 + psf_var * (_norm_coords(xs, n) ** 2 + _norm_coords(ys, n) ** 2)
    fw_t = fwhm_t * vary
    tmodel = render_stars(n, n, xs, ys, flux, lambda dx, dy, i: moffat_stamp(dx, dy, fw_t[i][:, None, None], beta))
    tmpl = rng.poisson(tmodel + sky).astype(np.float64) + rng.normal(0.0, rn, (n, n)) - sky
    alpha = moffat_alpha(fw_t, beta)
    peak = flux * (beta - 1.0) / (math.pi * alpha * alpha)
    bright = peak > 5e4
    mask = disk_mask(n, n, xs[bright], ys[bright], np.full(int(bright.sum()), 3.0 * 2.6)).astype(np.uint8)
    cat = dict(xs=xs, ys=ys, flux=flux, vary=vary, beta=beta, sky=sky, read_noise=rn, psf_var=psf_var)
    return tmpl, mask, cat


def template_epoch(seed, n, cat, j, nsci):
    """Science epoch j of a template group (see template_group)."""
    rng = np.random.default_rng([seed, j + 1])
    beta, sky, rn, psf_var = cat["beta"], cat["sky"], cat["read_noise"], cat["psf_var"]
    xs, ys, flux = cat["xs"], cat["ys"], cat["flux"]
    fwhm_s = 2.0 + 0.6 * j / max(1, nsci - 1)
    fw_s = fwhm_s * cat["vary"]
    smodel = render_stars(n, n, xs, ys, flux, lambda dx, dy, i: moffat_stamp(dx, dy, fw_s[i][:, None, None], beta))
    gx = _norm_coords(np.arange(n), n)[None, :]
    gy = _norm_coords(np.arange(n), n)[:, None]
    c = rng.normal(0.0, 0.3, 5)
    smodel = smodel + 5.0 * (0.6 + c[0] + (0.5 + c[1]) * gx - (0.4 + c[2]) * gy + 0.3 * gx * gx
                             - (0.2 + c[3]) * gx * gy + (0.25 + c[4]) * gy * gy)
    tx, ty = rng.uniform(0.1 * n, 0.9 * n, 2)
    tv = 1.0 + psf_var * (_norm_coords(tx, n) ** 2 + _norm_coords(ty, n) ** 2)
    smodel = smodel + render_stars(n, n, np.array([tx]), np.array([ty]), np.array([2.0e5]),
                                   lambda dx, dy, i: moffat_stamp(dx, dy, fwhm_s * tv, beta))
    sci = rng.poisson(smodel + sky).astype(np.float64) + rng.normal(0.0, rn, (n, n)) - sky
    return sci, dict(epoch=j, fwhm_s=fwhm_s, transient_xy=(float(tx), float(ty)))


def template_group(seed, n, nsci, w=9, dk=2, db=2, nstar=None):
    """One template and ``nsci`` science epochs of the same field (the S x T pairing).

    The template is rendered once as in the 4088^2 recipe (Moffat beta=3,
    FWHM 1.8 at the centre varying by 5 % quadratically to the corners, sky
    1000 e- with Poisson noise, read noise 8 e-, sky-subtracted).  Science
    epoch j sees the same stars through its own PSF (FWHM_s,j = 2.0 +
    0.6 j / max(1, nsci - 1) at the centre, the same variation), its own
    noise, its own quadratic background of amplitude ~5 e- and a transient of
    2e5 e- at its own position.  The mask is the template's: a disk of radius
    3 * 2.6 around every star whose template peak exceeds 5e4 e-; it is the
    same array for every epoch.  The template depends on ``seed`` alone and
    epoch j on (``seed``, j), so one epoch can be rendered on its own
    (template_group_pair).  Returns a list of ``nsci`` Pairs whose ``tmpl``
    and ``mask`` are the same objects.
    """
    tmpl, mask, cat = template_frame(seed, n, nstar)
    out = []
    for j in range(nsci):
        sci, info = template_epoch(seed, n, cat, j, nsci)
        out.append(Pair(sci, tmpl, mask, w=w, dk=dk, db=db, truth=dict(name="template group", seed=seed, **info)))
    return out


def template_group_pair(seed, n, j, nsci, w=9, dk=2, db=2, nstar=None):
    """Epoch j of template_group(seed, n, nsci, ...) alone (the same arrays)."""
    tmpl, mask, cat = template_frame(seed, n, nstar)
    sci, info = template_epoch(seed, n, cat, j, nsci)
    return Pair(sci, tmpl, mask, w=w, dk=dk, db=db, truth=dict(name="template group", seed=seed, **info))


def random_pair(seed, ny, nx, w, dk, db, mask_frac=0.1, stars=True):
    """Small generic pair for tests: any shape, random mask of ~``mask_frac``.

    With ``stars`` the images are sparse Gaussian star fields plus unit
    Gaussian noise (a realistic, reasonably conditioned system); otherwise
    they are plain standard-normal noise.
    """
    rng = np.random.default_rng(seed)
    if stars:
        k = max(4, int(0.01 * ny * nx))
        xs = rng.uniform(0, nx - 1, k)
        ys = rng.uniform(0, ny - 1, k)
        fl = powerlaw_fluxes(rng, k, 50.0, 5e3)
        tmpl = render_stars(ny, nx, xs, ys, fl, lambda dx, dy, i: gaussian_stamp(dx, dy, 0.9))
        sci = render_stars(ny, nx, xs + 0.3, ys - 0.2, fl * 1.1,
                           lambda dx, dy, i: gaussian_stamp(dx, dy, 1.3))
        tmpl = tmpl + rng.normal(0.0, 1.0, (ny, nx))
        sci = sci + rng.normal(0.0, 1.0, (ny, nx)) + 2.0
    else:
        tmpl = rng.normal(0.0, 1.0, (ny, nx))
        sci = rng.normal(0.0, 1.0, (ny, nx))
    mask = (rng.random((ny, nx)) < mask_frac).astype(np.uint8)
    return Pair(sci, tmpl, mask, w=w, dk=dk, db=db, truth=dict(name="random", seed=seed))


CONFIGS = {
    "c1": pair_c1,
    "c2": pair_c2,
    "c3": pair_c3,
}


# ---------------------------------------------------------------------------
# frames at focal-plane positions (training data of the warm-start network)
# ---------------------------------------------------------------------------

WS_STAMP_HALF = 16      # the network sees 33 x 33 PSF stamps
WS_SPAN = 0.25          # half-width of one frame in focal-plane units ([-1, 1] across the array)
WS_CURV_S = 0.15        # science FWHM grows by 15 % from the focal-plane centre to a corner axis
WS_CURV_T = 0.05


def psf_stamp(fwhm, beta, half=WS_STAMP_HALF):
    """Unit-sum Moffat PSF on a (2 half + 1)^2 grid, centred on the middle pixel."""
    off = np.arange(-half, half + 1, dtype=np.float64)
    return moffat_stamp(off[None, :], off[:, None], fwhm, beta)


def pair_ws(seed, n=512, w=9, dk=2, db=2, beta=3.0):
    """One frame of the warm-start workload: a C3-like sky-subtracted Moffat field.

    The frame sits at a random focal-plane position (X, Y) in [-1, 1]^2 and
    covers +-WS_SPAN around it; the FWHM of each image varies quadratically
    over the focal plane, FWHM = FWHM0 (1 + curv (Xf^2 + Yf^2)), with
    per-frame FWHM0 (seeing) drawn for the science image from [1.9, 2.6] and
    for the template from [1.5, 1.8].  Star density, fluxes, sky, noise, the
    DB = 2 background and the bright-star masks follow the 4088^2 recipe.
    ``truth`` carries the network inputs: the two PSF stamps at the frame
    centre and (X, Y).
    """
    rng = np.random.default_rng(seed)
    X, Y = rng.uniform(-1.0, 1.0, 2)
    f_s0 = rng.uniform(1.9, 2.6)
    f_t0 = rng.uniform(1.5, 1.8)
    nstar = int(round(2.39e-3 * n * n))
    xs = rng.uniform(-5.0, n + 4.0, nstar)
    ys = rng.uniform(-5.0, n + 4.0, nstar)
    flux = powerlaw_fluxes(rng, nstar, 5e2, 5e6)
    Xf = X + WS_SPAN * _norm_coords(xs, n)
    Yf = Y + WS_SPAN * _norm_coords(ys, n)
    fw_s = f_s0 * (1.0 + WS_CURV_S * (Xf * Xf + Yf * Yf))
    fw_t = f_t0 * (1.0 + WS_CURV_T * (Xf * Xf + Yf * Yf))
    tmodel = render_stars(n, n, xs, ys, flux,
                          lambda dx, dy, i: moffat_stamp(dx, dy, fw_t[i][:, None, None], beta), half=12)
    smodel = render_stars(n, n, xs, ys, flux,
                          lambda dx, dy, i: moffat_stamp(dx, dy, fw_s[i][:, None, None], beta), half=12)
    gx = _norm_coords(np.arange(n), n)[None, :]
    gy = _norm_coords(np.arange(n), n)[:, None]
    bc = rng.normal(0.0, 1.0, 6)
    smodel = smodel + 5.0 * (bc[0] + bc[1] * gx + bc[2] * gy + 0.5 * (bc[3] * gx * gx + bc[4] * gx * gy
                                                                      + bc[5] * gy * gy))
    sky, read_noise = 1000.0, 8.0
    tmpl = rng.poisson(tmodel + sky).astype(np.float64) + rng.normal(0.0, read_noise, (n, n)) - sky
    sci = rng.poisson(smodel + sky).astype(np.float64) + rng.normal(0.0, read_noise, (n, n)) - sky
    alpha = moffat_alpha(fw_t, beta)
    peak = flux * (beta - 1.0) / (math.pi * alpha * alpha)
    bright = peak > 5e4
    m = disk_mask(n, n, xs[bright], ys[bright], 3.0 * fw_s[bright])
    c_s = f_s0 * (1.0 + WS_CURV_S * (X * X + Y * Y))
    c_t = f_t0 * (1.0 + WS_CURV_T * (X * X + Y * Y))
    return Pair(sci, tmpl, m.astype(np.uint8), w=w, dk=dk, db=db,
                truth=dict(name="WS", X=float(X), Y=float(Y), stamp_s=psf_stamp(c_s, beta),
                           stamp_t=psf_stamp(c_t, beta), fwhm_s0=float(f_s0), fwhm_t0=float(f_t0)))


# ---------------------------------------------------------------------------
# counter-based noise and the 4088^2 warm-start recipe (rendered on the GPU
# by the library's renderer; the numpy renderer below is its reference)
# ---------------------------------------------------------------------------
# Philox4x32-10 (Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as easy
# as 1, 2, 3", SC 2011): a 4 x 32-bit counter and a 2 x 32-bit key, ten rounds
# of two 32x32->64-bit multiplies with the published constants, the key bumped
# by the Weyl increments between rounds.

PHILOX_M0, PHILOX_M1 = 0xD2511F53, 0xCD9E8D57
PHILOX_W0, PHILOX_W1 = 0x9E3779B9, 0xBB67AE85


def philox4x32(c0, c1, c2, c3, k0, k1):
    """Philox4x32-10 of counter arrays (uint32) under key (k0, k1); returns four uint32 arrays."""
    M = np.uint64(0xFFFFFFFF)
    c0, c1, c2, c3 = (np.asarray(c, np.uint64) for c in (c0, c1, c2, c3))
    k0, k1 = np.uint64(k0), np.uint64(k1)
    for _ in range(10):
        p0 = np.uint64(PHILOX_M0) * c0
        p1 = np.uint64(PHILOX_M1) * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & M
        hi1, lo1 = p1 >> np.uint64(32), p1 & M
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0) & M, lo1, (hi0 ^ c3 ^ k1) & M, lo0
        k0 = (k0 + np.uint64(PHILOX_W0)) & M
        k1 = (k1 + np.uint64(PHILOX_W1)) & M
    return tuple(x.astype(np.uint32) for x in (c0, c1, c2, c3))


def philox_normals(index, stream, seed):
    """Two standard normals per element of `index` (uint64 pixel index) for noise stream
    `stream`: counter (index low, index high, stream, 0), key (seed low, seed high);
    uniforms u = (hi 21 bits << 32 | lo 32 bits + 0.5) / 2^53 from word pairs, Box-Muller."""
    index = np.asarray(index, np.uint64)
    seed = int(seed)
    w = philox4x32(index & np.uint64(0xFFFFFFFF), index >> np.uint64(32),
                   np.full(index.shape, stream, np.uint64), np.zeros(index.shape, np.uint64),
                   seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    def unif(hi, lo):
        v = ((hi.astype(np.uint64) >> np.uint64(11)) << np.uint64(32)) | lo.astype(np.uint64)
        return (v.astype(np.float64) + 0.5) / float(1 << 53)
    u1, u2 = unif(w[0], w[1]), unif(w[2], w[3])
    r = np.sqrt(-2.0 * np.log(u1))
    return r * np.cos(2.0 * np.pi * u2), r * np.sin(2.0 * np.pi * u2)


WS_BETA_RANGE = (2.5, 4.0)
WS_FWHM_S_RANGE = (1.9, 2.6)
WS_FWHM_T_RANGE = (1.6, 2.0)
WS_HALF = 12            # star stamps of the warm-start frames are 25 x 25


def ws_catalog(seed, n=4088, density=2.39e-3, fmin=5e2, fmax=5e6):
    """Everything random in one warm-start frame (host side, PCG64): focal-plane
    position, seeing, Moffat beta, stars, background coefficients and the noise seed.
    The frame covers +-WS_SPAN of the focal plane around (X, Y); the FWHM of each
    image varies quadratically over the focal plane as in pair_ws."""
    rng = np.random.default_rng(seed)
    X, Y = rng.uniform(-1.0, 1.0, 2)
    f_s0 = rng.uniform(*WS_FWHM_S_RANGE)
    f_t0 = rng.uniform(*WS_FWHM_T_RANGE)
    beta = rng.uniform(*WS_BETA_RANGE)
    nstar = int(round(density * n * n))
    xs = rng.uniform(-5.0, n + 4.0, nstar)
    ys = rng.uniform(-5.0, n + 4.0, nstar)
    flux = powerlaw_fluxes(rng, nstar, fmin, fmax)
    bc = rng.normal(0.0, 1.0, 6)
    noise_seed = int(rng.integers(0, 2 ** 63))
    Xf = X + WS_SPAN * _norm_coords(xs, n)
    Yf = Y + WS_SPAN * _norm_coords(ys, n)
    fw_s = f_s0 * (1.0 + WS_CURV_S * (Xf * Xf + Yf * Yf))
    fw_t = f_t0 * (1.0 + WS_CURV_T * (Xf * Xf + Yf * Yf))
    alpha_t = moffat_alpha(fw_t, beta)
    peak = flux * (beta - 1.0) / (math.pi * alpha_t * alpha_t)
    bright = peak > 5e4
    c_s = f_s0 * (1.0 + WS_CURV_S * (X * X + Y * Y))
    c_t = f_t0 * (1.0 + WS_CURV_T * (X * X + Y * Y))
    return dict(n=n, X=float(X), Y=float(Y), fwhm_s0=float(f_s0), fwhm_t0=float(f_t0), beta=float(beta),
                xs=xs, ys=ys, flux=flux, fw_s=fw_s, fw_t=fw_t, bc=bc, noise_seed=noise_seed,
                mask_r=np.where(bright, 3.0 * fw_s, 0.0),
                stamp_s=psf_stamp(c_s, beta), stamp_t=psf_stamp(c_t, beta))


WS_SKY, WS_READ = 1000.0, 8.0


def ws_background(cat):
    """The science image's quadratic background of a warm-start frame (e-)."""
    n = cat["n"]
    gx = _norm_coords(np.arange(n), n)[None, :]
    gy = _norm_coords(np.arange(n), n)[:, None]
    bc = cat["bc"]
    return 5.0 * (bc[0] + bc[1] * gx + bc[2] * gy + 0.5 * (bc[3] * gx * gx + bc[4] * gx * gy + bc[5] * gy * gy))


def render_ws_reference(cat):
    """Reference rendering of a catalogue (what the GPU renderer computes): Moffat
    stars normalised over their 25 x 25 stamps, the background, and noise
    lam + sqrt(lam) z1 + 8 z2 - sky with lam = model + sky (the normal limit of
    Poisson(lam) at lam >= 1000 e-) from philox_normals (stream 0: science,
    1: template); mask of the bright-star disks.  Returns (sci, tmpl, mask)."""
    n = cat["n"]
    beta = cat["beta"]
    fw_s, fw_t = cat["fw_s"], cat["fw_t"]
    tm = render_stars(n, n, cat["xs"], cat["ys"], cat["flux"],
                      lambda dx, dy, i: moffat_stamp(dx, dy, fw_t[i][:, None, None], beta), half=WS_HALF)
    sm = render_stars(n, n, cat["xs"], cat["ys"], cat["flux"],
                      lambda dx, dy, i: moffat_stamp(dx, dy, fw_s[i][:, None, None], beta), half=WS_HALF)
    sm = sm + ws_background(cat)
    idx = np.arange(n * n, dtype=np.uint64)
    out = []
    for stream, model in ((0, sm), (1, tm)):
        z1, z2 = philox_normals(idx, stream, cat["noise_seed"])
        lam = np.maximum(model.ravel(), 0.0) + WS_SKY
        out.append((lam + np.sqrt(lam) * z1 + WS_READ * z2 - WS_SKY).reshape(n, n))
    b = cat["mask_r"] > 0.0
    mask = disk_mask(n, n, cat["xs"][b], cat["ys"][b], cat["mask_r"][b])
    return out[0], out[1], mask.astype(np.uint8)
