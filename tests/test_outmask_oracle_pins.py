"""Pins of the output-masked fit's oracle (oracle/outmask_oracle.py).

The fit restricts the least squares to the good output pixels.  Pinned by:
  * brute force -- the pixel-loop design matrix of test_oracle_pins with the
    excluded rows dropped, solved by SVD least squares (never forms Omega);
  * the correction route (zero-filled system minus the excluded rows)
    against the definition route, entry by entry;
  * the excluded rows written by loops against masked_rows;
  * exact recovery of a known kernel when the excluded science pixels hold
    arbitrary values, which the zero-filled fit cannot do (the pin that tells
    the two readings apart);
  * no mask: the same system as the zero-filled fit;
  * insensitivity to the science values at excluded pixels.
"""
import numpy as np
import pytest

import oracle
import synth
from test_oracle_pins import brute_phi

CASES = [
    # (ny, nx, w, dk, db, mask_frac, seed)
    (14, 13, 1, 1, 1, 0.15, 2),
    (16, 16, 2, 2, 2, 0.10, 3),
    (19, 16, 2, 1, 2, 0.20, 4),
    (16, 20, 3, 0, 1, 0.05, 5),
    (13, 15, 0, 2, 0, 0.10, 6),
]


@pytest.mark.parametrize("ny,nx,w,dk,db,frac,seed", CASES)
@pytest.mark.parametrize("mode", ["direct", "fft"])
def test_bruteforce_lstsq_over_good_pixels(ny, nx, w, dk, db, frac, seed, mode):
    p = synth.random_pair(seed, ny, nx, w, dk, db, mask_frac=frac, stars=False)
    phi, tgt = brute_phi(p.sci, p.tmpl, p.mask, w, dk, db)
    keep = p.mask.ravel() == 0
    theta_ref, *_ = np.linalg.lstsq(phi[keep], tgt[keep], rcond=None)
    sv = np.linalg.svd(phi[keep], compute_uv=False)
    cond = sv[0] / sv[-1]
    om, be = oracle.normal_system_outmask(p.sci, p.tmpl, p.mask, w, dk, db, mode=mode)
    ref_om = phi[keep].T @ phi[keep]
    np.testing.assert_allclose(om, ref_om, rtol=0, atol=1e-11 * np.abs(ref_om).max())
    theta = oracle.solve(om, be)
    assert oracle.rel_err(theta, theta_ref) < 1e-13 * cond * cond + 1e-12
    # the fit is a different one from the zero-filled fit whenever an excluded
    # pixel sees template light
    om_zf, _ = oracle.normal_system(p.sci, p.tmpl, p.mask, w, dk, db, mode="direct")
    if frac > 0 and w > 0:
        assert np.abs(om_zf - om).max() > 1e-6 * np.abs(om).max()


@pytest.mark.parametrize("ny,nx,w,dk,db,frac,seed", CASES[:3])
def test_masked_rows_are_the_excluded_rows_of_phi(ny, nx, w, dk, db, frac, seed):
    p = synth.random_pair(seed, ny, nx, w, dk, db, mask_frac=frac, stars=False)
    phi, _ = brute_phi(p.sci, p.tmpl, p.mask, w, dk, db)
    L = 2 * w + 1
    nkk = L * L * oracle.num_basis(dk)
    rows = oracle.masked_rows(p.tmpl, p.mask, w, dk)
    excl = np.flatnonzero(p.mask.ravel() != 0)        # row-major pixel order
    np.testing.assert_array_equal(rows, phi[excl, :nkk])
    # ... whose background part and target vanish (G = 0 there)
    assert np.all(phi[excl, nkk:] == 0)


def test_exact_recovery_with_corrupted_excluded_pixels():
    """Noiseless S from a known theta everywhere, then arbitrary values on the
    excluded pixels: the output-masked fit returns theta exactly; the
    zero-filled fit, which fits 0 there, does not."""
    ny, nx, w, dk, db = 40, 36, 2, 1, 1
    rng = np.random.default_rng(77)
    p = synth.random_pair(78, ny, nx, w, dk, db, mask_frac=0.08, stars=True)
    L = 2 * w + 1
    n = oracle.num_coeffs(w, dk, db)
    theta_true = rng.normal(0.0, 0.1, n)
    theta_true[oracle.theta_index(0, 0, 0, w)] = 1.0
    phi, _ = oracle.design_matrix(p.sci, p.tmpl, p.mask, w, dk, db)
    nkk = L * L * oracle.num_basis(dk)
    mb = oracle.monomials(ny, nx, db)
    # model at every pixel: the kernel part through the zero-filled template,
    # the background without the output mask
    model = (phi[:, :nkk] @ theta_true[:nkk]).reshape(ny, nx) + np.tensordot(theta_true[nkk:], mb, axes=(0, 0))
    sci = model.copy()
    bad = p.mask != 0
    sci[bad] = rng.normal(0.0, 1e4, int(bad.sum()))
    got = oracle.fit_outmask(sci, p.tmpl, p.mask, w, dk, db, mode="direct")["theta"]
    assert oracle.rel_err(got, theta_true) < 1e-10
    got_fft = oracle.fit_outmask(sci, p.tmpl, p.mask, w, dk, db, mode="fft")["theta"]
    assert oracle.rel_err(got_fft, theta_true) < 1e-10
    zf = oracle.fit(sci, p.tmpl, p.mask, w, dk, db, mode="direct")["theta"]
    assert oracle.rel_err(zf, theta_true) > 1e-3


def test_no_mask_is_the_zero_filled_system():
    p = synth.random_pair(21, 24, 22, 2, 1, 1, mask_frac=0.0, stars=True)
    om, be = oracle.normal_system_outmask(p.sci, p.tmpl, None, 2, 1, 1, mode="direct")
    om0, be0 = oracle.normal_system(p.sci, p.tmpl, None, 2, 1, 1, mode="direct")
    np.testing.assert_array_equal(om, om0)
    np.testing.assert_array_equal(be, be0)
    assert oracle.masked_rows(p.tmpl, None, 2, 1).shape == (0, 25 * 3)


def test_excluded_science_values_do_not_matter():
    p = synth.random_pair(22, 30, 28, 2, 2, 1, mask_frac=0.15, stars=True)
    a = oracle.fit_outmask(p.sci, p.tmpl, p.mask, 2, 2, 1, mode="fft")["theta"]
    s2 = p.sci.copy()
    s2[p.mask != 0] += 1e5
    b = oracle.fit_outmask(s2, p.tmpl, p.mask, 2, 2, 1, mode="fft")["theta"]
    assert oracle.rel_err(b, a) < 1e-12
