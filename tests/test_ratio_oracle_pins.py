"""Pins of the constant-photometric-ratio oracle (oracle.ratio_oracle) against
facts that do not come from its own KKT formula:

  * feasibility: the kernel sums of the non-constant monomials vanish;
  * optimality, from the Lagrange conditions: the gradient residual
    beta - Omega theta is zero on the constant monomial's coefficients and on
    the background, and constant over the coefficients of each other monomial;
  * a second derivation: minimising over a basis of C's null space
    (scipy.linalg.null_space) gives the same theta;
  * a general-purpose constrained minimiser (SLSQP) agrees on a tiny problem;
  * a noise-free pair made by a kernel that already satisfies the
    constraint is fitted exactly, and the constrained optimum is never better
    than the free one;
  * the point-source meaning: the fitted kernel, applied with the kernel
    oracle to point sources anywhere in the frame, conserves one and the
    same flux ratio, while the free fit's ratio varies."""
import numpy as np
import pytest
import scipy.linalg
import scipy.optimize

import oracle
import synth
from oracle import ratio_oracle as RO


def _system(seed, n, w, dk, db, mask_frac=0.1):
    p = synth.random_pair(seed, n, n, w, dk, db, mask_frac=mask_frac)
    om, be = oracle.normal_system(p.sci, p.tmpl, p.mask, w, dk, db, mode="direct")
    return p, om, be


@pytest.mark.parametrize("w,dk,db", [(1, 1, 1), (2, 2, 1), (1, 3, 0)])
def test_feasible_and_stationary(w, dk, db):
    _, om, be = _system(11 + w + dk, 20, w, dk, db)
    th, lam = RO.solve_const_ratio(om, be, w, dk, db)
    L2 = (2 * w + 1) ** 2
    nk = oracle.num_basis(dk)
    s = RO.kernel_sums(th, w, dk)
    assert np.all(np.abs(s[1:]) <= 1e-11 * np.abs(th[:nk * L2]).sum())
    g = be - om @ th
    scale = np.abs(be).max()
    assert np.abs(g[:L2]).max() <= 1e-10 * scale                 # constant monomial: free
    assert np.abs(g[nk * L2:]).max() <= 1e-10 * scale            # background: free
    for a in range(1, nk):                                       # constrained blocks: one multiplier each
        blk = g[a * L2:(a + 1) * L2]
        assert np.ptp(blk) <= 1e-10 * scale
        assert abs(blk.mean() - lam[a - 1]) <= 1e-9 * scale


@pytest.mark.parametrize("w,dk,db", [(1, 2, 1), (2, 1, 2)])
def test_null_space_derivation(w, dk, db):
    _, om, be = _system(23 + w, 18, w, dk, db)
    th, _ = RO.solve_const_ratio(om, be, w, dk, db)
    Z = scipy.linalg.null_space(RO.ratio_constraints(w, dk, db))
    y = np.linalg.solve(Z.T @ om @ Z, Z.T @ be)
    assert oracle.rel_err(th, Z @ y) <= 1e-9


def test_general_minimiser_tiny():
    w, dk, db = 1, 1, 0
    _, om, be = _system(31, 10, w, dk, db, mask_frac=0.0)
    th, _ = RO.solve_const_ratio(om, be, w, dk, db)
    C = RO.ratio_constraints(w, dk, db)
    sc = np.abs(be).max()
    res = scipy.optimize.minimize(lambda t: (t @ om @ t - 2 * be @ t) / sc, np.zeros(om.shape[0]),
                                  jac=lambda t: (2 * om @ t - 2 * be) / sc,
                                  constraints=[{"type": "eq", "fun": lambda t: C @ t, "jac": lambda t: C}],
                                  method="SLSQP", options=dict(ftol=1e-14, maxiter=2000))
    assert res.success
    assert oracle.rel_err(res.x, th) <= 1e-5


def test_feasible_truth_is_recovered_and_optimum_ordering():
    w, dk, db, n = 1, 2, 1, 16
    p = synth.random_pair(41, n, n, w, dk, db, mask_frac=0.0)   # masked pixels have target 0, not Phi theta
    rng = np.random.default_rng(5)
    nc = oracle.num_coeffs(w, dk, db)
    L2 = (2 * w + 1) ** 2
    nk = oracle.num_basis(dk)
    truth = rng.normal(0.0, 0.1, nc)
    for a in range(1, nk):                           # make every spatial term sum to zero
        truth[a * L2:(a + 1) * L2] -= truth[a * L2:(a + 1) * L2].mean()
    phi, _ = oracle.design_matrix(p.sci, p.tmpl, p.mask, w, dk, db)
    sci = (phi @ truth).reshape(n, n)                # noise-free science image
    om, be = oracle.normal_system(sci, p.tmpl, p.mask, w, dk, db, mode="direct")
    th, lam = RO.solve_const_ratio(om, be, w, dk, db)
    assert oracle.rel_err(th, truth) <= 1e-9
    assert np.abs(lam).max() <= 1e-8 * np.abs(be).max()
    # on real data the constrained objective is never below the free one
    _, om2, be2 = _system(43, n, w, dk, db)
    free = oracle.solve(om2, be2)
    con, _ = RO.solve_const_ratio(om2, be2, w, dk, db)
    f = lambda t: t @ om2 @ t - 2 * be2 @ t  # noqa: E731
    assert f(con) >= f(free) - 1e-9 * abs(f(free))


def test_point_sources_see_one_flux_ratio():
    w, dk, db, n = 2, 2, 1, 24
    p, om, be = _system(53, n, w, dk, db)
    con, _ = RO.solve_const_ratio(om, be, w, dk, db)
    free = oracle.solve(om, be)
    ratios = {}
    for name, th in (("con", con), ("free", free)):
        r = []
        for (y0, x0) in [(3, 3), (3, 20), (12, 12), (20, 4), (19, 19)]:
            delta = np.zeros((n, n))
            delta[y0, x0] = 1.0
            r.append(oracle.apply_kernel(delta, th, w, dk).sum())
        ratios[name] = np.asarray(r)
        # the ratio map is what a point source at that pixel sees
        rm = RO.ratio_map(th, w, dk, n, n)
        assert np.allclose([rm[y, x] for (y, x) in [(3, 3), (3, 20), (12, 12), (20, 4), (19, 19)]], r,
                           rtol=1e-12, atol=1e-12)
    assert np.ptp(ratios["con"]) <= 1e-12 * np.abs(ratios["con"]).max()
    assert np.ptp(ratios["free"]) > 1e-6 * np.abs(ratios["free"]).max()
