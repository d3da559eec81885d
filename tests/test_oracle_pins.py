"""Pins of the CPU FP64 oracle against things other than itself.

Each test checks the oracle against an independent statement of the fit:
  * brute force -- the design matrix written pixel by pixel with plain
    Python loops, solved by SVD least squares (numpy.linalg.lstsq), which
    never forms the normal matrix;
  * a closed form -- with a 1x1 kernel, no spatial variation and a constant
    background the fit is ordinary least squares of S on R over the good
    pixels;
  * exact recovery of a known kernel and background from noiseless data;
  * the sign of a pure shift;
  * flux conservation of the convolution;
  * invariants (symmetry, positive definiteness, Toeplitz blocks, residual,
    insensitivity to excluded pixels, linearity in S);
  * the FFT route against the explicit-design-matrix route.
"""
import itertools

import numpy as np
import pytest

import oracle
import synth


# ---------------------------------------------------------------------------
# brute-force statement of the fit, pixel by pixel (independent of the oracle)
# ---------------------------------------------------------------------------

def _mono(deg):
    out = []
    for d in range(deg + 1):
        for q in range(d + 1):
            out.append((d - q, q))
    return out


def brute_phi(S, R, M, w, dk, db):
    """Design matrix and target with plain loops over pixels and columns."""
    ny, nx = S.shape
    L = 2 * w + 1
    km, bm = _mono(dk), _mono(db)
    n = L * L * len(km) + len(bm)
    phi = np.zeros((ny * nx, n))
    tgt = np.zeros(ny * nx)

    def xh(x):
        return 2.0 * x / (nx - 1) - 1.0

    def yh(y):
        return 2.0 * y / (ny - 1) - 1.0

    def good(y, x):
        return M is None or M[y, x] == 0

    def tmpl_ok(y, x):
        return good(y, x) and w <= y < ny - w and w <= x < nx - w

    for y in range(ny):
        for x in range(nx):
            row = y * nx + x
            if good(y, x):
                tgt[row] = S[y, x]
            col = 0
            for (p, q) in km:
                for uy in range(-w, w + 1):
                    for ux in range(-w, w + 1):
                        sy, sx = y - uy, x - ux          # (T_u X)(y, x) = X(y - u_y, x - u_x)
                        if 0 <= sy < ny and 0 <= sx < nx and tmpl_ok(sy, sx):
                            phi[row, col] = xh(sx) ** p * yh(sy) ** q * R[sy, sx]
                        col += 1
            for (p, q) in bm:
                if good(y, x):
                    phi[row, col] = xh(x) ** p * yh(y) ** q
                col += 1
    return phi, tgt


def brute_diff(S, R, theta, w, dk, db):
    """D = S - kernel model (unmasked R, zero outside the frame) - background, by loops."""
    ny, nx = S.shape
    L = 2 * w + 1
    km, bm = _mono(dk), _mono(db)
    D = np.array(S, dtype=np.float64)
    for y in range(ny):
        for x in range(nx):
            acc = 0.0
            col = 0
            for (p, q) in km:
                for uy in range(-w, w + 1):
                    for ux in range(-w, w + 1):
                        sy, sx = y - uy, x - ux
                        if 0 <= sy < ny and 0 <= sx < nx:
                            acc += theta[col] * (2.0 * sx / (nx - 1) - 1.0) ** p \
                                * (2.0 * sy / (ny - 1) - 1.0) ** q * R[sy, sx]
                        col += 1
            for (p, q) in bm:
                acc += theta[col] * (2.0 * x / (nx - 1) - 1.0) ** p * (2.0 * y / (ny - 1) - 1.0) ** q
                col += 1
            D[y, x] -= acc
    return D


CASES = [
    # (ny, nx, w, dk, db, mask_frac, seed)
    (12, 12, 1, 0, 0, 0.0, 1),
    (14, 13, 1, 1, 1, 0.15, 2),
    (16, 16, 2, 2, 2, 0.10, 3),
    (19, 16, 2, 1, 2, 0.20, 4),
    (16, 20, 3, 0, 1, 0.05, 5),
    (13, 15, 0, 2, 0, 0.10, 6),
]


@pytest.mark.parametrize("ny,nx,w,dk,db,frac,seed", CASES)
@pytest.mark.parametrize("mode", ["direct", "fft"])
def test_bruteforce_lstsq(ny, nx, w, dk, db, frac, seed, mode):
    p = synth.random_pair(seed, ny, nx, w, dk, db, mask_frac=frac, stars=False)
    phi, tgt = brute_phi(p.sci, p.tmpl, p.mask, w, dk, db)
    theta_ref, *_ = np.linalg.lstsq(phi, tgt, rcond=None)
    sv = np.linalg.svd(phi, compute_uv=False)
    cond = sv[0] / sv[-1]
    om, be = oracle.normal_system(p.sci, p.tmpl, p.mask, w, dk, db, mode=mode)
    theta = oracle.solve(om, be)
    assert oracle.rel_err(theta, theta_ref) < 1e-13 * cond * cond + 1e-12
    # the normal matrix itself, entry by entry, against Phi^T Phi of the brute-force Phi
    np.testing.assert_allclose(om, phi.T @ phi, rtol=0, atol=1e-11 * np.abs(phi.T @ phi).max())
    np.testing.assert_allclose(be, phi.T @ tgt, rtol=0, atol=1e-11 * np.abs(phi.T @ tgt).max())
    D = oracle.difference(p.sci, p.tmpl, theta, w, dk, db, mode=mode)
    D_ref = brute_diff(p.sci, p.tmpl, theta_ref, w, dk, db)
    assert oracle.rel_err(D, D_ref) < 1e-12 * cond * cond + 1e-11


def test_closed_form_ols():
    """w=0, DK=DB=0: k = cov(S,R)/var(R), c = mean(S) - k mean(R) over good pixels."""
    p = synth.random_pair(11, 40, 36, 0, 0, 0, mask_frac=0.2, stars=True)
    g = p.mask == 0
    s, r = p.sci[g], p.tmpl[g]
    k = np.mean((s - s.mean()) * (r - r.mean())) / np.mean((r - r.mean()) ** 2)
    c = s.mean() - k * r.mean()
    for mode in ("direct", "fft"):
        om, be = oracle.normal_system(p.sci, p.tmpl, p.mask, 0, 0, 0, mode=mode)
        th = oracle.solve(om, be)
        assert abs(th[0] - k) <= 1e-12 * abs(k)
        assert abs(th[1] - c) <= 1e-10 * max(1.0, abs(c))


def _strip_vanishing_template(rng, ny, nx, w):
    R = rng.normal(0.0, 1.0, (ny, nx)) + rng.random((ny, nx)) * 5.0
    R[:w, :] = 0.0
    R[ny - w:, :] = 0.0
    R[:, :w] = 0.0
    R[:, nx - w:] = 0.0
    return R


@pytest.mark.parametrize("ny,nx,w,dk_true,dk,db_true,db", [
    (24, 24, 2, 1, 1, 1, 1),
    (28, 26, 3, 1, 2, 0, 2),
    (32, 32, 2, 2, 2, 2, 2),
])
def test_exact_recovery(ny, nx, w, dk_true, dk, db_true, db):
    """Noiseless S built from a known theta (brute force) is fitted back exactly."""
    rng = np.random.default_rng(100 + ny + w)
    R = _strip_vanishing_template(rng, ny, nx, w)
    L = 2 * w + 1
    nk, nb = oracle.num_basis(dk), oracle.num_basis(db)
    theta_true = np.zeros(L * L * nk + nb)
    nk_t, nb_t = oracle.num_basis(dk_true), oracle.num_basis(db_true)
    theta_true[:L * L * nk_t] = rng.normal(0.0, 1.0, L * L * nk_t)
    theta_true[L * L * nk:L * L * nk + nb_t] = rng.normal(0.0, 3.0, nb_t)
    # S = model(theta_true): brute-force difference image of S = 0 is -model
    S = -brute_diff(np.zeros((ny, nx)), R, theta_true, w, dk, db)
    for mode in ("direct", "fft"):
        res = oracle.fit(S, R, None, w, dk, db, mode=mode)
        assert oracle.rel_err(res["theta"], theta_true) < 1e-10
        assert np.abs(res["diff"]).max() <= 1e-12 * np.abs(S).max()


@pytest.mark.parametrize("d", [(0, 0), (1, 0), (0, 1), (-2, 1), (2, -2), (-1, -1)])
def test_shift_sign(d):
    """S = R moved by +d (content at x moves to x + d) gives k_{0,d} = 1, all else 0."""
    w, ny, nx = 2, 24, 22
    rng = np.random.default_rng(7)
    R = _strip_vanishing_template(rng, ny, nx, w)
    S = np.zeros_like(R)
    dy, dx = d
    for y in range(ny):
        for x in range(nx):
            if 0 <= y - dy < ny and 0 <= x - dx < nx:
                S[y, x] = R[y - dy, x - dx]
    th = oracle.fit(S, R, None, w, 0, 0, mode="direct")["theta"]
    expect = np.zeros_like(th)
    expect[(dy + w) * (2 * w + 1) + (dx + w)] = 1.0
    np.testing.assert_allclose(th, expect, atol=1e-11)


def test_flux_conservation():
    """With R vanishing on the strip, the kernel model sums to sum_z R(z) kappa(z)."""
    rng = np.random.default_rng(21)
    ny, nx, w, dk, db = 30, 27, 3, 2, 1
    R = _strip_vanishing_template(rng, ny, nx, w)
    L = 2 * w + 1
    nk = oracle.num_basis(dk)
    theta = np.concatenate([rng.normal(0, 1, L * L * nk), np.zeros(oracle.num_basis(db))])
    for mode in ("direct", "fft"):
        model = -oracle.difference(np.zeros((ny, nx)), R, theta, w, dk, db, mode=mode)
        xh = 2.0 * np.arange(nx) / (nx - 1) - 1.0
        yh = 2.0 * np.arange(ny) / (ny - 1) - 1.0
        kappa = np.zeros((ny, nx))
        for a, (p, q) in enumerate(_mono(dk)):
            kappa += theta[a * L * L:(a + 1) * L * L].sum() * np.outer(yh ** q, xh ** p)
        assert abs(model.sum() - (R * kappa).sum()) <= 1e-11 * np.abs(R * kappa).sum()


def test_transient_flux_c1():
    """Injected point source in the 256^2 pair is recovered within 1% by aperture flux in D."""
    p = synth.pair_c1()
    res = oracle.fit(p.sci, p.tmpl, p.mask, p.w, p.dk, p.db, mode="fft")
    D = res["diff"]
    tx, ty = p.truth["transient_xy"]
    yy, xx = np.mgrid[0:256, 0:256]
    r = np.hypot(xx - tx, yy - ty)
    ap = r <= 6.0
    ann = (r > 12.0) & (r < 20.0)
    flux = (D[ap] - np.median(D[ann])).sum()
    # the aperture holds all but the far Gaussian tail of the transient's PSF
    sig = p.truth["transient_sigma"]
    enclosed = 1.0 - np.exp(-0.5 * (6.0 / sig) ** 2)
    assert abs(flux / (p.truth["transient_flux"] * enclosed) - 1.0) < 0.01


@pytest.fixture(scope="module")
def small_system():
    p = synth.random_pair(31, 40, 44, 3, 2, 2, mask_frac=0.1, stars=True)
    om, be = oracle.normal_system(p.sci, p.tmpl, p.mask, p.w, p.dk, p.db, mode="direct")
    return p, om, be


def test_invariants_symmetry_pd_toeplitz(small_system):
    p, om, be = small_system
    assert np.abs(om - om.T).max() <= 1e-12 * np.abs(om).max()
    assert np.linalg.eigvalsh(om)[0] > 0
    L = 2 * p.w + 1
    nk = oracle.num_basis(p.dk)
    us = [(uy, ux) for uy in range(-p.w, p.w + 1) for ux in range(-p.w, p.w + 1)]
    for a, b in itertools.product(range(nk), range(nk)):
        blk = om[a * L * L:(a + 1) * L * L, b * L * L:(b + 1) * L * L]
        seen = {}
        for i, u in enumerate(us):
            for j, v in enumerate(us):
                key = (u[0] - v[0], u[1] - v[1])
                if key in seen:
                    assert abs(blk[i, j] - seen[key]) <= 1e-11 * np.abs(blk).max()
                else:
                    seen[key] = blk[i, j]


def test_invariants_residual_and_linearity(small_system):
    p, om, be = small_system
    th = oracle.solve(om, be)
    assert np.linalg.norm(be - om @ th) / np.linalg.norm(be) <= 1e-12
    # theta is linear in S
    th2 = oracle.solve(*oracle.normal_system(2.5 * p.sci, p.tmpl, p.mask, p.w, p.dk, p.db, mode="direct"))
    assert oracle.rel_err(th2, 2.5 * th) < 1e-10


def test_invariants_excluded_pixels(small_system):
    p, om, be = small_system
    th = oracle.solve(om, be)
    rng = np.random.default_rng(5)
    bad = p.mask != 0
    S2 = p.sci.copy()
    R2 = p.tmpl.copy()
    S2[bad] += rng.normal(0, 100, bad.sum())
    R2[bad] += rng.normal(0, 100, bad.sum())
    w = p.w
    R2[:w, :] += 50.0   # the template's w-strip never enters the fit
    R2[:, -w:] -= 30.0
    for mode in ("direct", "fft"):
        th2 = oracle.solve(*oracle.normal_system(S2, R2, p.mask, p.w, p.dk, p.db, mode=mode))
        assert oracle.rel_err(th2, th) < 1e-11
    # ... but D uses the unmasked template, so changes there show up in D
    D1 = oracle.difference(p.sci, p.tmpl, th, p.w, p.dk, p.db, mode="direct")
    D2 = oracle.difference(p.sci, R2, th, p.w, p.dk, p.db, mode="direct")
    assert np.abs(D1 - D2).max() > 1.0


@pytest.mark.parametrize("ny,nx,w,dk,db,seed", [
    (48, 48, 3, 2, 2, 41), (64, 40, 4, 1, 2, 42), (33, 57, 2, 2, 1, 43), (26, 26, 6, 0, 0, 44)])
def test_fft_route_equals_direct(ny, nx, w, dk, db, seed):
    p = synth.random_pair(seed, ny, nx, w, dk, db, mask_frac=0.1, stars=True)
    od, bd = oracle.normal_system(p.sci, p.tmpl, p.mask, w, dk, db, mode="direct")
    of, bf = oracle.normal_system(p.sci, p.tmpl, p.mask, w, dk, db, mode="fft")
    assert np.abs(of - od).max() <= 1e-12 * np.abs(od).max()
    assert np.abs(bf - bd).max() <= 1e-12 * np.abs(bd).max()
    th = oracle.solve(od, bd)
    Dd = oracle.difference(p.sci, p.tmpl, th, w, dk, db, mode="direct")
    Df = oracle.difference(p.sci, p.tmpl, th, w, dk, db, mode="fft")
    assert np.abs(Dd - Df).max() <= 1e-12 * np.abs(p.sci).max()


def test_planted_mistakes_are_caught():
    """A wrong shift sign or a transposed operand in the normal matrix breaks the brute-force match."""
    p = synth.random_pair(3, 16, 16, 2, 1, 1, mask_frac=0.1, stars=False)
    phi, tgt = brute_phi(p.sci, p.tmpl, p.mask, 2, 1, 1)
    om, _ = oracle.normal_system(p.sci, p.tmpl, p.mask, 2, 1, 1, mode="fft")
    ref = phi.T @ phi
    assert np.abs(om - ref).max() <= 1e-11 * np.abs(ref).max()
    # a sign flip of the lag (C_ab(v - u) instead of C_ab(u - v)) only agrees on symmetric blocks
    L = 5
    nk = 3
    flipped = om.copy()
    for a in range(nk):
        for b in range(nk):
            blk = om[a * L * L:(a + 1) * L * L, b * L * L:(b + 1) * L * L]
            flipped[a * L * L:(a + 1) * L * L, b * L * L:(b + 1) * L * L] = blk.T
    assert np.abs(flipped - ref).max() > 1e-6 * np.abs(ref).max()


def test_single_entry_and_pixel_functions_agree_with_full_system():
    """omega_entries / beta_entries / difference_at (used for sampled checks) match the full oracle."""
    p = synth.random_pair(81, 30, 34, 2, 2, 1, mask_frac=0.1, stars=True)
    om, be = oracle.normal_system_direct(p.sci, p.tmpl, p.mask, p.w, p.dk, p.db)
    rng = np.random.default_rng(3)
    n = om.shape[0]
    pairs = [tuple(x) for x in rng.integers(0, n, (25, 2))] + [(n - 1, n - 2), (0, n - 1)]
    got = oracle.omega_entries(p.sci, p.tmpl, p.mask, p.w, p.dk, p.db, pairs)
    ref = np.array([om[r, c] for r, c in pairs])
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * np.abs(om).max())
    rows = list(rng.integers(0, n, 10)) + [n - 1]
    np.testing.assert_allclose(oracle.beta_entries(p.sci, p.tmpl, p.mask, p.w, p.dk, p.db, rows), be[rows],
                               rtol=0, atol=1e-12 * np.abs(be).max())
    th = oracle.solve(om, be)
    D = oracle.difference(p.sci, p.tmpl, th, p.w, p.dk, p.db, mode="direct")
    ys, xs = np.meshgrid(np.arange(30), np.arange(34), indexing="ij")   # every pixel, borders included
    ys, xs = ys.ravel(), xs.ravel()
    np.testing.assert_allclose(oracle.difference_at(p.sci, p.tmpl, th, p.w, p.dk, p.db, ys, xs),
                               D[ys, xs], rtol=0, atol=1e-12 * np.abs(p.sci).max())


# ---------------------------------------------------------------------------
# background for a fixed kernel, and the residual ratio that judges a guess
# ---------------------------------------------------------------------------

def test_fit_background_equals_brute_force_lstsq():
    """For a fixed (arbitrary) kernel, the restricted normal-equation solve
    equals an SVD least-squares fit of the background columns of the
    brute-force design matrix to S_m - Phi_K k (which never forms Omega)."""
    p = synth.random_pair(61, 18, 17, 2, 1, 2, mask_frac=0.15)
    S, R, Mk, w, dk, db = p.sci, p.tmpl, p.mask, 2, 1, 2
    phi, tgt = brute_phi(S, R, Mk, w, dk, db)
    nkk = (2 * w + 1) ** 2 * oracle.num_basis(dk)
    k = np.random.default_rng(5).normal(0.0, 0.2, nkk)
    c_ref, *_ = np.linalg.lstsq(phi[:, nkk:], tgt - phi[:, :nkk] @ k, rcond=None)
    om, be = oracle.normal_system(S, R, Mk, w, dk, db, mode="direct")
    th = oracle.fit_background(om, be, np.concatenate([k, np.zeros(len(c_ref))]), nkk)
    np.testing.assert_array_equal(th[:nkk], k)
    np.testing.assert_allclose(th[nkk:], c_ref, rtol=1e-9, atol=1e-9 * np.abs(c_ref).max())


def test_fit_background_keeps_the_full_solution_and_rho_vanishes():
    """At the full least-squares solution the background rows already hold,
    so completing its kernel returns its own background, and rho ~ 0; rho
    equals ||Phi^T (S_m - Phi theta)|| / ||Phi^T S_m|| for any theta."""
    p = synth.random_pair(62, 20, 21, 2, 1, 1, mask_frac=0.1)
    S, R, Mk, w, dk, db = p.sci, p.tmpl, p.mask, 2, 1, 1
    om, be = oracle.normal_system(S, R, Mk, w, dk, db, mode="direct")
    th = oracle.solve(om, be)
    nkk = (2 * w + 1) ** 2 * oracle.num_basis(dk)
    th2 = oracle.fit_background(om, be, th, nkk)
    assert oracle.rel_err(th2, th) < 1e-10
    assert oracle.residual_ratio(om, be, th) < 1e-12
    phi, tgt = brute_phi(S, R, Mk, w, dk, db)
    guess = th + np.random.default_rng(1).normal(0.0, 0.01, th.size)
    ref = np.linalg.norm(phi.T @ (tgt - phi @ guess)) / np.linalg.norm(phi.T @ tgt)
    assert abs(oracle.residual_ratio(om, be, guess) - ref) <= 1e-9 * ref


# ---------------------------------------------------------------------------
# the error metric and the condition number reported with every result
# ---------------------------------------------------------------------------

def test_rel_err_closed_forms():
    """rel_err is the whole-array 2-norm ratio ||x - ref|| / ||ref|| (A11 reading):
    pinned by offsets whose norms are fixed by geometry, not by retyping the formula."""
    ref = np.array([0.0, 0.0, 12.0, 5.0])                 # ||ref|| = 13
    assert oracle.rel_err(ref, ref) == 0.0
    # an offset of 2-norm 5 (3-4-5 triangle) gives 5/13; a max-norm reading would give 4/12,
    # a 1-norm reading 7/17
    assert oracle.rel_err(ref + np.array([3.0, 4.0, 0.0, 0.0]), ref) == pytest.approx(5.0 / 13.0, rel=1e-15)
    # scaling: x = c ref -> |c - 1|
    for cfac, want in ((3.0, 2.0), (-1.0, 2.0), (0.0, 1.0), (1.5, 0.5)):
        assert oracle.rel_err(cfac * ref, ref) == pytest.approx(want, rel=1e-15)
    # 2-D arrays: the Frobenius norm over the whole array (equal to the flattened vector)
    r2 = np.arange(1.0, 13.0).reshape(3, 4)
    x2 = r2.copy()
    x2[1, 2] += 2.0
    x2[2, 0] -= 1.0
    assert oracle.rel_err(x2, r2) == pytest.approx(np.sqrt(5.0) / np.sqrt(650.0), rel=1e-14)
    # an orthogonal offset of relative size t: rel_err = t whatever the direction
    rng = np.random.default_rng(5)
    v = rng.normal(size=50)
    e = rng.normal(size=50)
    e -= (e @ v) / (v @ v) * v
    e *= 0.25 * np.linalg.norm(v) / np.linalg.norm(e)
    assert oracle.rel_err(v + e, v) == pytest.approx(0.25, rel=1e-13)
    # a zero reference: the absolute norm (denominator 1)
    assert oracle.rel_err(np.array([3.0, 4.0]), np.zeros(2)) == 5.0


def test_cond_number_closed_forms():
    """cond_number is the 2-norm condition number lambda_max / lambda_min of an SPD matrix."""
    assert oracle.cond_number(np.diag([1.0, 10.0, 1000.0])) == pytest.approx(1000.0, rel=1e-14)
    # invariant under an orthogonal change of basis
    q, _ = np.linalg.qr(np.random.default_rng(1).normal(size=(6, 6)))
    a = q @ np.diag([2.0, 3.0, 5.0, 7.0, 11.0, 0.5]) @ q.T
    assert oracle.cond_number(a) == pytest.approx(22.0, rel=1e-12)
    # the 4 x 4 Hilbert matrix, cond_2 = 1.5514e4 (a textbook value)
    h4 = 1.0 / (np.arange(4)[:, None] + np.arange(4)[None, :] + 1.0)
    assert oracle.cond_number(h4) == pytest.approx(15513.74, rel=1e-6)
    # singular or indefinite: infinite
    assert oracle.cond_number(np.array([[1.0, 1.0], [1.0, 1.0]])) == float("inf")
    assert oracle.cond_number(np.diag([1.0, -2.0])) == float("inf")
