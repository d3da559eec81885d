"""GPU parity: the HIP path through the C ABI against the CPU FP64 oracle.

Tolerances (relative 2-norm errors against the oracle, as in the project's
target): FP64 mode <= 1e-9 on the coefficients and on the difference image;
FP32C mode <= 1e-5 on the coefficients and <= 1e-5 on the difference image
for the sizes where the FP32 transforms allow it (see the 4088 notes in the
design document).  Normal-matrix entries are compared element by element
relative to max |Omega|.
"""
import numpy as np
import pytest

import oracle
import synth
from paper_2509_18544_amd import binding as B

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

from gpu_util import run_pair  # noqa: E402

F64, F32C = B.SFFT_MODE_F64, B.SFFT_MODE_F32C
TOL = {F64: dict(theta=1e-9, diff=1e-9, omega=1e-12), F32C: dict(theta=1e-5, diff=1e-5, omega=2e-6)}


def inputs_as_seen(p, mode):
    """The images as the GPU path receives them: float32 in FP32C mode (upcast exactly)."""
    if mode == F32C:
        return p.sci.astype(np.float32).astype(np.float64), p.tmpl.astype(np.float32).astype(np.float64)
    return p.sci, p.tmpl


def _check_against_oracle(p, mode, res, ref=None, tol=None):
    tol = tol or TOL[mode]
    if ref is None:
        s_in, r_in = inputs_as_seen(p, mode)
        ref = oracle.fit(s_in, r_in, p.mask, p.w, p.dk, p.db)
    assert res["info"] == 0 and res["status"] == B.SFFT_OK
    if "omega" in res:
        scale = np.abs(ref["omega"]).max()
        err = np.abs(res["omega"] - ref["omega"]).max() / scale
        assert err <= tol["omega"], f"Omega entry error {err:.3e}"
        berr = np.abs(res["beta"] - ref["beta"]).max() / np.abs(ref["beta"]).max()
        assert berr <= tol["omega"], f"beta entry error {berr:.3e}"
    et = oracle.rel_err(res["theta"], ref["theta"])
    ed = oracle.rel_err(res["diff"], ref["diff"])
    assert et <= tol["theta"], f"e_theta {et:.3e}"
    assert ed <= tol["diff"], f"e_D {ed:.3e}"
    return et, ed


SMALL = [
    # ny, nx, w, dk, db, mask_frac, seed
    (64, 64, 2, 1, 1, 0.10, 1),
    (100, 90, 3, 2, 2, 0.05, 2),     # not a power of two, rectangular
    (128, 200, 4, 2, 1, 0.10, 3),    # Px = 256, Py = 128
    (37, 41, 1, 0, 0, 0.00, 4),      # smallest transform size (64)
    (70, 66, 0, 2, 2, 0.10, 5),      # w = 0
    (130, 129, 5, 1, 2, 0.20, 6),    # ragged tails past a power of two
]


FFT_ROUTE, DIRECT_ROUTE, MFMA_ROUTE = B.SFFT_FLAG_ASSEMBLY_FFT, B.SFFT_FLAG_ASSEMBLY_DIRECT, B.SFFT_FLAG_ASSEMBLY_MFMA


@pytest.mark.parametrize("route", [FFT_ROUTE, DIRECT_ROUTE, MFMA_ROUTE])
@pytest.mark.parametrize("mode", [F64, F32C])
@pytest.mark.parametrize("case", SMALL)
def test_small_parity(case, mode, route):
    ny, nx, w, dk, db, frac, seed = case
    p = synth.random_pair(seed, ny, nx, w, dk, db, mask_frac=frac, stars=True)
    res = run_pair(p.sci, p.tmpl, p.mask, w, dk, db, mode=mode, flags=route)
    _check_against_oracle(p, mode, res)


@pytest.mark.parametrize("route", [FFT_ROUTE, DIRECT_ROUTE, MFMA_ROUTE])
@pytest.mark.parametrize("mode", [F64, F32C])
def test_c1_parity(mode, route):
    p = synth.pair_c1()
    res = run_pair(p.sci, p.tmpl, p.mask, p.w, p.dk, p.db, mode=mode, flags=route)
    et, ed = _check_against_oracle(p, mode, res)
    print(f"C1 mode={mode} route={route} e_theta={et:.3e} e_D={ed:.3e}")


def test_routes_agree_on_omega():
    """The direct sums, the matrix-core products and the transforms give the same
    Omega up to rounding (FP64), entry by entry."""
    p = synth.random_pair(81, 150, 140, 4, 2, 1, mask_frac=0.1, stars=True)
    a = run_pair(p.sci, p.tmpl, p.mask, p.w, p.dk, p.db, flags=FFT_ROUTE)
    scale = np.abs(a["omega"]).max()
    for route in (DIRECT_ROUTE, MFMA_ROUTE):
        b = run_pair(p.sci, p.tmpl, p.mask, p.w, p.dk, p.db, flags=route)
        assert np.abs(a["omega"] - b["omega"]).max() <= 1e-12 * scale, route
        assert np.abs(a["beta"] - b["beta"]).max() <= 1e-12 * np.abs(a["beta"]).max(), route


@pytest.mark.parametrize("mode", [F64, F32C])
def test_route_autotune_keeps_the_fastest_and_the_result(mode):
    """sfft_autotune_route times every allowed route on the real pair and keeps
    the fastest on an AUTO plan; the fit after it still matches the oracle."""
    p = synth.random_pair(82, 192, 176, 5, 1, 1, mask_frac=0.05, stars=True)
    dt = torch.float64 if mode == F64 else torch.float32
    S, R = torch.from_numpy(p.sci).to("cuda", dt), torch.from_numpy(p.tmpl).to("cuda", dt)
    M = torch.from_numpy(p.mask).cuda()
    plan = B.Plan(*p.sci.shape, p.w, p.dk, p.db, mode=mode)
    try:
        ms, route = B.sfft_autotune_route(plan.handle, S, R, M, S.stride(0))
        timed = {k: v for k, v in ms.items() if v is not None}
        assert set(timed) == {"fft", "direct", "mfma"} and all(v > 0 for v in timed.values())
        assert route == min(timed, key=timed.get)
        plan.build(S, R, M)
        coeffs, info = plan.solve()
        diff = plan.subtract(S, R, coeffs)
        res = dict(theta=coeffs.cpu().numpy(), diff=diff.cpu().numpy().astype(np.float64),
                   info=int(info.item()), status=plan.status()[0])
        _check_against_oracle(p, mode, res)
        print(f"route timings {ms} -> {route}")
    finally:
        plan.close()


@pytest.fixture(scope="module")
def c2_pair():
    return synth.pair_c2()


@pytest.mark.parametrize("mode", [F64, F32C])
def test_c2_parity(c2_pair, mode):
    p = c2_pair
    s_in, r_in = inputs_as_seen(p, mode)
    ref = oracle.fit(s_in, r_in, p.mask, p.w, p.dk, p.db, mode="fft")
    res = run_pair(p.sci, p.tmpl, p.mask, p.w, p.dk, p.db, mode=mode)
    et, ed = _check_against_oracle(p, mode, res, ref=ref)
    print(f"C2 mode={mode} e_theta={et:.3e} e_D={ed:.3e}")


@pytest.mark.parametrize("mode", [F64, F32C])
def test_subtract_alone(mode):
    """sfft_subtract with the oracle's coefficients reproduces the oracle's D."""
    p = synth.random_pair(21, 150, 140, 4, 2, 2, mask_frac=0.1, stars=True)
    ref = oracle.fit(p.sci, p.tmpl, p.mask, p.w, p.dk, p.db)
    res = run_pair(p.sci, p.tmpl, p.mask, p.w, p.dk, p.db, mode=mode, theta_in=ref["theta"],
                   want_system=False)
    tol = 1e-12 if mode == F64 else 1e-6
    if mode == F32C:
        # same coefficients; S and R rounded to float32 on the way in
        d_ref = oracle.difference(p.sci.astype(np.float32), p.tmpl.astype(np.float32), ref["theta"],
                                  p.w, p.dk, p.db)
    else:
        d_ref = ref["diff"]
    assert oracle.rel_err(res["diff"], d_ref) <= tol


def test_pitched_rows_and_null_mask():
    p = synth.random_pair(31, 80, 72, 3, 1, 1, mask_frac=0.0, stars=True)
    a = run_pair(p.sci, p.tmpl, None, p.w, p.dk, p.db)
    b = run_pair(p.sci, p.tmpl, np.zeros_like(p.mask), p.w, p.dk, p.db, pitch=96)
    np.testing.assert_array_equal(a["theta"], b["theta"])
    np.testing.assert_array_equal(a["diff"], b["diff"])
    _check_against_oracle(p, F64, a)


def test_deterministic_replay():
    p = synth.random_pair(41, 96, 96, 3, 2, 2, mask_frac=0.1, stars=True)
    a = run_pair(p.sci, p.tmpl, p.mask, p.w, p.dk, p.db, mode=F32C)
    b = run_pair(p.sci, p.tmpl, p.mask, p.w, p.dk, p.db, mode=F32C)
    np.testing.assert_array_equal(a["omega"], b["omega"])
    np.testing.assert_array_equal(a["theta"], b["theta"])
    np.testing.assert_array_equal(a["diff"], b["diff"])


def test_residual_judge():
    p = synth.random_pair(51, 64, 64, 2, 1, 1, mask_frac=0.1, stars=True)
    res = run_pair(p.sci, p.tmpl, p.mask, p.w, p.dk, p.db)
    assert res["rho"] <= 1e-12


def test_fully_masked_is_not_spd():
    p = synth.random_pair(61, 40, 40, 2, 1, 1, mask_frac=0.0, stars=True)
    mask = np.ones_like(p.mask)
    res = run_pair(p.sci, p.tmpl, mask, p.w, p.dk, p.db, want_system=False)
    assert res["info"] > 0
    assert res["status"] == B.SFFT_ENOTSPD
    assert np.all(res["theta"] == 0.0)      # coefficients left untouched


def test_nonfinite_input_flagged():
    p = synth.random_pair(71, 40, 40, 2, 1, 1, mask_frac=0.0, stars=True)
    sci = p.sci.copy()
    sci[5, 7] = np.nan
    res = run_pair(sci, p.tmpl, p.mask, p.w, p.dk, p.db, want_system=False)
    assert res["nonfinite"] == 1
    assert res["status"] == B.SFFT_ENONFINITE


def test_solve_before_build_and_bad_args():
    plan = B.Plan(64, 64, 2, 1, 1)
    try:
        c = torch.zeros(plan.n, dtype=torch.float64, device="cuda")
        i = torch.zeros(1, dtype=torch.int32, device="cuda")
        with pytest.raises(B.SfftError) as e:
            B.sfft_solve(plan.handle, c, i)
        assert e.value.status == B.SFFT_ESTATE
        x = torch.zeros((64, 64), dtype=torch.float64, device="cuda")
        with pytest.raises(B.SfftError) as e:
            B.sfft_build_system(plan.handle, x, x, None, 32)     # ld < nx
        assert e.value.status == B.SFFT_EINVAL
    finally:
        plan.close()


def test_native_library_is_loaded():
    """The HIP library the tests call is the in-tree build, and it is mapped."""
    import os
    in_tree = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                           "paper_2509_18544_amd", "_lib", "libsfft.so")
    assert os.path.realpath(B.LIB_PATH) == os.path.realpath(in_tree)
    B.lib()
    maps = open("/proc/self/maps").read()
    assert os.path.realpath(in_tree) in maps


@pytest.mark.parametrize("mode", [F64, F32C])
def test_fit_background_and_residual_of_a_guess(mode):
    """A perturbed kernel is completed with the GPU's background fit and
    judged with its residual; both against the oracle on the same guess."""
    p = synth.random_pair(71, 96, 80, 3, 2, 2, mask_frac=0.1, stars=True)
    s_in, r_in = inputs_as_seen(p, mode)
    om, be = oracle.normal_system(s_in, r_in, p.mask, p.w, p.dk, p.db)
    th = oracle.solve(om, be)
    nkk = (2 * p.w + 1) ** 2 * oracle.num_basis(p.dk)
    guess = th.copy()
    guess[:nkk] += np.random.default_rng(2).normal(0.0, 0.02 * np.abs(th[:nkk]).max(), nkk)
    guess[nkk:] = 12345.0                                  # must be overwritten
    ref = oracle.fit_background(om, be, guess, nkk)
    rho_ref = oracle.residual_ratio(om, be, ref)
    dt = torch.float64 if mode == F64 else torch.float32
    plan = B.Plan(*p.sci.shape, p.w, p.dk, p.db, mode=mode)
    try:
        plan.build(torch.from_numpy(s_in).to("cuda", dt), torch.from_numpy(r_in).to("cuda", dt),
                   torch.from_numpy(p.mask).cuda())
        C = torch.from_numpy(guess).cuda()
        plan.fit_background(C)
        rho = plan.residual(C)
        torch.cuda.synchronize()
        c = C.cpu().numpy()
        np.testing.assert_array_equal(c[:nkk], guess[:nkk])
        # FP32C: the FP32 forward spectra put ~2e-6 relative errors on Omega's entries, which the
        # cancellation in beta - Omega theta of a near-solution guess amplifies
        tol_b, tol_r = (1e-9, 1e-9) if mode == F64 else (1e-4, 1e-3)
        eb = oracle.rel_err(c[nkk:], ref[nkk:])
        er = abs(rho.item() - rho_ref) / rho_ref
        print(f"mode {mode}: background {eb:.2e}, rho {rho.item():.3e} vs {rho_ref:.3e}")
        assert eb <= tol_b and er <= tol_r
    finally:
        plan.close()


@pytest.mark.parametrize("mode", [F64, F32C])
def test_autotune_keeps_results_within_rounding(mode):
    """The tuned correlation chunk only regroups the residue sums: Omega, theta
    and D stay within rounding of the default plan, and still meet the oracle bar."""
    p = synth.random_pair(91, 200, 180, 4, 2, 2, mask_frac=0.1, stars=True)
    s_in, r_in = inputs_as_seen(p, mode)
    dt = torch.float64 if mode == F64 else torch.float32
    S = torch.from_numpy(s_in).to("cuda", dt)
    R = torch.from_numpy(r_in).to("cuda", dt)
    Mk = torch.from_numpy(p.mask).cuda()
    out = []
    for tune in (False, True):
        plan = B.Plan(*p.sci.shape, p.w, p.dk, p.db, mode=mode, flags=FFT_ROUTE)
        try:
            if tune:
                rep = B.sfft_autotune(plan.handle, S, R, Mk, S.stride(0))
                assert len(rep) >= 1 and all(ms > 0 for _, ms in rep)
            plan.build(S, R, Mk)
            om, be = plan.system()
            c, info = plan.solve()
            d = plan.subtract(S, R, c)
            torch.cuda.synchronize()
            out.append((om.cpu().numpy(), c.cpu().numpy(), d.cpu().numpy().astype(np.float64)))
        finally:
            plan.close()
    (om0, c0, d0), (om1, c1, d1) = out
    assert np.abs(om1 - om0).max() <= 1e-12 * np.abs(om0).max()
    ref = oracle.fit(s_in, r_in, p.mask, p.w, p.dk, p.db)
    assert oracle.rel_err(c1, ref["theta"]) <= TOL[mode]["theta"]
    assert oracle.rel_err(d1, ref["diff"]) <= TOL[mode]["diff"]


@pytest.mark.parametrize("route", [FFT_ROUTE, DIRECT_ROUTE, MFMA_ROUTE])
@pytest.mark.parametrize("shape", [(6, 6, 1, 0, 0), (10, 7, 1, 1, 1), (2, 2, 0, 0, 0), (3, 64, 0, 1, 0)])
def test_smallest_frames(shape, route):
    """Frames at the size limit N = 4w + 2 and degenerate thin frames (plain noise images)."""
    ny, nx, w, dk, db = shape
    p = synth.random_pair(100 + ny * nx, ny, nx, w, dk, db, mask_frac=0.0, stars=False)
    res = run_pair(p.sci, p.tmpl, p.mask, w, dk, db, flags=route)
    ref = oracle.fit(p.sci, p.tmpl, p.mask, w, dk, db, mode="direct")
    assert res["info"] == 0
    assert oracle.rel_err(res["theta"], ref["theta"]) <= 1e-9
    assert oracle.rel_err(res["diff"], ref["diff"]) <= 1e-9


# Kernel half-widths above 9 (lag windows of 41..61 rows, several passes of
# correlation items, the y-convolution instantiations for 10..15) and the
# polynomial degrees 3 and 4 (10 and 15 monomials, up to 31 planes) that the
# descriptor accepts.  The direct route takes w <= 9 only.
WIDE = [
    # ny, nx, w, dk, db, mask_frac, seed, routes
    (96, 96, 10, 1, 1, 0.05, 301, (FFT_ROUTE, MFMA_ROUTE)),
    (72, 80, 15, 0, 0, 0.05, 302, (FFT_ROUTE, MFMA_ROUTE)),
    (100, 92, 12, 0, 2, 0.10, 303, (FFT_ROUTE, MFMA_ROUTE)),
    (64, 64, 2, 4, 4, 0.10, 304, (FFT_ROUTE, DIRECT_ROUTE, MFMA_ROUTE)),
    (80, 76, 3, 3, 3, 0.10, 305, (FFT_ROUTE, DIRECT_ROUTE, MFMA_ROUTE)),
    (64, 80, 3, 4, 0, 0.05, 306, (FFT_ROUTE, DIRECT_ROUTE, MFMA_ROUTE)),
    (70, 70, 1, 0, 4, 0.05, 307, (FFT_ROUTE, DIRECT_ROUTE, MFMA_ROUTE)),
]


@pytest.mark.parametrize("mode", [F64, F32C])
@pytest.mark.parametrize("case", WIDE)
def test_wide_kernels_and_high_degrees(case, mode):
    ny, nx, w, dk, db, frac, seed, routes = case
    p = synth.random_pair(seed, ny, nx, w, dk, db, mask_frac=frac, stars=True)
    s_in, r_in = inputs_as_seen(p, mode)
    ref = oracle.fit(s_in, r_in, p.mask, w, dk, db, mode="direct")
    for route in routes:
        res = run_pair(p.sci, p.tmpl, p.mask, w, dk, db, mode=mode, flags=route)
        et, ed = _check_against_oracle(p, mode, res, ref=ref)
        print(f"{case[:5]} mode={mode} route={route}: e_theta={et:.2e} e_D={ed:.2e}")


@pytest.mark.parametrize("mode", [F64, F32C])
def test_autotune_wide_kernel_against_oracle(mode):
    """Autotuning a w >= 10 plan with more correlation items than one pass of
    the block takes (w = 10, DK = 3: 65 items of one rotation, one lane each,
    two passes) over every chunk size the LDS allows keeps Omega and theta at
    the oracle bar."""
    p = synth.random_pair(311, 256, 240, 10, 3, 1, mask_frac=0.05, stars=True)
    s_in, r_in = inputs_as_seen(p, mode)
    dt = torch.float64 if mode == F64 else torch.float32
    S = torch.from_numpy(s_in).to("cuda", dt)
    R = torch.from_numpy(r_in).to("cuda", dt)
    Mk = torch.from_numpy(p.mask).cuda()
    ref = oracle.fit(s_in, r_in, p.mask, p.w, p.dk, p.db, mode="fft")
    plan = B.Plan(*p.sci.shape, p.w, p.dk, p.db, mode=mode, flags=FFT_ROUTE)
    try:
        rep = B.sfft_autotune(plan.handle, S, R, Mk, S.stride(0))
        assert len(rep) >= 2
        chosen = min(rep, key=lambda cm: cm[1])[0]
        print(f"mode={mode}: candidates {rep}, chosen {chosen}")
        plan.build(S, R, Mk)
        om, be = plan.system()
        c, info = plan.solve()
        d = plan.subtract(S, R, c)
        st, inf, nf = plan.status()
        res = dict(omega=om.cpu().numpy(), beta=be.cpu().numpy(), theta=c.cpu().numpy(),
                   diff=d.cpu().numpy().astype(np.float64), info=int(info.item()), status=st)
    finally:
        plan.close()
    _check_against_oracle(p, mode, res, ref=ref)


@pytest.mark.parametrize("mode", [F64, F32C])
def test_caller_workspace(mode):
    """A plan on a caller-owned workspace gives the same results, bit for bit,
    as a plan that allocates its own."""
    p = synth.random_pair(321, 96, 88, 3, 2, 2, mask_frac=0.1, stars=True)
    a = run_pair(p.sci, p.tmpl, p.mask, p.w, p.dk, p.db, mode=mode)
    dt = torch.float64 if mode == F64 else torch.float32
    d = B.make_desc(96, 88, p.w, p.dk, p.db, mode)
    need = B.sfft_workspace_bytes(d)
    ws = torch.full((need + 512,), 0xA5, dtype=torch.uint8, device="cuda")   # not zeroed: nothing may rely on it
    S = torch.from_numpy(p.sci).to("cuda", dt)
    R = torch.from_numpy(p.tmpl).to("cuda", dt)
    Mk = torch.from_numpy(p.mask).cuda()
    h = B.sfft_plan(d, None, ws[256:], need)
    try:
        B.sfft_build_system(h, S, R, Mk, S.stride(0))
        om = torch.empty((a["omega"].shape[0],) * 2, dtype=torch.float64, device="cuda")
        be = torch.empty((a["omega"].shape[0],), dtype=torch.float64, device="cuda")
        B.sfft_get_system(h, om, be)
        c = torch.zeros_like(be)
        info = torch.zeros(1, dtype=torch.int32, device="cuda")
        B.sfft_solve(h, c, info)
        D = torch.empty_like(S)
        B.sfft_subtract(h, S, R, c, D, S.stride(0))
        assert B.sfft_status(h)[0] == B.SFFT_OK
        np.testing.assert_array_equal(om.cpu().numpy(), a["omega"])
        np.testing.assert_array_equal(c.cpu().numpy(), a["theta"])
        np.testing.assert_array_equal(D.cpu().numpy().astype(np.float64), a["diff"])
    finally:
        B.sfft_destroy(h)
    # the bytes outside the borrowed range are untouched
    assert torch.all(ws[:256] == 0xA5).item() and torch.all(ws[256 + need:] == 0xA5).item()
