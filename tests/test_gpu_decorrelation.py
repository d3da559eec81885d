"""Decorrelation kernel (pipeline step 7) on the GPU through the C ABI against
the CPU FP64 oracle: the kernel itself (max-abs error <= 1e-12 of max |psi|),
and the chain cross-convolution -> fit -> subtraction -> decorrelation of the
difference image against the oracle's chain (relative 2-norm <= 1e-9, FP64)."""
import numpy as np
import pytest

import oracle
import synth
from paper_2509_18544_amd import binding as B

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

F64 = B.SFFT_MODE_F64


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.float64))).cuda()


@pytest.mark.parametrize("ny,nx,w,dk,s,t,ss,sr", [
    (256, 256, 5, 1, 8, 10, 6.0, 4.0),
    (300, 280, 3, 2, 12, 15, 30.0, 20.0),
    (128, 96, 9, 0, 15, 7, 1.0, 3.0),
    (64, 64, 0, 0, 0, 0, 2.0, 2.0),
])
def test_decorrelation_kernel_against_oracle(ny, nx, w, dk, s, t, ss, sr):
    rng = np.random.default_rng(ny + w)
    L = 2 * w + 1
    nk = oracle.num_basis(dk)
    theta = np.zeros(nk * L * L + 1)
    theta[:L * L] = (synth.psf_stamp(1.2, 3.0, half=w) if w > 0 else np.ones((1, 1))).ravel()
    theta[L * L:nk * L * L] = 0.05 * rng.normal(size=(nk - 1) * L * L)
    ps = synth.psf_stamp(2.3, 3.0, half=s) if s > 0 else np.ones((1, 1))
    pr = synth.psf_stamp(1.9, 3.0, half=s) if s > 0 else np.ones((1, 1))
    plan = B.Plan(ny, nx, w, dk, 0, mode=F64)
    try:
        psi = torch.empty((2 * t + 1) ** 2, dtype=torch.float64, device="cuda")
        B.sfft_decorrelation_kernel(plan.handle, _dev(theta), _dev(ps), _dev(pr), s, ss, sr, t, psi)
        got = psi.cpu().numpy().reshape(2 * t + 1, 2 * t + 1)
    finally:
        plan.close()
    ref = oracle.decorrelation_kernel(theta, w, dk, ny, nx, ps, pr, ss, sr, t)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"psi ({ny}x{nx}, w={w}, dk={dk}, s={s}, t={t}): max err {err:.2e}")
    assert err <= 1e-12


def test_decorrelation_arguments_checked():
    plan = B.Plan(64, 64, 2, 0, 0, mode=F64)
    try:
        one = torch.ones(961, dtype=torch.float64, device="cuda")
        out = torch.empty(961, dtype=torch.float64, device="cuda")
        for s, t, ss, sr in ((16, 3, 1.0, 1.0), (3, 16, 1.0, 1.0), (3, 3, 0.0, 1.0), (3, 3, 1.0, float("nan")),
                             (-1, 3, 1.0, 1.0)):
            with pytest.raises(B.SfftError) as e:
                B.sfft_decorrelation_kernel(plan.handle, one, one, one, s, ss, sr, t, out)
            assert e.value.status == B.SFFT_EINVAL
    finally:
        plan.close()


def test_cross_convolve_subtract_decorrelate_chain():
    """Steps 5-7 on the 256^2 pair: every stage on the GPU, FP64, against the
    oracle's chain on the same inputs."""
    p = synth.pair_c1()
    ny, nx = p.sci.shape
    s, t = 8, 12
    pr = synth.psf_stamp(2.0, 3.0, half=s)      # template PSF P_R
    ps = synth.psf_stamp(2.4, 3.0, half=s)      # science PSF P_S
    sig_s, sig_r = 10.0, 10.0
    # GPU chain
    S, R, M = _dev(p.sci), _dev(p.tmpl), torch.from_numpy(p.mask).cuda()
    conv = B.Plan(ny, nx, s, 0, 0, mode=F64)
    plan = B.Plan(ny, nx, p.w, p.dk, p.db, mode=F64)
    dplan = B.Plan(ny, nx, t, 0, 0, mode=F64)
    try:
        S2 = conv.apply_kernel(S, _dev(pr.ravel()))
        R2 = conv.apply_kernel(R, _dev(ps.ravel()))
        plan.build(S2, R2, M)
        coeffs, info = plan.solve()
        D = plan.subtract(S2, R2, coeffs)
        psi = torch.empty((2 * t + 1) ** 2, dtype=torch.float64, device="cuda")
        B.sfft_decorrelation_kernel(plan.handle, coeffs, _dev(ps), _dev(pr), s, sig_s, sig_r, t, psi)
        Dd = dplan.apply_kernel(D, psi)
        assert plan.status()[0] == B.SFFT_OK and int(info.item()) == 0
        got = dict(S2=S2.cpu().numpy(), theta=coeffs.cpu().numpy(), D=D.cpu().numpy(),
                   psi=psi.cpu().numpy().reshape(2 * t + 1, -1), Dd=Dd.cpu().numpy())
    finally:
        conv.close()
        plan.close()
        dplan.close()
    # oracle chain
    s2 = oracle.convolve(p.sci, pr)
    r2 = oracle.convolve(p.tmpl, ps)
    ref = oracle.fit(s2, r2, p.mask, p.w, p.dk, p.db)
    psi_ref = oracle.decorrelation_kernel(ref["theta"], p.w, p.dk, ny, nx, ps, pr, sig_s, sig_r, t)
    dd_ref = oracle.convolve(ref["diff"], psi_ref)
    errs = dict(S2=oracle.rel_err(got["S2"], s2), theta=oracle.rel_err(got["theta"], ref["theta"]),
                D=oracle.rel_err(got["D"], ref["diff"]), psi=oracle.rel_err(got["psi"], psi_ref),
                Dd=oracle.rel_err(got["Dd"], dd_ref))
    print("chain errors", {k: f"{v:.2e}" for k, v in errs.items()})
    assert all(v <= 1e-9 for v in errs.values()), errs
