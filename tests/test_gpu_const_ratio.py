"""Constant photometric ratio on the GPU (SFFT_FLAG_CONST_RATIO) against the
CPU oracle's KKT solution (oracle.ratio_oracle).

Coefficients and difference image to the mode's bar (FP64 <= 1e-9, FP32C <=
1e-5 relative 2-norm; the oracle sees the float32-rounded images in FP32C),
the constraint itself (kernel sums of the non-constant monomials vanish to
FP64 rounding), the maximum constraint count (DK = 4: 14 columns), the
batched path (flagged and free pairs of several shapes in one batch, each
equal bit for bit to its single-pair plan), the no-allocation entry point,
and the no-op at DK = 0."""
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
BAR = {F64: 1e-9, F32C: 1e-5}
CR = B.SFFT_FLAG_CONST_RATIO

CASES = [
    # ny, nx, w, dk, db, mask_frac, seed
    (64, 64, 2, 1, 1, 0.10, 11),
    (100, 90, 3, 2, 2, 0.05, 12),     # rectangular, not a power of two
    (130, 129, 5, 3, 1, 0.20, 13),    # ragged tails
    (96, 96, 3, 4, 2, 0.10, 14),      # DK = 4: the most constraints (14)
]


def _as_seen(p, mode):
    if mode == F32C:
        return p.sci.astype(np.float32).astype(np.float64), p.tmpl.astype(np.float32).astype(np.float64)
    return p.sci, p.tmpl


def _reference(p, mode):
    s_in, r_in = _as_seen(p, mode)
    om, be = oracle.normal_system(s_in, r_in, p.mask, p.w, p.dk, p.db)
    th, _ = oracle.solve_const_ratio(om, be, p.w, p.dk, p.db)
    return th, oracle.difference(s_in, r_in, th, p.w, p.dk, p.db)


def _sums_vanish(theta, w, dk):
    L2 = (2 * w + 1) ** 2
    nk = oracle.num_basis(dk)
    s = oracle.kernel_sums(theta, w, dk)
    return np.abs(s[1:]).max() <= 1e-12 * np.abs(theta[:nk * L2]).sum()


@pytest.mark.parametrize("mode", [F64, F32C])
@pytest.mark.parametrize("case", CASES)
def test_const_ratio_matches_oracle(case, mode):
    ny, nx, w, dk, db, mf, seed = case
    p = synth.random_pair(seed, ny, nx, w, dk, db, mask_frac=mf)
    th_ref, d_ref = _reference(p, mode)
    res = run_pair(p.sci, p.tmpl, p.mask, w, dk, db, mode=mode, flags=CR, want_system=False)
    assert res["info"] == 0 and res["status"] == B.SFFT_OK
    et = oracle.rel_err(res["theta"], th_ref)
    ed = oracle.rel_err(res["diff"], d_ref)
    print(f"{case} mode {mode}: e_theta {et:.2e} e_D {ed:.2e}")
    assert et <= BAR[mode] and ed <= BAR[mode]
    assert _sums_vanish(res["theta"], w, dk)
    # the constraint changes the answer: the free fit's spatial sums do not vanish
    free = run_pair(p.sci, p.tmpl, p.mask, w, dk, db, mode=mode, want_system=False)
    assert not _sums_vanish(free["theta"], w, dk)


def test_dk0_is_a_no_op():
    p = synth.random_pair(21, 80, 80, 3, 0, 1, mask_frac=0.1)
    a = run_pair(p.sci, p.tmpl, p.mask, 3, 0, 1, flags=CR, want_system=False)
    b = run_pair(p.sci, p.tmpl, p.mask, 3, 0, 1, want_system=False)
    np.testing.assert_array_equal(a["theta"], b["theta"])
    np.testing.assert_array_equal(a["diff"], b["diff"])


@pytest.mark.parametrize("mode", [F64, F32C])
def test_batch_mixes_constrained_and_free_pairs(mode):
    shapes = [(96, 80, 3, 2, 2, CR), (128, 128, 5, 1, 1, 0), (70, 100, 2, 2, 1, CR), (96, 80, 3, 2, 2, 0),
              (150, 131, 6, 1, 2, CR | B.SFFT_FLAG_ASSEMBLY_FFT)]
    pairs = [synth.random_pair(300 + i, ny, nx, w, dk, db, mask_frac=0.1) for i, (ny, nx, w, dk, db, _) in
             enumerate(shapes)]
    dt = torch.float64 if mode == F64 else torch.float32
    descs = [B.make_desc(ny, nx, w, dk, db, mode, flags=f) for (ny, nx, w, dk, db, f) in shapes]
    h = B.sfft_batch_plan(descs)
    try:
        S = [torch.from_numpy(p.sci).to("cuda", dt) for p in pairs]
        R = [torch.from_numpy(p.tmpl).to("cuda", dt) for p in pairs]
        M = [torch.from_numpy(p.mask).cuda() for p in pairs]
        C = [torch.zeros(B.sfft_num_coeffs(d), dtype=torch.float64, device="cuda") for d in descs]
        Dd = [torch.empty_like(s) for s in S]
        info = torch.full((len(pairs),), -7, dtype=torch.int32, device="cuda")
        B.sfft_batch_run(h, S, R, M, [s.stride(0) for s in S], C, Dd, info)
        assert B.sfft_status(h)[0] == B.SFFT_OK
        assert info.cpu().tolist() == [0] * len(pairs)
        for i, (p, (ny, nx, w, dk, db, f)) in enumerate(zip(pairs, shapes)):
            single = run_pair(p.sci, p.tmpl, p.mask, w, dk, db, mode=mode, flags=f, want_system=False)
            np.testing.assert_array_equal(C[i].cpu().numpy(), single["theta"])
            np.testing.assert_array_equal(Dd[i].cpu().numpy().astype(np.float64), single["diff"])
            if f & CR:
                th_ref, _ = _reference(p, mode)
                assert oracle.rel_err(single["theta"], th_ref) <= BAR[mode]
                assert _sums_vanish(single["theta"], w, dk)
    finally:
        B.sfft_destroy(h)


def test_no_alloc_entry_point_takes_the_flag():
    p = synth.random_pair(41, 120, 112, 4, 2, 1, mask_frac=0.1)
    desc = B.make_desc(120, 112, 4, 2, 1, F64, flags=CR)
    S = torch.from_numpy(p.sci).cuda()
    R = torch.from_numpy(p.tmpl).cuda()
    M = torch.from_numpy(p.mask).cuda()
    coeffs = torch.zeros(B.sfft_num_coeffs(desc), dtype=torch.float64, device="cuda")
    diff = torch.empty_like(S)
    info = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    B.sfft_subtract_pair_noalloc(desc, S, R, M, S.stride(0), coeffs, diff, info)
    torch.cuda.synchronize()
    ref = run_pair(p.sci, p.tmpl, p.mask, 4, 2, 1, flags=CR, want_system=False)
    assert int(info.item()) == 0
    np.testing.assert_array_equal(coeffs.cpu().numpy(), ref["theta"])
    np.testing.assert_array_equal(diff.cpu().numpy(), ref["diff"])
