"""Output-masked fit on the GPU (SFFT_FLAG_OUTPUT_MASK) against its oracle.

The least squares runs over the good output pixels only: the zero-filled
normal matrix minus the Gram matrix of the excluded pixels' design rows, a
symmetric rank-|M| update on the FP64 matrix cores.  Omega, theta and D are
compared with oracle.fit_outmask on frames whose kernel block spans several
64 x 64 tiles with a ragged last tile and whose excluded pixels fill several
64-pixel chunks with a ragged last chunk; every assembly route, both
precision modes, the batch and the shared-template batch.
"""
import numpy as np
import pytest

import oracle
import synth
from paper_2509_18544_amd import binding as B

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from gpu_util import run_pair  # noqa: E402

F64, F32C = B.SFFT_MODE_F64, B.SFFT_MODE_F32C
OM = B.SFFT_FLAG_OUTPUT_MASK

CASES = [
    # (seed, ny, nx, w, dk, db, mask_frac): kernel block L^2 nK and tiles of 64
    (41, 64, 60, 3, 2, 2, 0.10),     # 294 = 4 tiles + 38
    (42, 96, 80, 9, 2, 2, 0.10),     # 2166 = 33 tiles + 54; 768 excluded pixels = 12 chunks
    (43, 70, 90, 5, 1, 0, 0.03),     # 363 = 5 tiles + 43; 189 excluded = 2 chunks + 61
    (44, 48, 48, 2, 0, 1, 0.30),     # 25: one ragged tile
]


def _inputs(case):
    seed, ny, nx, w, dk, db, frac = case
    p = synth.random_pair(seed, ny, nx, w, dk, db, mask_frac=frac, stars=True)
    mask = p.mask.copy()
    mask[0, :] = 1           # a whole row, and pixels on the frame edge
    mask[:, nx - 1] = 1
    return p, mask


@pytest.mark.parametrize("mode", [F64, F32C])
@pytest.mark.parametrize("case", CASES)
def test_output_mask_matches_oracle(case, mode):
    p, mask = _inputs(case)
    seed, ny, nx, w, dk, db, frac = case
    cast = np.float64 if mode == F64 else np.float32
    s_in, r_in = p.sci.astype(cast).astype(np.float64), p.tmpl.astype(cast).astype(np.float64)
    ref = oracle.fit_outmask(s_in, r_in, mask, w, dk, db, mode="fft")
    got = run_pair(p.sci, p.tmpl, mask, w, dk, db, mode=mode, flags=OM | B.SFFT_FLAG_ASSEMBLY_FFT)
    assert got["status"] == B.SFFT_OK and got["info"] == 0
    scale = np.abs(ref["omega"]).max()
    om_tol = 1e-12 if mode == F64 else 2e-6
    assert np.abs(got["omega"] - ref["omega"]).max() <= om_tol * scale
    tol = 1e-9 if mode == F64 else 1e-5
    assert oracle.rel_err(got["theta"], ref["theta"]) <= tol
    assert oracle.rel_err(got["diff"], ref["diff"]) <= tol
    # the corrected system differs from the zero-filled one
    zf = oracle.normal_system(s_in, r_in, mask, w, dk, db, mode="fft")[0]
    assert np.abs(got["omega"] - zf).max() > 1e3 * om_tol * scale


@pytest.mark.parametrize("route", [B.SFFT_FLAG_ASSEMBLY_DIRECT, B.SFFT_FLAG_ASSEMBLY_MFMA])
def test_output_mask_on_every_route(route):
    p, mask = _inputs(CASES[0])
    seed, ny, nx, w, dk, db, frac = CASES[0]
    ref = oracle.fit_outmask(p.sci, p.tmpl, mask, w, dk, db, mode="fft")
    got = run_pair(p.sci, p.tmpl, mask, w, dk, db, mode=F64, flags=OM | route)
    assert np.abs(got["omega"] - ref["omega"]).max() <= 1e-12 * np.abs(ref["omega"]).max()
    assert oracle.rel_err(got["theta"], ref["theta"]) <= 1e-9


def test_output_mask_without_excluded_pixels_is_the_zero_filled_fit():
    p, _ = _inputs(CASES[0])
    seed, ny, nx, w, dk, db, frac = CASES[0]
    for mask in (None, np.zeros_like(p.mask)):
        a = run_pair(p.sci, p.tmpl, mask, w, dk, db, mode=F64, flags=OM)
        b = run_pair(p.sci, p.tmpl, mask, w, dk, db, mode=F64, flags=0)
        np.testing.assert_array_equal(a["omega"], b["omega"])
        np.testing.assert_array_equal(a["theta"], b["theta"])


def test_output_mask_with_constant_ratio():
    p, mask = _inputs(CASES[2])
    seed, ny, nx, w, dk, db, frac = CASES[2]
    om, be = oracle.normal_system_outmask(p.sci, p.tmpl, mask, w, dk, db, mode="fft")
    ref, _ = oracle.solve_const_ratio(om, be, w, dk, db)
    got = run_pair(p.sci, p.tmpl, mask, w, dk, db, mode=F64, flags=OM | B.SFFT_FLAG_CONST_RATIO)
    assert oracle.rel_err(got["theta"], ref) <= 1e-9


@pytest.mark.parametrize("mode", [F64, F32C])
def test_output_mask_in_shared_template_batch(mode):
    """Two templates, three science epochs each: the owners correct Omega once;
    the sharing pairs' theta and D meet the oracle bar on their own triples."""
    ga = synth.template_group(51, 96, 3, w=3, dk=2, db=2, nstar=120)
    gb = synth.template_group(52, 80, 3, w=4, dk=1, db=1, nstar=90)
    pairs = [ga[0], gb[0], ga[1], ga[2], gb[1], gb[2]]
    tmpl_of = [0, 1, 0, 0, 1, 1]
    dt = torch.float64 if mode == F64 else torch.float32
    descs = [B.make_desc(p.sci.shape[0], p.sci.shape[1], p.w, p.dk, p.db, mode, flags=OM) for p in pairs]
    S = [torch.from_numpy(p.sci).to("cuda", dt) for p in pairs]
    R, M = [], []
    for i, p in enumerate(pairs):
        if tmpl_of[i] == i:
            R.append(torch.from_numpy(p.tmpl).to("cuda", dt))
            M.append(torch.from_numpy(p.mask).cuda())
        else:
            R.append(R[tmpl_of[i]])
            M.append(M[tmpl_of[i]])
    h = B.sfft_batch_plan_shared(descs, tmpl_of)
    try:
        C = [torch.zeros(B.sfft_num_coeffs(d), dtype=torch.float64, device="cuda") for d in descs]
        Dd = [torch.empty_like(s) for s in S]
        info = torch.full((len(pairs),), -7, dtype=torch.int32, device="cuda")
        B.sfft_batch_run(h, S, R, M, [s.stride(0) for s in S], C, Dd, info)
        torch.cuda.synchronize()
        assert info.cpu().tolist() == [0] * len(pairs)
        cast = np.float64 if mode == F64 else np.float32
        tol = 1e-9 if mode == F64 else 1e-5
        for i, p in enumerate(pairs):
            ref = oracle.fit_outmask(p.sci.astype(cast).astype(np.float64), p.tmpl.astype(cast).astype(np.float64),
                                     p.mask, p.w, p.dk, p.db, mode="fft")
            assert oracle.rel_err(C[i].cpu().numpy(), ref["theta"]) <= tol, i
            assert oracle.rel_err(Dd[i].cpu().numpy().astype(np.float64), ref["diff"]) <= tol, i
    finally:
        B.sfft_destroy(h)
