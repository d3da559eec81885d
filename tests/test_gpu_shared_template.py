"""Batches whose science images share a template and mask (S x T pairing).

The normal matrix depends only on the template and the mask, so a pair that
shares them forms only its right-hand side and is solved with the owner's
factor.  Every pair must meet the oracle bar on its own (science, template,
mask) triple, agree with the unshared batch up to rounding (the shared pair's
correlation sums are grouped differently), report its owner's outcome, and
replay bitwise from a captured graph.
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

F64, F32C = B.SFFT_MODE_F64, B.SFFT_MODE_F32C


def _workload():
    """Two templates of different shapes, interleaved, plus a pair on its own:
    pairs 0, 2, 4 share template A (owner 0), pairs 1, 3 template B (owner 1)."""
    ga = synth.template_group(31, 96, 3, w=3, dk=2, db=2, nstar=120)
    gb = synth.template_group(32, 128, 2, w=5, dk=1, db=1, nstar=200)
    lone = synth.random_pair(33, 80, 72, 2, 1, 2, mask_frac=0.05)
    pairs = [ga[0], gb[0], ga[1], gb[1], ga[2], lone]
    tmpl_of = [0, 1, 0, 1, 0, 5]
    return pairs, tmpl_of


def _buffers(pairs, tmpl_of, dt):
    """Device buffers; a sharing pair is handed its owner's template and mask tensors."""
    S = [torch.from_numpy(p.sci).to("cuda", dt) for p in pairs]
    R, M = [], []
    for i, p in enumerate(pairs):
        o = tmpl_of[i]
        if o == i:
            R.append(torch.from_numpy(p.tmpl).to("cuda", dt))
            M.append(torch.from_numpy(p.mask).cuda())
        else:
            R.append(R[o])
            M.append(M[o])
    return S, R, M


def _run(h, S, R, M, descs):
    C = [torch.zeros(B.sfft_num_coeffs(d), dtype=torch.float64, device="cuda") for d in descs]
    Dd = [torch.empty_like(s) for s in S]
    info = torch.full((len(S),), -7, dtype=torch.int32, device="cuda")
    B.sfft_batch_run(h, S, R, M, [s.stride(0) for s in S], C, Dd, info)
    torch.cuda.synchronize()
    return [c.cpu().numpy() for c in C], [d.cpu().numpy().astype(np.float64) for d in Dd], info.cpu().tolist()


@pytest.mark.parametrize("mode", [F64, F32C])
def test_shared_template_batch_matches_oracle_and_unshared(mode):
    pairs, tmpl_of = _workload()
    dt = torch.float64 if mode == F64 else torch.float32
    descs = [B.make_desc(p.sci.shape[0], p.sci.shape[1], p.w, p.dk, p.db, mode) for p in pairs]
    S, R, M = _buffers(pairs, tmpl_of, dt)
    hs = B.sfft_batch_plan_shared(descs, tmpl_of)
    hu = B.sfft_batch_plan(descs)
    try:
        Cs, Ds, infs = _run(hs, S, R, M, descs)
        Cu, Du, infu = _run(hu, S, R, M, descs)
        assert B.sfft_status(hs)[0] == B.SFFT_OK
        assert infs == [0] * len(pairs) and infu == [0] * len(pairs)
        cast = np.float64 if mode == F64 else np.float32
        tol = 1e-9 if mode == F64 else 1e-5
        agree = 1e-12 if mode == F64 else 1e-6
        for i, p in enumerate(pairs):
            ref = oracle.fit(p.sci.astype(cast).astype(np.float64), p.tmpl.astype(cast).astype(np.float64),
                             p.mask, p.w, p.dk, p.db)
            et, ed = oracle.rel_err(Cs[i], ref["theta"]), oracle.rel_err(Ds[i], ref["diff"])
            assert et <= tol and ed <= tol, (i, et, ed)
            assert oracle.rel_err(Cs[i], Cu[i]) <= agree, i
            assert oracle.rel_err(Ds[i], Du[i]) <= agree, i
            if tmpl_of[i] == i:
                # an owner runs exactly the unshared schedule
                np.testing.assert_array_equal(Cs[i], Cu[i])
                np.testing.assert_array_equal(Ds[i], Du[i])
    finally:
        B.sfft_destroy(hs)
        B.sfft_destroy(hu)


def test_sharing_pair_reports_its_owners_failed_factor():
    """A fully masked template (not positive definite) fails its owner and every
    pair that shares it; the other template's pairs are untouched."""
    pairs, tmpl_of = _workload()
    pairs = pairs[:4]
    tmpl_of = tmpl_of[:4]
    bad_mask = np.ones_like(pairs[0].mask)
    for i in (0, 2):
        pairs[i] = synth.Pair(pairs[i].sci, pairs[i].tmpl, bad_mask, pairs[i].w, pairs[i].dk, pairs[i].db, {})
    descs = [B.make_desc(p.sci.shape[0], p.sci.shape[1], p.w, p.dk, p.db) for p in pairs]
    S, R, M = _buffers(pairs, tmpl_of, torch.float64)
    h = B.sfft_batch_plan_shared(descs, tmpl_of)
    try:
        C, Dd, info = _run(h, S, R, M, descs)
        assert B.sfft_status(h)[0] == B.SFFT_ENOTSPD
        assert info[0] > 0 and info[2] == info[0] and info[1] == 0 and info[3] == 0
        assert np.all(C[0] == 0) and np.all(C[2] == 0)
        for i in (1, 3):
            p = pairs[i]
            ref = oracle.fit(p.sci, p.tmpl, p.mask, p.w, p.dk, p.db)
            assert oracle.rel_err(C[i], ref["theta"]) <= 1e-9
    finally:
        B.sfft_destroy(h)


def test_sharing_pair_must_be_given_the_owners_template():
    pairs, tmpl_of = _workload()
    descs = [B.make_desc(p.sci.shape[0], p.sci.shape[1], p.w, p.dk, p.db) for p in pairs]
    S, R, M = _buffers(pairs, tmpl_of, torch.float64)
    h = B.sfft_batch_plan_shared(descs, tmpl_of)
    try:
        C = [torch.zeros(B.sfft_num_coeffs(d), dtype=torch.float64, device="cuda") for d in descs]
        Dd = [torch.empty_like(s) for s in S]
        ld = [s.stride(0) for s in S]
        for swap in ("tmpl", "mask"):
            R2, M2 = list(R), list(M)
            if swap == "tmpl":
                R2[2] = R[0].clone()          # equal values, another buffer
            else:
                M2[4] = M[0].clone()
            with pytest.raises(B.SfftError) as e:
                B.sfft_batch_run(h, S, R2, M2, ld, C, Dd)
            assert e.value.status == B.SFFT_EINVAL
    finally:
        B.sfft_destroy(h)


@pytest.mark.parametrize("mode", [F64, F32C])
def test_shared_template_graph_replays_equal_eager(mode):
    pairs, tmpl_of = _workload()
    dt = torch.float64 if mode == F64 else torch.float32
    descs = [B.make_desc(p.sci.shape[0], p.sci.shape[1], p.w, p.dk, p.db, mode) for p in pairs]
    stream = torch.cuda.Stream()
    h = B.sfft_batch_plan_shared(descs, tmpl_of, stream)
    try:
        with torch.cuda.stream(stream):
            S, R, M = _buffers(pairs, tmpl_of, dt)
            ld = [s.stride(0) for s in S]
            new_c = lambda: [torch.zeros(B.sfft_num_coeffs(d), dtype=torch.float64, device="cuda")  # noqa: E731
                             for d in descs]
            Ce, Cg = new_c(), new_c()
            De, Dg = [torch.empty_like(s) for s in S], [torch.empty_like(s) for s in S]
            ie = torch.zeros(len(pairs), dtype=torch.int32, device="cuda")
            ig = torch.full_like(ie, -7)
        stream.synchronize()
        B.sfft_batch_run(h, S, R, M, ld, Ce, De, ie)
        stream.synchronize()
        B.sfft_batch_capture(h, S, R, M, ld, Cg, Dg, ig)
        stream.synchronize()
        for rep in range(3):
            with torch.cuda.stream(stream):
                for t in Cg + Dg:
                    t.fill_(float("nan"))
                ig.fill_(-7)
            B.sfft_batch_launch(h)
            stream.synchronize()
            assert ig.cpu().tolist() == [0] * len(pairs), rep
            for i in range(len(pairs)):
                np.testing.assert_array_equal(Cg[i].cpu().numpy(), Ce[i].cpu().numpy())
                np.testing.assert_array_equal(Dg[i].cpu().numpy(), De[i].cpu().numpy())
            B.sfft_batch_run(h, S, R, M, ld, Ce, De, ie)
            stream.synchronize()
    finally:
        B.sfft_destroy(h)


@pytest.mark.parametrize("mode", [F64, F32C])
def test_shared_template_wide_kernel(mode):
    """w = 10: the sharing pairs' template-science windows have 21 lag rows,
    more than a narrow correlation item takes, so their right-hand-side-only
    plans use the wide items; the pairs still meet the oracle bar and agree
    with the unshared batch."""
    pairs = synth.template_group(34, 112, 3, w=10, dk=1, db=1, nstar=140)
    tmpl_of = [0, 0, 0]
    dt = torch.float64 if mode == F64 else torch.float32
    descs = [B.make_desc(p.sci.shape[0], p.sci.shape[1], p.w, p.dk, p.db, mode) for p in pairs]
    S, R, M = _buffers(pairs, tmpl_of, dt)
    hs = B.sfft_batch_plan_shared(descs, tmpl_of)
    hu = B.sfft_batch_plan(descs)
    try:
        Cs, Ds, infs = _run(hs, S, R, M, descs)
        Cu, Du, infu = _run(hu, S, R, M, descs)
        assert infs == [0] * len(pairs) and infu == [0] * len(pairs)
        cast = np.float64 if mode == F64 else np.float32
        tol = 1e-9 if mode == F64 else 1e-5
        agree = 1e-12 if mode == F64 else 1e-6
        for i, p in enumerate(pairs):
            ref = oracle.fit(p.sci.astype(cast).astype(np.float64), p.tmpl.astype(cast).astype(np.float64),
                             p.mask, p.w, p.dk, p.db)
            assert oracle.rel_err(Cs[i], ref["theta"]) <= tol, i
            assert oracle.rel_err(Ds[i], ref["diff"]) <= tol, i
            assert oracle.rel_err(Cs[i], Cu[i]) <= agree, i
    finally:
        B.sfft_destroy(hs)
        B.sfft_destroy(hu)
