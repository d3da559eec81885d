"""Batched uneven cutouts (the S x T workload: N in {512, 1024, 2048},
w in 5..9, DK in {1, 2}, DB = DK).

* A subset in one eager sfft_batch_run, FP32C and FP64, every pair against the
  CPU FP64 oracle on the same inputs.
* All 128 pairs of the workload captured into one HIP graph (FP32C) and
  replayed: every replay equals the eager run bit for bit, every pair reports
  info = 0, and one pair of every (N, w, DK) combination present is checked
  against the oracle (relative 2-norm errors of theta and D <= 1e-5).
"""
import multiprocessing as mp
import os

import numpy as np
import pytest

import synth
from paper_2509_18544_amd import binding as B

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from gpu_util import oracle_reference, pin_worker  # noqa: E402

PICK = [2, 3, 6, 8, 10, 11, 4]      # 512/1024 cutouts of both degrees and one 2048, DK = 1


def _pool():
    """Host worker processes (spawned: this process already uses the GPU), one core each."""
    cores = sorted(os.sched_getaffinity(0))
    ctx = mp.get_context("spawn")
    return ctx.Pool(max(1, min(16, len(cores))), initializer=pin_worker, initargs=(cores, ctx.Value("i", 0)))


@pytest.fixture(scope="module")
def c4_all():
    descs = synth.batch_c4_descriptors()
    with _pool() as pool:
        pairs = pool.map(synth.pair_c4, descs)
    return descs, pairs


def _refs(pairs, idx, cast):
    with _pool() as pool:
        return pool.map(oracle_reference, [(pairs[i].sci, pairs[i].tmpl, pairs[i].mask, pairs[i].w,
                                            pairs[i].dk, pairs[i].db, cast) for i in idx])


@pytest.mark.parametrize("mode", [B.SFFT_MODE_F32C, B.SFFT_MODE_F64])
def test_c4_batch_against_oracle(c4_all, mode):
    pairs = [c4_all[1][i] for i in PICK]
    dt = torch.float64 if mode == B.SFFT_MODE_F64 else torch.float32
    cast = np.float64 if mode == B.SFFT_MODE_F64 else np.float32
    descs = [B.make_desc(p.sci.shape[0], p.sci.shape[1], p.w, p.dk, p.db, mode) for p in pairs]
    refs = _refs(pairs, range(len(pairs)), cast)
    h = B.sfft_batch_plan(descs)
    try:
        S = [torch.from_numpy(p.sci).to("cuda", dt) for p in pairs]
        R = [torch.from_numpy(p.tmpl).to("cuda", dt) for p in pairs]
        M = [torch.from_numpy(p.mask).cuda() for p in pairs]
        C = [torch.zeros(B.sfft_num_coeffs(d), dtype=torch.float64, device="cuda") for d in descs]
        Dd = [torch.empty_like(s) for s in S]
        info = torch.full((len(pairs),), -1, dtype=torch.int32, device="cuda")
        B.sfft_batch_run(h, S, R, M, [s.stride(0) for s in S], C, Dd, info)
        st, _, _ = B.sfft_status(h)
        assert st == B.SFFT_OK and info.cpu().tolist() == [0] * len(pairs)
        tol = 1e-9 if mode == B.SFFT_MODE_F64 else 1e-5
        for i, p in enumerate(pairs):
            th, dref = refs[i]
            et = np.linalg.norm(C[i].cpu().numpy() - th) / np.linalg.norm(th)
            ed = np.linalg.norm(Dd[i].cpu().numpy().astype(np.float64) - dref) / np.linalg.norm(dref)
            print(f"pair {PICK[i]} N={p.sci.shape[0]} w={p.w} DK={p.dk}: e_theta={et:.2e} e_D={ed:.2e}")
            assert et <= tol and ed <= tol
    finally:
        B.sfft_destroy(h)


@pytest.mark.timeout(900)
def test_c4_all_128_pairs_in_one_graph(c4_all):
    descs_c4, pairs = c4_all
    mode = B.SFFT_MODE_F32C
    print(f"C4: {len(pairs)} pairs, N = {sorted({p.sci.shape[0] for p in pairs})}", flush=True)
    descs = [B.make_desc(p.sci.shape[0], p.sci.shape[1], p.w, p.dk, p.db, mode) for p in pairs]
    stream = torch.cuda.Stream()
    h = B.sfft_batch_plan(descs, stream)
    try:
        with torch.cuda.stream(stream):
            S = [torch.from_numpy(p.sci).to("cuda", torch.float32) for p in pairs]
            R = [torch.from_numpy(p.tmpl).to("cuda", torch.float32) for p in pairs]
            M = [torch.from_numpy(p.mask).cuda() for p in pairs]
            C = [torch.zeros(B.sfft_num_coeffs(d), dtype=torch.float64, device="cuda") for d in descs]
            Dd = [torch.empty_like(s) for s in S]
            info = torch.full((len(pairs),), -1, dtype=torch.int32, device="cuda")
        lds = [s.stride(0) for s in S]
        stream.synchronize()
        B.sfft_batch_run(h, S, R, M, lds, C, Dd, info)
        st, _, _ = B.sfft_status(h)
        assert st == B.SFFT_OK and info.cpu().tolist() == [0] * len(pairs)
        eager = [(c.cpu().numpy(), d.cpu().numpy()) for c, d in zip(C, Dd)]
        B.sfft_batch_capture(h, S, R, M, lds, C, Dd, info)
        for rep in range(2):
            with torch.cuda.stream(stream):
                for c, d in zip(C, Dd):
                    c.fill_(float("nan"))
                    d.fill_(float("nan"))
                info.fill_(-1)
            B.sfft_batch_launch(h)
            stream.synchronize()
            assert info.cpu().tolist() == [0] * len(pairs)
            for i, (c, d) in enumerate(zip(C, Dd)):
                assert np.array_equal(c.cpu().numpy(), eager[i][0]), f"replay {rep}: pair {i} theta"
                assert np.array_equal(d.cpu().numpy(), eager[i][1]), f"replay {rep}: pair {i} D"
            print(f"replay {rep}: all {len(pairs)} pairs equal the eager run", flush=True)
    finally:
        B.sfft_destroy(h)
    # one pair of every (N, w, DK) combination present, against the oracle
    first = {}
    for i, d in enumerate(descs_c4):
        first.setdefault((d["n"], d["w"], d["dk"]), i)
    idx = sorted(first.values())
    refs = _refs(pairs, idx, np.float32)
    worst = (0.0, 0.0)
    for i, (th, dref) in zip(idx, refs):
        et = np.linalg.norm(eager[i][0] - th) / np.linalg.norm(th)
        ed = np.linalg.norm(eager[i][1].astype(np.float64) - dref) / np.linalg.norm(dref)
        worst = (max(worst[0], et), max(worst[1], ed))
        assert et <= 1e-5 and ed <= 1e-5, (i, descs_c4[i], et, ed)
    print(f"{len(idx)} (N, w, DK) combinations against the oracle: max e_theta={worst[0]:.2e} "
          f"max e_D={worst[1]:.2e}")
