"""Batched uneven cutouts (the S x T workload: N in {512, 1024, 2048},
w in 5..9, DK in {1, 2}, DB = DK) in one sfft_batch_run, FP32C and FP64,
every pair checked against the CPU FP64 oracle on the same inputs."""
import numpy as np
import pytest

import oracle
import synth
from paper_2509_18544_amd import binding as B

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

PICK = [2, 3, 6, 8, 10, 11, 4]      # 512/1024 cutouts of both degrees and one 2048, DK = 1


@pytest.fixture(scope="module")
def c4_pairs():
    descs = synth.batch_c4_descriptors()
    return [synth.pair_c4(descs[i]) for i in PICK]


@pytest.mark.parametrize("mode", [B.SFFT_MODE_F32C, B.SFFT_MODE_F64])
def test_c4_batch_against_oracle(c4_pairs, mode):
    pairs = c4_pairs
    dt = torch.float64 if mode == B.SFFT_MODE_F64 else torch.float32
    cast = np.float64 if mode == B.SFFT_MODE_F64 else np.float32
    descs = [B.make_desc(p.sci.shape[0], p.sci.shape[1], p.w, p.dk, p.db, mode) for p in pairs]
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
            s_in = p.sci.astype(cast).astype(np.float64)
            r_in = p.tmpl.astype(cast).astype(np.float64)
            ref = oracle.fit(s_in, r_in, p.mask, p.w, p.dk, p.db, mode="fft")
            et = oracle.rel_err(C[i].cpu().numpy(), ref["theta"])
            ed = oracle.rel_err(Dd[i].cpu().numpy().astype(np.float64), ref["diff"])
            print(f"pair {PICK[i]} N={p.sci.shape[0]} w={p.w} DK={p.dk}: e_theta={et:.2e} e_D={ed:.2e}")
            assert et <= tol and ed <= tol
    finally:
        B.sfft_destroy(h)
