"""The learned warm start on the GPU.

The network is trained by the library's own forward/backward/Adam kernels on
solutions the library itself computes: frames rendered on the GPU by
sfft_render_ws_frame (the warm-start recipe of synth.ws_catalog: Roman-like
star fields whose PSF varies with the focal-plane position, the seeing and
the Moffat exponent), solved in FP64 batches (w = 9, DK = DB = 2).  On
held-out frames it is compared with the method without it, i.e. the mean
kernel of the training set: coefficient error and quick-look difference-image
error against the full FP64 solve, the residual judge rho and the fallback
rate, and the per-pair times.  The gain bar asks for at least 64 % of the
kernels' spread about the mean kernel (e_net <= 0.6 e_mean, 2048^2 frames); a
network that explains 1 % of it gives e_net ~ 0.995 e_mean and fails.  The fallback policy
is checked to return exactly the plain solve when rho is above the threshold,
and exactly the completed guess when it is below."""
import json
import os

import numpy as np
import pytest

from paper_2509_18544_amd import binding as B
from paper_2509_18544_amd import learned as L

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

NK = L.DIMS[-1]


def test_trained_network_gains_over_the_mean_kernel(tmp_path):
    n = 2048
    feats, th, info = L.make_dataset_gpu(6144, seed0=700000, n=n)
    assert (info == 0).all()
    net = L.Net(L.DIMS, max_batch=128, seed=1)
    try:
        hist = net.train(feats, th[:, :NK], epochs=60, batch=128)
        rep = L.evaluate_gpu(net, 12, seed0=800000, n=n, base_mean=th.mean(axis=0))
        rep.update(loss_first=hist[0], loss_last=hist[-1])
        print(json.dumps(rep))
        assert hist[-1] < hist[0]
        assert rep["e_kernel_net"] <= 0.6 * rep["e_kernel_mean"]
        assert rep["e_diff_quicklook_net"] <= 0.5 * rep["e_diff_quicklook_mean"]
        assert rep["ms_quicklook"] < rep["ms_full"]
        assert 0.0 <= rep["fallback_rate"] <= 1.0
        # checkpoint round trip: same parameters, Adam state and predictions
        path = os.path.join(str(tmp_path), "net")
        net.save(path)
        net2 = L.Net.load(path, max_batch=64)
        try:
            assert torch.equal(net2.params, net.params) and torch.equal(net2.m2, net.m2)
            a = torch.zeros((4, NK), dtype=torch.float64, device="cuda")
            b = torch.zeros_like(a)
            net.predict(feats[:4], a, NK)
            net2.predict(feats[:4], b, NK)
            torch.cuda.synchronize()
            assert torch.equal(a, b)
        finally:
            net2.close()
    finally:
        net.close()


def test_policy_takes_the_guess_or_the_plain_solve():
    import synth
    p = synth.pair_ws(900001, n=256)
    f = L.pair_features(p)
    net = L.Net(L.DIMS, max_batch=8, seed=3)
    net.xs = L.Standardizer(np.zeros(L.DIMS[0]), np.ones(L.DIMS[0]))
    net.ys = L.Standardizer(np.zeros(NK), np.full(NK, 1e-3))
    S = torch.from_numpy(p.sci).cuda()
    R = torch.from_numpy(p.tmpl).cuda()
    M = torch.from_numpy(p.mask).cuda()
    plan = B.Plan(256, 256, p.w, p.dk, p.db)
    try:
        plan.build(S, R, M)
        c_ref, _ = plan.solve()
        d_ref = plan.subtract(S, R, c_ref)
        guess = L.WarmStart(net).coefficients(plan, f)
        d_guess = plan.subtract(S, R, guess)
        torch.cuda.synchronize()
        # an untrained network is far off: the plain solve is taken, bit for bit
        ws = L.WarmStart(net, tau=1e-5)
        c, d, rho, used = ws.subtract(plan, S, R, M, f)
        torch.cuda.synchronize()
        assert not used and rho > 1e-5 and ws.fallback_rate == 1.0
        assert torch.equal(c, c_ref) and torch.equal(d, d_ref)
        # with an unbounded threshold the completed guess is used as it is
        ws = L.WarmStart(net, tau=float("inf"))
        c, d, rho, used = ws.subtract(plan, S, R, M, f)
        torch.cuda.synchronize()
        assert used and ws.fallback_rate == 0.0
        assert torch.equal(c, guess) and torch.equal(d, d_guess)
    finally:
        plan.close()
        net.close()
