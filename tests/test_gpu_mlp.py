"""The warm-start network's HIP kernels (include/sfft_mlp.h) against the
FP64 network reference: FP32 forward and gradients within 1e-4 (relative to
the largest reference magnitude), MSE and Adam within FP32 rounding, BF16
inference within 2e-2 (norm-wise), at ragged sizes that span several 64 x 64
tiles and at the full 2180-512-512-512-2166 shape."""
import numpy as np
import pytest

from oracle import mlp_oracle as M
from paper_2509_18544_amd import binding as B

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

SMALL = [70, 96, 33, 129]
FULL = [2180, 512, 512, 512, 2166]


def _dev(a, dt=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dt)


def _setup(dims, batch, seed):
    rng = np.random.default_rng(seed)
    p = M.init_params(dims, seed)
    # non-zero biases so the bias paths are exercised
    off = 0
    for i in range(len(dims) - 1):
        off += dims[i] * dims[i + 1]
        p[off:off + dims[i + 1]] = rng.normal(0, 0.1, dims[i + 1])
        off += dims[i + 1]
    p = p.astype(np.float32).astype(np.float64)      # the GPU sees FP32 parameters
    x = rng.normal(0, 1, (batch, dims[0])).astype(np.float32).astype(np.float64)
    t = rng.normal(0, 1, (batch, dims[-1])).astype(np.float32).astype(np.float64)
    return p, x, t


def _maxrel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.mark.parametrize("dims,batch", [(SMALL, 37), (SMALL, 1), (FULL, 256)])
def test_forward_backward_mse_against_oracle(dims, batch):
    p, x, t = _setup(dims, batch, 7)
    h = B.sfft_mlp_create(dims, max(batch, 64))
    try:
        assert B.sfft_mlp_param_count(h) == M.param_count(dims) == p.size
        P, X, T = _dev(p), _dev(x), _dev(t)
        Y = torch.empty(batch, dims[-1], device="cuda")
        B.sfft_mlp_forward(h, P, X, batch, Y)
        dY = torch.empty_like(Y)
        loss = torch.zeros(1, dtype=torch.float64, device="cuda")
        B.sfft_mlp_mse(h, Y, T, batch, dY, loss)
        G = torch.full_like(P, float("nan"))
        B.sfft_mlp_backward(h, P, X, dY, batch, G)
        torch.cuda.synchronize()

        y_ref, hs = M.forward(p, dims, x)
        l_ref, dy_ref = M.mse(y_ref, t)
        g_ref, _ = M.backward(p, dims, hs, dy_ref)
        ey = _maxrel(Y.cpu().double().numpy(), y_ref)
        el = abs(loss.item() - l_ref) / l_ref
        edy = _maxrel(dY.cpu().double().numpy(), dy_ref)
        g = G.cpu().double().numpy()
        assert np.all(np.isfinite(g))
        print(f"dims={dims} batch={batch}: forward {ey:.2e} loss {el:.2e} dy {edy:.2e}")
        assert ey <= 1e-4 and el <= 1e-4 and edy <= 1e-4
        for (gw, gb), (rw, rb) in zip(M.unpack(g, dims), M.unpack(g_ref, dims)):
            ew, eb = _maxrel(gw, rw), _maxrel(gb, rb)
            print(f"  layer grads: W {ew:.2e} b {eb:.2e}")
            assert ew <= 1e-4 and eb <= 1e-4
    finally:
        B.sfft_mlp_destroy(h)


def test_adam_steps_against_oracle():
    dims = SMALL
    rng = np.random.default_rng(3)
    n = M.param_count(dims)
    p = rng.normal(0, 1, n).astype(np.float32).astype(np.float64)
    h = B.sfft_mlp_create(dims, 8)
    try:
        P = _dev(p)
        M1 = torch.zeros_like(P)
        M2 = torch.zeros_like(P)
        m, v, pr = np.zeros(n), np.zeros(n), p.copy()
        for step in range(1, 4):
            g = rng.normal(0, 1, n).astype(np.float32).astype(np.float64)
            B.sfft_mlp_adam_step(h, P, _dev(g), M1, M2, step, lr=1e-2, b1=0.9, b2=0.999, eps=1e-8)
            # the ABI takes FP32 hyperparameters: the oracle gets the same rounded values
            f = lambda v: float(np.float32(v))  # noqa: E731
            pr, m, v = M.adam_step(pr, g, m, v, step, lr=f(1e-2), b1=f(0.9), b2=f(0.999), eps=f(1e-8))
        torch.cuda.synchronize()
        assert _maxrel(P.cpu().double().numpy() - p, pr - p) <= 1e-4
        assert _maxrel(M1.cpu().double().numpy(), m) <= 1e-5
        assert _maxrel(M2.cpu().double().numpy(), v) <= 1e-5
    finally:
        B.sfft_mlp_destroy(h)


@pytest.mark.parametrize("dims,batch", [(SMALL, 37), (FULL, 128)])
def test_bf16_inference_against_oracle(dims, batch):
    p, x, _ = _setup(dims, batch, 11)
    rng = np.random.default_rng(12)
    scale = rng.uniform(0.5, 2.0, dims[-1])
    shift = rng.normal(0, 1, dims[-1])
    h = B.sfft_mlp_create(dims, batch)
    try:
        P, X = _dev(p), _dev(x)
        ld = dims[-1] + 5
        TH = torch.full((batch, ld), float("nan"), dtype=torch.float64, device="cuda")
        B.sfft_mlp_set_weights_bf16(h, P)
        B.sfft_mlp_infer(h, X, batch, _dev(scale, torch.float64), _dev(shift, torch.float64), TH, ld)
        torch.cuda.synchronize()
        th = TH.cpu().numpy()
        assert np.all(np.isnan(th[:, dims[-1]:]))       # the row pitch is respected
        y_ref, _ = M.forward(p, dims, x)
        ref = y_ref * scale + shift
        e = np.linalg.norm(th[:, :dims[-1]] - ref) / np.linalg.norm(ref)
        e0 = np.linalg.norm((th[:, :dims[-1]] - shift) / scale - y_ref) / np.linalg.norm(y_ref)
        print(f"dims={dims}: BF16 inference rel err {e:.2e} (network output {e0:.2e})")
        assert e0 <= 2e-2 and e <= 2e-2
    finally:
        B.sfft_mlp_destroy(h)


def test_call_order_and_arguments():
    h = B.sfft_mlp_create(SMALL, 16)
    try:
        n = B.sfft_mlp_param_count(h)
        P = torch.zeros(n, device="cuda")
        X = torch.zeros(4, SMALL[0], device="cuda")
        dY = torch.zeros(4, SMALL[-1], device="cuda")
        G = torch.zeros_like(P)
        with pytest.raises(B.SfftError) as e:
            B.sfft_mlp_backward(h, P, X, dY, 4, G)          # no forward yet
        assert e.value.status == B.SFFT_ESTATE
        TH = torch.zeros(4, SMALL[-1], dtype=torch.float64, device="cuda")
        with pytest.raises(B.SfftError) as e:
            B.sfft_mlp_infer(h, X, 4, None, None, TH, SMALL[-1])   # no BF16 weights yet
        assert e.value.status == B.SFFT_ESTATE
        Y = torch.zeros(4, SMALL[-1], device="cuda")
        B.sfft_mlp_forward(h, P, X, 4, Y)
        with pytest.raises(B.SfftError) as e:
            B.sfft_mlp_backward(h, P, X, dY, 3, G)          # batch differs from the forward's
        assert e.value.status == B.SFFT_ESTATE
        with pytest.raises(B.SfftError) as e:
            B.sfft_mlp_forward(h, P, X, 17, Y)              # above max_batch
        assert e.value.status == B.SFFT_EINVAL
        torch.cuda.synchronize()
    finally:
        B.sfft_mlp_destroy(h)
