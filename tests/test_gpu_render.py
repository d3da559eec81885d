"""The GPU renderer of the warm-start frames (sfft_render_ws_frame) against the
host reference renderer (synth.render_ws_reference) on the same catalogue:
the same Philox4x32-10 noise, the same stars, background and mask.  Images to
1e-10 of their largest value (FP64 sums in another order, other pow/log
implementations), the mask exactly."""
import numpy as np
import pytest

import synth
from paper_2509_18544_amd import binding as B

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2509_18544_amd import learned as LN  # noqa: E402


@pytest.mark.parametrize("seed,n", [(11, 256), (12, 300), (13, 4088)])
def test_render_matches_reference(seed, n):
    _, small, arrays, start = LN.ws_frame_host((seed, n))
    r = LN.FrameRenderer(1, n)
    r.render(0, small, arrays, start)
    r.settle()
    cat = synth.ws_catalog(seed, n=n)
    sci, tmpl, mask = synth.render_ws_reference(cat)
    gs, gt, gm = r.S[0].cpu().numpy(), r.R[0].cpu().numpy(), r.M[0].cpu().numpy()
    es = np.abs(gs - sci).max() / np.abs(sci).max()
    et = np.abs(gt - tmpl).max() / np.abs(tmpl).max()
    print(f"n={n}: {arrays.shape[1]} stars, image errors {es:.2e} {et:.2e}, masked {int(mask.sum())}")
    assert es <= 1e-10 and et <= 1e-10
    assert np.array_equal(gm, mask)
