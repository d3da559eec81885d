"""Pins of the warm-start frame recipe's host side (synth): the counter-based
noise generator against the published Philox4x32-10 known-answer vectors
(Salmon et al., SC 2011, Random123 distribution), the normals' moments, and the
reference renderer's noise-free content (flux of a star fully inside the frame,
the background polynomial, the mask disks)."""
import numpy as np

import synth


def test_philox4x32_10_known_answers():
    cases = [
        ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
        ((0xFFFFFFFF,) * 4, (0xFFFFFFFF, 0xFFFFFFFF), (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
        ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
         (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
    ]
    for ctr, key, want in cases:
        got = synth.philox4x32(*[[c] for c in ctr], *key)
        assert tuple(int(g[0]) for g in got) == want


def test_philox_normals_moments():
    z1, z2 = synth.philox_normals(np.arange(400000, dtype=np.uint64), 1, 12345)
    for z in (z1, z2):
        assert abs(z.mean()) < 0.006 and abs(z.var() - 1.0) < 0.01
    assert abs(np.mean(z1 * z2)) < 0.006
    # another stream or seed gives different numbers; the same ones repeat
    a, _ = synth.philox_normals(np.arange(10, dtype=np.uint64), 0, 12345)
    b, _ = synth.philox_normals(np.arange(10, dtype=np.uint64), 1, 12345)
    c, _ = synth.philox_normals(np.arange(10, dtype=np.uint64), 0, 12345)
    assert not np.allclose(a, b) and np.array_equal(a, c)


def test_reference_renderer_content():
    cat = synth.ws_catalog(7, n=128)
    # one bright star at the centre only, no background, to read the content back
    for k in ("xs", "ys", "flux", "fw_s", "fw_t", "mask_r"):
        cat[k] = cat[k][:1].copy()
    cat["xs"][0], cat["ys"][0], cat["flux"][0] = 63.3, 64.6, 2.0e6
    cat["mask_r"][0] = 6.0
    cat["bc"] = np.zeros(6)
    sci, tmpl, mask = synth.render_ws_reference(cat)
    # noise-free part: the star's flux (its 25 x 25 stamp is inside the frame)
    assert abs(tmpl.sum() - 2.0e6) < 6 * np.sqrt(128 * 128 * (1000.0 + 64.0) + 2.0e6)
    yy, xx = np.mgrid[0:128, 0:128]
    assert np.array_equal(mask.astype(bool), (xx - 63.3) ** 2 + (yy - 64.6) ** 2 <= 36.0)
    assert np.unravel_index(np.argmax(sci), sci.shape) in ((64, 63), (65, 63))
