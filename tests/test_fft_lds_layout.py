"""The padded LDS index algebra the transform kernels rely on (host check).

The in-LDS accessors of the radix passes place element i0 + c of row b at
lds_pad(b N + i0) + pad_off(c), with lds_pad(i) = i + i/16 and pad_off(c) =
c + c/16, instead of lds_pad(b N + i0 + c).  That is exact only because, in
every pass, c either is a multiple of 16 or keeps i0 + c inside the
16-element group of i0.  This enumerates every pass shape the kernels
instantiate (transform lengths 2^4 .. 2^12, later passes of radix 8 or 16,
the first pass taking the remainder) for the loads (i0 = j < M, c = r M), the
stores (i0 = (j - k) R + k, c = r Ns) and the column pass's residue-major
store of its last pass (slot i0 * 16 + r), and checks the identity element by
element.  No GPU and no oracle are involved.
"""
import pytest


def lds_pad(i):
    return i + (i >> 4)


def pad_off(c):
    return c + (c >> 4)


def passes(lgn, lgm):
    lgr0 = (lgn % lgm) or lgm
    out = [(lgr0, 0)]
    ns = lgr0
    while ns < lgn:
        out.append((lgm, ns))
        ns += lgm
    return out


@pytest.mark.parametrize("lgm", [3, 4])
@pytest.mark.parametrize("lgn", list(range(4, 13)))
def test_split_padded_offsets_are_exact(lgn, lgm):
    n = 1 << lgn
    for lgr, lgns in passes(lgn, lgm):
        r_ = 1 << lgr
        m = n >> lgr
        ns = 1 << lgns
        for b in range(3):
            for j in range(m):
                k = j & (ns - 1)
                base = ((j - k) << lgr) + k
                for r in range(r_):
                    assert lds_pad(b * n + j + r * m) == lds_pad(b * n + j) + pad_off(r * m)
                    assert lds_pad(b * n + base + r * ns) == lds_pad(b * n + base) + pad_off(r * ns)


@pytest.mark.parametrize("lgpy", list(range(6, 13)))
def test_column_residue_store(lgpy):
    # last column pass: radix 16, span P1 = Py / 16; X(ky), ky = i0 + r P1,
    # goes to slot (ky mod P1) * 16 + ky / P1 = i0 * 16 + r
    py = 1 << lgpy
    p1 = py >> 4
    lgp1 = lgpy - 4
    for kb in range(2):
        for i0 in range(p1):
            for r in range(16):
                ky = i0 + r * p1
                slot = ((ky & (p1 - 1)) << 4) + (ky >> lgp1)
                assert slot == i0 * 16 + r
                assert lds_pad(kb * py + slot) == lds_pad(kb * py + (i0 << 4)) + ((r * p1) >> lgp1)


def test_passes_tile_every_length():
    for lgm in (3, 4):
        for lgn in range(4, 13):
            ps = passes(lgn, lgm)
            assert sum(lgr for lgr, _ in ps) == lgn
            assert all(lgr == lgm for lgr, _ in ps[1:])


def test_corr_staging_plane_index_is_exact():
    """The correlation kernel's staging finds the plane of staged element e as
    the FP32 truncation of (e + 1/2) / npr instead of an integer division; it
    must equal floor(e / npr) for every chunk width (npr = 8 residues' pairs,
    up to 8 x 256) and every element of up to 62 staged planes."""
    import numpy as np
    for npr in range(8, 2049, 8):
        e = np.arange(0, 62 * npr, dtype=np.int64)
        inv = np.float32(1.0) / np.float32(npr)
        q = ((e.astype(np.float32) + np.float32(0.5)) * inv).astype(np.int32)
        assert np.array_equal(q, e // npr), npr
