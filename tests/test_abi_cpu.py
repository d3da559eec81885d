"""Host-side checks of the C ABI library (no GPU needed, no compute calls).

The library must load, export every function include/sfft.h declares, and
validate descriptors on the host before touching any device.
"""
import ctypes
import os

import pytest

from paper_2509_18544_amd import binding as B

if not os.path.exists(B.LIB_PATH):  # pragma: no cover
    pytest.skip("libsfft.so not built", allow_module_level=True)


def test_exports_every_declared_symbol():
    syms = B.header_symbols()
    assert len(syms) >= 11
    raw = ctypes.CDLL(B.LIB_PATH)
    for s in syms:
        assert hasattr(raw, s), s


def test_num_coeffs_and_workspace():
    d = B.make_desc(4088, 4088, 9, 2, 2, B.SFFT_MODE_F32C)
    assert B.sfft_num_coeffs(d) == 19 * 19 * 6 + 6 == 2172
    ws32 = B.sfft_workspace_bytes(d)
    ws64 = B.sfft_workspace_bytes(B.make_desc(4088, 4088, 9, 2, 2, B.SFFT_MODE_F64))
    # spectra dominate: 13 planes of 4096 x 2049 complex
    assert 13 * 4096 * 2049 * 8 < ws32 < ws64
    assert B.sfft_num_coeffs(B.make_desc(256, 256, 5, 1, 1)) == 121 * 3 + 3
    # every assembly route is a valid descriptor; the workspace holds all their buffers
    sizes = {f: B.sfft_workspace_bytes(B.make_desc(1024, 1024, 9, 2, 2, B.SFFT_MODE_F32C, flags=f))
             for f in (B.SFFT_FLAG_ASSEMBLY_AUTO, B.SFFT_FLAG_ASSEMBLY_FFT, B.SFFT_FLAG_ASSEMBLY_DIRECT,
                       B.SFFT_FLAG_ASSEMBLY_MFMA)}
    assert len(set(sizes.values())) == 1
    # the constant photometric ratio adds its constraint columns (nK - 1 = 5 here, six vectors each)
    cr = B.make_desc(1024, 1024, 9, 2, 2, B.SFFT_MODE_F32C, flags=B.SFFT_FLAG_CONST_RATIO | B.SFFT_FLAG_ASSEMBLY_FFT)
    assert B.sfft_num_coeffs(cr) == 2172
    extra = B.sfft_workspace_bytes(cr) - sizes[B.SFFT_FLAG_ASSEMBLY_FFT]
    assert 6 * 5 * 2172 * 8 <= extra <= 6 * 5 * 2172 * 8 + 4096


@pytest.mark.parametrize("bad", [
    dict(ny=10, nx=10, w=3, dk=1, db=1),          # N < 4w + 2
    dict(ny=64, nx=64, w=-1, dk=1, db=1),
    dict(ny=64, nx=64, w=2, dk=-1, db=1),
    dict(ny=64, nx=64, w=2, dk=1, db=-2),
    dict(ny=5000, nx=64, w=2, dk=1, db=1),        # larger than 4096
    dict(ny=64, nx=64, w=2, dk=1, db=1, mode=7),
    dict(ny=64, nx=64, w=2, dk=1, db=1, flags=7),        # route bits plus an unknown bit
    dict(ny=64, nx=64, w=2, dk=1, db=1, flags=4),        # unknown flag bit
    dict(ny=64, nx=64, w=2, dk=1, db=1, flags=64),       # unknown flag bit above the output-mask flag
    dict(ny=64, nx=2048, w=2, dk=1, db=1, flags=2),      # direct sums limited to nx <= 1024
    dict(ny=64, nx=64, w=10, dk=1, db=1, flags=2),       # ... and to w <= 9
    dict(ny=4096, nx=4096, w=15, dk=3, db=3),     # more unknowns than the solver holds
])
def test_invalid_descriptors(bad):
    d = B.make_desc(**bad)
    with pytest.raises(B.SfftError) as e:
        B.sfft_num_coeffs(d)
    assert e.value.status == B.SFFT_EINVAL
    # sfft_plan rejects the descriptor before any device call
    h = ctypes.c_void_p(0)
    st = B.lib().sfft_plan(ctypes.byref(d), None, None, 0, ctypes.byref(h))
    assert st == B.SFFT_EINVAL and not h.value


def test_strerror_covers_codes():
    for code in (0, -1, -2, -3, -4, -5, -6, -7):
        assert B.strerror(code) and B.strerror(code) != "unknown status"
    assert B.strerror(123) == "unknown status"


def test_null_arguments():
    lib = B.lib()
    assert lib.sfft_num_coeffs(None, None) == B.SFFT_EINVAL
    assert lib.sfft_build_system(None, None, None, None, 0) == B.SFFT_EINVAL
    assert lib.sfft_solve(None, None, None) == B.SFFT_EINVAL
    assert lib.sfft_subtract(None, None, None, None, None, 0) == B.SFFT_EINVAL
    lib.sfft_destroy(None)


def test_noalloc_rejects_bad_arguments_before_any_device_call():
    """The no-allocation entry point checks its descriptor and pointers on the
    host first: these return SFFT_EINVAL with no GPU present (the fake
    pointers are never dereferenced)."""
    lib = B.lib()
    fake = ctypes.c_void_p(0x100000)
    good = B.make_desc(64, 64, 2, 1, 1, B.SFFT_MODE_F64)
    bad = B.make_desc(64, 64, -1, 1, 1, B.SFFT_MODE_F64)
    assert lib.sfft_subtract_pair_noalloc(None, None, fake, fake, None, 64, fake, fake, None) == B.SFFT_EINVAL
    assert lib.sfft_subtract_pair_noalloc(ctypes.byref(bad), None, fake, fake, None, 64, fake, fake,
                                          None) == B.SFFT_EINVAL
    for args in ((None, fake, fake, fake), (fake, None, fake, fake), (fake, fake, None, fake),
                 (fake, fake, fake, None)):
        sci, tmpl, coeffs, diff = args
        assert lib.sfft_subtract_pair_noalloc(ctypes.byref(good), None, sci, tmpl, None, 64, coeffs, diff,
                                              None) == B.SFFT_EINVAL
    # a row pitch shorter than the frame
    assert lib.sfft_subtract_pair_noalloc(ctypes.byref(good), None, fake, fake, None, 63, fake, fake,
                                          None) == B.SFFT_EINVAL


@pytest.mark.parametrize("dims,nl,max_batch", [
    ([10, 0, 5], 2, 4),            # zero width
    ([10, 9000, 5], 2, 4),         # wider than the kernels take
    ([10, 5], 0, 4),               # no layer
    ([10, 5], 1, 0),               # empty batch
])
def test_mlp_create_rejects_bad_shapes(dims, nl, max_batch):
    arr = (ctypes.c_int32 * len(dims))(*dims)
    h = ctypes.c_void_p(0)
    st = B.lib().sfft_mlp_create(arr, nl, max_batch, None, ctypes.byref(h))
    assert st == B.SFFT_EINVAL and not h.value


def test_caller_workspace_too_small_is_enomem():
    """sfft_plan with a caller workspace smaller than sfft_workspace_bytes returns
    SFFT_ENOMEM before touching the device (the pointer is never dereferenced)."""
    d = B.make_desc(256, 256, 5, 1, 1, B.SFFT_MODE_F32C)
    need = B.sfft_workspace_bytes(d)
    h = ctypes.c_void_p(0)
    fake = ctypes.c_void_p(0x100000)
    for have in (0, 1, need - 1):
        st = B.lib().sfft_plan(ctypes.byref(d), None, fake, have, ctypes.byref(h))
        assert st == B.SFFT_ENOMEM and not h.value

    # a misaligned workspace is rejected first
    st = B.lib().sfft_plan(ctypes.byref(d), None, ctypes.c_void_p(0x100010), need, ctypes.byref(h))
    assert st == B.SFFT_EINVAL and not h.value


def test_align_argument_checks():
    lib = B.lib()
    m = B.make_map([0.0, 1.0, 0.0], [0.0, 0.0, 1.0])
    P = ctypes.c_void_p
    a, b = P(1 << 20), P(1 << 30)      # never dereferenced: every call below fails its checks first
    ok_args = lambda **k: dict(dict(map=ctypes.byref(m), mode=B.SFFT_MODE_F64, tmpl=a, nyt=64, nxt=64,  # noqa: E731
                                    ldt=64, out=b, ny=64, nx=64, ld=64), **k)

    def call(d):
        return lib.sfft_align_image(d["map"], d["mode"], None, d["tmpl"], None, d["nyt"], d["nxt"], d["ldt"],
                                    d["out"], b if d["out"] is not None else None, d["ny"], d["nx"], d["ld"])
    assert call(ok_args(map=None)) == B.SFFT_EINVAL
    assert call(ok_args(mode=5)) == B.SFFT_EINVAL
    assert call(ok_args(tmpl=None)) == B.SFFT_EINVAL
    assert call(ok_args(ldt=63)) == B.SFFT_EINVAL
    assert call(ok_args(ld=10)) == B.SFFT_EINVAL
    assert call(ok_args(ny=0)) == B.SFFT_EINVAL
    assert call(ok_args(nxt=70000, ldt=70000)) == B.SFFT_EINVAL
    assert call(ok_args(out=P((1 << 20) + 8 * 100))) == B.SFFT_EINVAL      # output overlaps the template
    bad = B.make_map([0.0, 1.0, 0.0], [0.0, 0.0, 1.0])
    bad.deg = 4
    assert call(ok_args(map=ctypes.byref(bad))) == B.SFFT_EINVAL
    assert lib.sfft_align_psf(ctypes.byref(m), 0.0, 0.0, None, a, 32, b, 10) == B.SFFT_EINVAL
    assert lib.sfft_align_psf(ctypes.byref(m), 0.0, 0.0, None, a, 10, b, -1) == B.SFFT_EINVAL
    assert lib.sfft_align_psf(ctypes.byref(m), 0.0, 0.0, None, None, 10, b, 10) == B.SFFT_EINVAL
    with pytest.raises(KeyError):
        B.make_map([0.0, 1.0], [0.0, 1.0])


@pytest.mark.parametrize("tmpl_of,descs_same", [
    ([1, 1], True),        # a pair may only share an earlier pair's template
    ([0, 2, 0], True),     # ... not a later one
    ([0, 0, 1], True),     # the owner must use its own template (tmpl_of[o] == o)
    ([-1, 0], True),
    ([0, 0], False),       # a sharing pair needs the owner's descriptor
])
def test_shared_batch_plan_rejects_bad_tables(tmpl_of, descs_same):
    d0 = B.make_desc(64, 64, 2, 1, 1, B.SFFT_MODE_F32C)
    d1 = d0 if descs_same else B.make_desc(64, 64, 3, 1, 1, B.SFFT_MODE_F32C)
    descs = [d0] + [d1] * (len(tmpl_of) - 1)
    with pytest.raises(B.SfftError) as e:
        B.sfft_batch_plan_shared(descs, tmpl_of, stream=0)
    assert e.value.status == B.SFFT_EINVAL
