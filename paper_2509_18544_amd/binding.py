"""ctypes binding of libsfft.so with the same names as the C ABI (include/sfft.h).

This module only marshals arguments: every step of the subtraction runs in
the HIP kernels of the library.  Device buffers are torch tensors on the GPU
(their data pointers are passed through); the HIP stream is torch's current
stream unless another is given.  If the library has not been built, loading
fails loudly -- there is no fallback of any kind.
"""
from __future__ import annotations

import ctypes
import glob
import os
import re

_HERE = os.path.dirname(os.path.abspath(__file__))
# always the in-tree build (python -m paper_2509_18544_amd.build); no override
LIB_PATH = os.path.join(_HERE, "_lib", "libsfft.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "sfft.h")

SFFT_OK = 0
SFFT_EINVAL = -1
SFFT_ENOMEM = -2
SFFT_EHIP = -3
SFFT_ENOTSPD = -4
SFFT_ESTATE = -5
SFFT_ENONFINITE = -6
SFFT_ETOOBIG = -7

SFFT_MODE_F64 = 0
SFFT_MODE_F32C = 1

SFFT_FLAG_ASSEMBLY_AUTO = 0
SFFT_FLAG_ASSEMBLY_FFT = 1
SFFT_FLAG_ASSEMBLY_DIRECT = 2
SFFT_FLAG_ASSEMBLY_MFMA = 3
SFFT_FLAG_CONST_RATIO = 16   # constant photometric ratio (spatial kernel sums vanish)
SFFT_FLAG_OUTPUT_MASK = 32   # least squares over the good output pixels only
ROUTES = ("fft", "direct", "mfma")


class SfftError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {strerror(status)} (status {status})")


class sfft_desc(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int32) for name in
                ("ny", "nx", "w", "dk", "db", "mode", "refine_steps", "flags")]


class sfft_ws_frame(ctypes.Structure):
    """One warm-start frame's catalogue (include/sfft_render.h); pointers are device addresses."""
    _fields_ = [("n", ctypes.c_int32), ("nstar", ctypes.c_int32), ("beta", ctypes.c_double),
                ("bc", ctypes.c_double * 6), ("noise_seed", ctypes.c_uint64),
                ("xs", ctypes.c_void_p), ("ys", ctypes.c_void_p), ("flux", ctypes.c_void_p),
                ("fw_s", ctypes.c_void_p), ("fw_t", ctypes.c_void_p), ("mask_r", ctypes.c_void_p),
                ("tile_start", ctypes.c_void_p)]


class sfft_pixel_map(ctypes.Structure):
    """Science-to-template pixel map (include/sfft_align.h): polynomial of degree deg in
    (x - x_ref, y - y_ref), monomials 1; u, v; u^2, uv, v^2; u^3, u^2 v, u v^2, v^3."""
    _fields_ = [("deg", ctypes.c_int32), ("x_ref", ctypes.c_double), ("y_ref", ctypes.c_double),
                ("cx", ctypes.c_double * 10), ("cy", ctypes.c_double * 10)]


def make_map(cx, cy, ref=(0.0, 0.0)) -> sfft_pixel_map:
    """A pixel map from coefficient lists of length 1, 3, 6 or 10."""
    deg = {1: 0, 3: 1, 6: 2, 10: 3}[len(cx)]
    if len(cy) != len(cx):
        raise ValueError("cx and cy need the same number of coefficients")
    m = sfft_pixel_map()
    m.deg = deg
    m.x_ref, m.y_ref = float(ref[0]), float(ref[1])
    for j in range(len(cx)):
        m.cx[j] = float(cx[j])
        m.cy[j] = float(cy[j])
    return m


_lib = None


def lib():
    """Load libsfft.so (once).  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build the HIP library first "
                           "(python -m paper_2509_18544_amd.build)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    D = ctypes.POINTER(sfft_desc)
    sig = {
        "sfft_num_coeffs": (ctypes.c_int, [D, ctypes.POINTER(i64)]),
        "sfft_workspace_bytes": (ctypes.c_int, [D, ctypes.POINTER(sz)]),
        "sfft_plan": (ctypes.c_int, [D, vp, vp, sz, ctypes.POINTER(vp)]),
        "sfft_build_system": (ctypes.c_int, [vp, vp, vp, vp, i64]),
        "sfft_get_system": (ctypes.c_int, [vp, vp, vp]),
        "sfft_solve": (ctypes.c_int, [vp, vp, vp]),
        "sfft_residual": (ctypes.c_int, [vp, vp, vp]),
        "sfft_fit_background": (ctypes.c_int, [vp, vp]),
        "sfft_subtract": (ctypes.c_int, [vp, vp, vp, vp, vp, i64]),
        "sfft_status": (ctypes.c_int, [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]),
        "sfft_timing_enable": (ctypes.c_int, [vp, ctypes.c_int]),
        "sfft_timing_read": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]),
        "sfft_batch_workspace_bytes": (ctypes.c_int, [D, i32, ctypes.POINTER(sz)]),
        "sfft_batch_plan": (ctypes.c_int, [D, i32, vp, ctypes.POINTER(vp)]),
        "sfft_batch_plan_shared": (ctypes.c_int, [D, ctypes.POINTER(i32), i32, vp, ctypes.POINTER(vp)]),
        "sfft_batch_run": (ctypes.c_int, [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                          ctypes.POINTER(i64), ctypes.POINTER(vp), ctypes.POINTER(vp), vp]),
        "sfft_batch_capture": (ctypes.c_int, [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                              ctypes.POINTER(i64), ctypes.POINTER(vp), ctypes.POINTER(vp), vp]),
        "sfft_batch_launch": (ctypes.c_int, [vp]),
        "sfft_autotune": (ctypes.c_int, [vp, vp, vp, vp, i64, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_float),
                                         i32, ctypes.POINTER(i32)]),
        "sfft_subtract_pair_noalloc": (ctypes.c_int, [D, vp, vp, vp, vp, i64, vp, vp, vp]),
        "sfft_apply_kernel": (ctypes.c_int, [vp, vp, vp, vp, i64]),
        "sfft_decorrelation_kernel": (ctypes.c_int, [vp, vp, vp, vp, i32, ctypes.c_double, ctypes.c_double, i32,
                                                     vp]),
        "sfft_autotune_route": (ctypes.c_int, [vp, vp, vp, vp, i64, ctypes.POINTER(ctypes.c_float),
                                               ctypes.POINTER(i32)]),
        "sfft_render_ws_frame": (ctypes.c_int, [ctypes.POINTER(sfft_ws_frame), vp, vp, vp, vp, i64, vp, vp]),
        "sfft_align_image": (ctypes.c_int, [ctypes.POINTER(sfft_pixel_map), i32, vp, vp, vp, i32, i32, i64, vp, vp,
                                            i32, i32, i64]),
        "sfft_align_psf": (ctypes.c_int, [ctypes.POINTER(sfft_pixel_map), ctypes.c_double, ctypes.c_double, vp, vp,
                                          i32, vp, i32]),
        "sfft_destroy": (None, [vp]),
        "sfft_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "sfft_mlp_create": (ctypes.c_int, [ctypes.POINTER(i32), i32, i32, vp, ctypes.POINTER(vp)]),
        "sfft_mlp_param_count": (ctypes.c_int, [vp, ctypes.POINTER(i64)]),
        "sfft_mlp_forward": (ctypes.c_int, [vp, vp, vp, i32, vp]),
        "sfft_mlp_backward": (ctypes.c_int, [vp, vp, vp, vp, i32, vp]),
        "sfft_mlp_mse": (ctypes.c_int, [vp, vp, vp, i32, vp, vp]),
        "sfft_mlp_adam_step": (ctypes.c_int, [vp, vp, vp, vp, vp, i32, ctypes.c_float, ctypes.c_float,
                                              ctypes.c_float, ctypes.c_float]),
        "sfft_mlp_set_weights_bf16": (ctypes.c_int, [vp, vp]),
        "sfft_mlp_infer": (ctypes.c_int, [vp, vp, i32, vp, vp, vp, i64]),
        "sfft_mlp_destroy": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def header_symbols(path: str = None):
    """Names of the functions declared in include/*.h (or in one header)."""
    paths = [path] if path else sorted(glob.glob(os.path.join(os.path.dirname(HEADER_PATH), "*.h")))
    text = "".join(open(p).read() for p in paths)
    return sorted(set(re.findall(r"\b(sfft_[a-z_0-9]+)\s*\(", text)))


def strerror(status: int) -> str:
    return lib().sfft_strerror(int(status)).decode()


def make_desc(ny, nx, w, dk, db, mode=SFFT_MODE_F64, refine_steps=-1, flags=0) -> sfft_desc:
    return sfft_desc(int(ny), int(nx), int(w), int(dk), int(db), int(mode), int(refine_steps), int(flags))


def _check(st, where):
    if st != SFFT_OK:
        raise SfftError(st, where)


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def sfft_num_coeffs(desc: sfft_desc) -> int:
    n = ctypes.c_int64(0)
    _check(lib().sfft_num_coeffs(ctypes.byref(desc), ctypes.byref(n)), "sfft_num_coeffs")
    return n.value


def sfft_workspace_bytes(desc: sfft_desc) -> int:
    b = ctypes.c_size_t(0)
    _check(lib().sfft_workspace_bytes(ctypes.byref(desc), ctypes.byref(b)), "sfft_workspace_bytes")
    return b.value


def sfft_plan(desc: sfft_desc, stream=None, workspace=None, workspace_bytes: int = 0):
    """Returns an opaque handle (int).  `stream`: torch.cuda.Stream, raw handle, or None."""
    h = ctypes.c_void_p(0)
    s = _stream_handle(stream)
    _check(lib().sfft_plan(ctypes.byref(desc), s, _ptr(workspace), int(workspace_bytes), ctypes.byref(h)),
           "sfft_plan")
    return h.value


def sfft_build_system(handle, sci, tmpl, mask, ld: int):
    _check(lib().sfft_build_system(handle, _ptr(sci), _ptr(tmpl), _ptr(mask), int(ld)), "sfft_build_system")


def sfft_get_system(handle, omega, rhs):
    _check(lib().sfft_get_system(handle, _ptr(omega), _ptr(rhs)), "sfft_get_system")


def sfft_solve(handle, coeffs, info):
    _check(lib().sfft_solve(handle, _ptr(coeffs), _ptr(info)), "sfft_solve")


def sfft_residual(handle, coeffs, rho):
    _check(lib().sfft_residual(handle, _ptr(coeffs), _ptr(rho)), "sfft_residual")


def sfft_fit_background(handle, coeffs):
    _check(lib().sfft_fit_background(handle, _ptr(coeffs)), "sfft_fit_background")


def sfft_subtract(handle, sci, tmpl, coeffs, diff, ld: int):
    _check(lib().sfft_subtract(handle, _ptr(sci), _ptr(tmpl), _ptr(coeffs), _ptr(diff), int(ld)),
           "sfft_subtract")


def sfft_apply_kernel(handle, img, kcoef, out, ld: int):
    _check(lib().sfft_apply_kernel(handle, _ptr(img), _ptr(kcoef), _ptr(out), int(ld)), "sfft_apply_kernel")


def sfft_decorrelation_kernel(handle, coeffs, psf_sci, psf_tmpl, s: int, sigma_sci: float, sigma_tmpl: float,
                              t: int, psi):
    _check(lib().sfft_decorrelation_kernel(handle, _ptr(coeffs), _ptr(psf_sci), _ptr(psf_tmpl), int(s),
                                           float(sigma_sci), float(sigma_tmpl), int(t), _ptr(psi)),
           "sfft_decorrelation_kernel")


def sfft_status(handle):
    """(status, info, nonfinite) after synchronising the plan's stream."""
    info = ctypes.c_int32(0)
    nf = ctypes.c_int32(0)
    st = lib().sfft_status(handle, ctypes.byref(info), ctypes.byref(nf))
    return st, info.value, nf.value


STAGES = ("moments", "row_fwd", "col_fwd", "corr", "row_win", "gather", "factor", "solve", "subtract", "outmask")


SFFT_TIMING_ALL = (1 << 9) - 1


def sfft_timing_enable(handle, stages=True):
    """stages: True (every stage), False (off), or an iterable of stage names."""
    if stages is True:
        mask = SFFT_TIMING_ALL
    elif stages is False or stages is None:
        mask = 0
    else:
        mask = 0
        for name in stages:
            mask |= 1 << STAGES.index(name)
    _check(lib().sfft_timing_enable(handle, int(mask)), "sfft_timing_enable")


def sfft_timing_read(handle):
    """{stage: (total_ms, count)} since the last read (synchronises the plan's stream)."""
    n = len(STAGES)
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_int64 * n)()
    _check(lib().sfft_timing_read(handle, ms, cnt), "sfft_timing_read")
    return {STAGES[i]: (ms[i], cnt[i]) for i in range(n)}


def _desc_array(descs):
    arr = (sfft_desc * len(descs))()
    for i, d in enumerate(descs):
        arr[i] = d
    return arr


def sfft_batch_workspace_bytes(descs) -> int:
    b = ctypes.c_size_t(0)
    _check(lib().sfft_batch_workspace_bytes(_desc_array(descs), len(descs), ctypes.byref(b)),
           "sfft_batch_workspace_bytes")
    return b.value


def sfft_batch_plan(descs, stream=None):
    h = ctypes.c_void_p(0)
    _check(lib().sfft_batch_plan(_desc_array(descs), len(descs), _stream_handle(stream), ctypes.byref(h)),
           "sfft_batch_plan")
    return h.value


def sfft_batch_plan_shared(descs, tmpl_of, stream=None):
    """tmpl_of[i]: the pair whose template and mask pair i uses (i, or an earlier owner)."""
    n = len(descs)
    h = ctypes.c_void_p(0)
    _check(lib().sfft_batch_plan_shared(_desc_array(descs), (ctypes.c_int32 * n)(*[int(v) for v in tmpl_of]), n,
                                        _stream_handle(stream), ctypes.byref(h)), "sfft_batch_plan_shared")
    return h.value


def sfft_batch_run(handle, sci, tmpl, mask, ld, coeffs, diff, info=None):
    """sci/tmpl/mask/coeffs/diff: lists of tensors (mask entries may be None); ld: list of ints."""
    n = len(sci)
    P = ctypes.c_void_p * n
    arr = lambda xs: P(*[_ptr(x) for x in xs])  # noqa: E731
    _check(lib().sfft_batch_run(handle, arr(sci), arr(tmpl), None if mask is None else arr(mask),
                                (ctypes.c_int64 * n)(*[int(v) for v in ld]), arr(coeffs), arr(diff), _ptr(info)),
           "sfft_batch_run")


def sfft_batch_capture(handle, sci, tmpl, mask, ld, coeffs, diff, info=None):
    """As sfft_batch_run, but captured into the handle's HIP graph (nothing runs)."""
    n = len(sci)
    P = ctypes.c_void_p * n
    arr = lambda xs: P(*[_ptr(x) for x in xs])  # noqa: E731
    _check(lib().sfft_batch_capture(handle, arr(sci), arr(tmpl), None if mask is None else arr(mask),
                                    (ctypes.c_int64 * n)(*[int(v) for v in ld]), arr(coeffs), arr(diff),
                                    _ptr(info)), "sfft_batch_capture")


def sfft_autotune(handle, sci, tmpl, mask, ld: int, cap: int = 16):
    """Tune the plan on these inputs; returns [(chunk, ms), ...] of the candidates timed."""
    c1 = (ctypes.c_int32 * max(cap, 1))()
    ms = (ctypes.c_float * max(cap, 1))()
    cnt = ctypes.c_int32(0)
    _check(lib().sfft_autotune(handle, _ptr(sci), _ptr(tmpl), _ptr(mask), int(ld), c1, ms, int(cap),
                               ctypes.byref(cnt)), "sfft_autotune")
    return [(int(c1[i]), float(ms[i])) for i in range(cnt.value)]


def sfft_autotune_route(handle, sci, tmpl, mask, ld: int):
    """Time the assembly with each route; returns ({route: ms or None}, route in use)."""
    ms = (ctypes.c_float * 3)()
    r = ctypes.c_int32(0)
    _check(lib().sfft_autotune_route(handle, _ptr(sci), _ptr(tmpl), _ptr(mask), int(ld), ms, ctypes.byref(r)),
           "sfft_autotune_route")
    return {ROUTES[i]: (None if ms[i] < 0 else float(ms[i])) for i in range(3)}, ROUTES[r.value - 1]


def sfft_render_ws_frame(frame: sfft_ws_frame, sci, tmpl, mask, ld: int, norm_scratch, overflow, stream=None):
    _check(lib().sfft_render_ws_frame(ctypes.byref(frame), _stream_handle(stream), _ptr(sci), _ptr(tmpl),
                                      _ptr(mask), int(ld), _ptr(norm_scratch), _ptr(overflow)),
           "sfft_render_ws_frame")


def sfft_align_image(pmap: sfft_pixel_map, mode: int, tmpl, tmpl_mask, out, out_mask, stream=None):
    """Resample the template (and mask) onto the science grid of `out` (device tensors, row pitch = stride(0))."""
    nyt, nxt = tmpl.shape
    ny, nx = out.shape
    if out_mask.shape != out.shape or out_mask.stride(0) != out.stride(0):
        raise ValueError("out_mask must have the shape and row pitch of out")
    if tmpl_mask is not None and (tmpl_mask.shape != tmpl.shape or tmpl_mask.stride(0) != tmpl.stride(0)):
        raise ValueError("tmpl_mask must have the shape and row pitch of tmpl")
    _check(lib().sfft_align_image(ctypes.byref(pmap), int(mode), _stream_handle(stream), _ptr(tmpl), _ptr(tmpl_mask),
                                  int(nyt), int(nxt), int(tmpl.stride(0)), _ptr(out), _ptr(out_mask), int(ny),
                                  int(nx), int(out.stride(0))), "sfft_align_image")


def sfft_align_psf(pmap: sfft_pixel_map, x0: float, y0: float, psf_t, psf_out, stream=None):
    """Aligned PSF stamp (device double, side 2s+1) from the template stamp at science point (x0, y0)."""
    st = (psf_t.shape[0] - 1) // 2
    s = (psf_out.shape[0] - 1) // 2
    _check(lib().sfft_align_psf(ctypes.byref(pmap), float(x0), float(y0), _stream_handle(stream), _ptr(psf_t),
                                int(st), _ptr(psf_out), int(s)), "sfft_align_psf")


def sfft_batch_launch(handle):
    _check(lib().sfft_batch_launch(handle), "sfft_batch_launch")


def sfft_subtract_pair_noalloc(desc: sfft_desc, sci, tmpl, mask, ld: int, coeffs, diff, info=None, stream=None):
    """One pair (build + solve + subtract) on the library's static scratch: no allocation."""
    _check(lib().sfft_subtract_pair_noalloc(ctypes.byref(desc), _stream_handle(stream), _ptr(sci), _ptr(tmpl),
                                            _ptr(mask), int(ld), _ptr(coeffs), _ptr(diff), _ptr(info)),
           "sfft_subtract_pair_noalloc")


# bytes of the static scratch (SFFT_NOALLOC_SCRATCH_BYTES in include/sfft.h)
SFFT_NOALLOC_SCRATCH_BYTES = 256 << 20


def sfft_destroy(handle):
    if handle:
        lib().sfft_destroy(handle)


def sfft_strerror(status: int) -> str:
    return strerror(status)


def _stream_handle(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


class Plan:
    """Owning wrapper: one plan on one stream, buffers as torch tensors."""

    def __init__(self, ny, nx, w, dk, db, mode=SFFT_MODE_F64, refine_steps=-1, stream=None, flags=0):
        import torch
        self.desc = make_desc(ny, nx, w, dk, db, mode, refine_steps, flags)
        self.n = sfft_num_coeffs(self.desc)
        self.mode = mode
        self.dtype = torch.float64 if mode == SFFT_MODE_F64 else torch.float32
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.handle = sfft_plan(self.desc, self.stream)

    def build(self, sci, tmpl, mask=None):
        ld = sci.stride(0)
        sfft_build_system(self.handle, sci, tmpl, mask, ld)

    def system(self):
        import torch
        om = torch.empty((self.n, self.n), dtype=torch.float64, device="cuda")
        be = torch.empty((self.n,), dtype=torch.float64, device="cuda")
        sfft_get_system(self.handle, om, be)
        return om, be

    def solve(self, coeffs=None, info=None):
        import torch
        if coeffs is None:
            coeffs = torch.zeros((self.n,), dtype=torch.float64, device="cuda")
        if info is None:
            info = torch.zeros((1,), dtype=torch.int32, device="cuda")
        sfft_solve(self.handle, coeffs, info)
        return coeffs, info

    def residual(self, coeffs):
        import torch
        rho = torch.zeros((1,), dtype=torch.float64, device="cuda")
        sfft_residual(self.handle, coeffs, rho)
        return rho

    def fit_background(self, coeffs):
        sfft_fit_background(self.handle, coeffs)
        return coeffs

    def subtract(self, sci, tmpl, coeffs, diff=None):
        import torch
        if diff is None:
            diff = torch.empty_like(sci)
        sfft_subtract(self.handle, sci, tmpl, coeffs, diff, sci.stride(0))
        return diff

    def apply_kernel(self, img, kcoef, out=None):
        """out = K * img with the plan's w and DK (kcoef: nK (2w+1)^2 device doubles)."""
        import torch
        if out is None:
            out = torch.empty_like(img)
        sfft_apply_kernel(self.handle, img, kcoef, out, img.stride(0))
        return out

    def status(self):
        return sfft_status(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            sfft_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- network (include/sfft_mlp.h)

def sfft_mlp_create(dims, max_batch: int, stream=None):
    nl = len(dims) - 1
    arr = (ctypes.c_int32 * len(dims))(*[int(d) for d in dims])
    h = ctypes.c_void_p(0)
    _check(lib().sfft_mlp_create(arr, nl, int(max_batch), _stream_handle(stream), ctypes.byref(h)),
           "sfft_mlp_create")
    return h


def sfft_mlp_param_count(handle) -> int:
    n = ctypes.c_int64(0)
    _check(lib().sfft_mlp_param_count(handle, ctypes.byref(n)), "sfft_mlp_param_count")
    return n.value


def sfft_mlp_forward(handle, params, x, batch: int, y):
    _check(lib().sfft_mlp_forward(handle, _ptr(params), _ptr(x), int(batch), _ptr(y)), "sfft_mlp_forward")


def sfft_mlp_backward(handle, params, x, dy, batch: int, grad):
    _check(lib().sfft_mlp_backward(handle, _ptr(params), _ptr(x), _ptr(dy), int(batch), _ptr(grad)),
           "sfft_mlp_backward")


def sfft_mlp_mse(handle, y, t, batch: int, dy, loss):
    _check(lib().sfft_mlp_mse(handle, _ptr(y), _ptr(t), int(batch), _ptr(dy), _ptr(loss)), "sfft_mlp_mse")


def sfft_mlp_adam_step(handle, params, grad, m1, m2, step: int, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    _check(lib().sfft_mlp_adam_step(handle, _ptr(params), _ptr(grad), _ptr(m1), _ptr(m2), int(step), float(lr),
                                    float(b1), float(b2), float(eps)), "sfft_mlp_adam_step")


def sfft_mlp_set_weights_bf16(handle, params):
    _check(lib().sfft_mlp_set_weights_bf16(handle, _ptr(params)), "sfft_mlp_set_weights_bf16")


def sfft_mlp_infer(handle, x, batch: int, scale, shift, theta, ld_theta: int):
    _check(lib().sfft_mlp_infer(handle, _ptr(x), int(batch), _ptr(scale), _ptr(shift), _ptr(theta),
                                int(ld_theta)), "sfft_mlp_infer")


def sfft_mlp_destroy(handle):
    if handle:
        lib().sfft_mlp_destroy(handle)
