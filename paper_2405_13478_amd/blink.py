"""ctypes binding of libblink.so: the C ABI of include/blink.h with torch tensors.

Argument marshalling only: shapes and dtypes are checked, device pointers and
the current HIP stream are handed to the library, which enqueues all the work.
There is no fallback: without the built library every call raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libblink.so")

NATURAL, UNIFORM = 0, 1
NORM_NONE, NORM_WEIGHTS = 0, 1
VIS_C64, VIS_F16, VIS_BF16 = 0, 1, 2
CALL_GRID, CALL_IMAGE, CALL_ADJOINT = 0, 1, 2

STATUS = {0: "BLINK_OK", -1: "BLINK_E_ARG", -2: "BLINK_E_SIZE", -3: "BLINK_E_UNSUPPORTED",
          -4: "BLINK_E_WORKSPACE", -5: "BLINK_E_HIP"}

# every symbol include/blink.h declares
EXPORTS = ("blink_status_string", "blink_supported_n", "blink_workspace_size", "blink_grid",
           "blink_fft2d", "blink_image_batch", "blink_degrid_adjoint", "blink_image_batch_timed",
           "blink_dynamic_spectra", "blink_correlate", "blink_image_batch_noalloc")

NOALLOC_SCRATCH_BYTES = 64 << 20       # BLINK_NOALLOC_SCRATCH_BYTES

REF_NONE, REF_MEAN, REF_MODEL = 0, 1, 2
REF_MAX_LEN = 128

# kernel classes reported by blink_image_batch_timed
KCLASS = ("sort", "bounds", "grid_cols", "rows")


class BlinkError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {STATUS.get(code, code)} ({status_string(code)})")
        self.code = code


class Problem(ctypes.Structure):
    _fields_ = [("n_time", ctypes.c_int32), ("n_chan", ctypes.c_int32), ("n_bl", ctypes.c_int32),
                ("n_ant", ctypes.c_int32), ("grid_n", ctypes.c_int32), ("out_n", ctypes.c_int32),
                ("pixscale", ctypes.c_double), ("weighting", ctypes.c_int32),
                ("norm", ctypes.c_int32), ("vis_type", ctypes.c_int32),
                ("chunk_images", ctypes.c_int32), ("cols_per_wg", ctypes.c_int32),
                ("rows_wg", ctypes.c_int32), ("kernel_support", ctypes.c_int32),
                ("kernel_beta", ctypes.c_double), ("phase_l", ctypes.c_double), ("phase_m", ctypes.c_double),
                ("reproject", ctypes.c_int32)]


class Inputs(ctypes.Structure):
    _fields_ = [("vis", ctypes.c_void_p), ("vis_scale", ctypes.c_void_p), ("uvw_m", ctypes.c_void_p),
                ("freq_hz", ctypes.c_void_p), ("flags", ctypes.c_void_p), ("ant1", ctypes.c_void_p),
                ("ant2", ctypes.c_void_p), ("gains", ctypes.c_void_p), ("cable_m", ctypes.c_void_p)]


class KernelTimes(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * 4), ("launches", ctypes.c_int64 * 4)]


_lib = None


def load_library(path: str | None = None):
    """Load libblink.so (built in-tree by ``__graft_entry__.build()``)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"libblink.so not built: {p} is missing (run __graft_entry__.build())")
    lib = ctypes.CDLL(p)
    vp, i32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t
    P, I = ctypes.POINTER(Problem), ctypes.POINTER(Inputs)
    lib.blink_status_string.argtypes = [i32]
    lib.blink_status_string.restype = ctypes.c_char_p
    lib.blink_supported_n.argtypes = [i32]
    lib.blink_supported_n.restype = i32
    lib.blink_workspace_size.argtypes = [P, i32]
    lib.blink_workspace_size.restype = sz
    lib.blink_grid.argtypes = [P, I, vp, vp, vp, vp, vp, sz, vp]
    lib.blink_grid.restype = i32
    lib.blink_fft2d.argtypes = [vp, vp, i32, i32, i32, vp]
    lib.blink_fft2d.restype = i32
    lib.blink_image_batch.argtypes = [P, I, vp, vp, vp, sz, vp]
    lib.blink_image_batch.restype = i32
    lib.blink_degrid_adjoint.argtypes = [P, I, vp, vp, vp, vp, vp, sz, vp]
    lib.blink_degrid_adjoint.restype = i32
    lib.blink_image_batch_noalloc.argtypes = [P, I, vp, vp, vp]
    lib.blink_image_batch_noalloc.restype = i32
    lib.blink_image_batch_timed.argtypes = [P, I, vp, vp, vp, sz, vp, ctypes.POINTER(KernelTimes)]
    lib.blink_image_batch_timed.restype = i32
    lib.blink_dynamic_spectra.argtypes = [vp, i32, i32, i32, i32, i32, vp, vp, vp]
    lib.blink_dynamic_spectra.restype = i32
    lib.blink_correlate.argtypes = [vp, i32, i32, i32, i32, vp, vp, vp]
    lib.blink_correlate.restype = i32
    if path is None:
        _lib = lib
    return lib


def status_string(code: int) -> str:
    try:
        return load_library().blink_status_string(int(code)).decode()
    except RuntimeError:
        return "library not loaded"


def supported_n(n: int) -> bool:
    return bool(load_library().blink_supported_n(int(n)))


# ---------------------------------------------------------------- helpers
def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dev(t, name, dtype=None, shape=None):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _check(code, what):
    if code != 0:
        raise BlinkError(code, what)


def make_problem(vis, uvw_m, freq_hz, grid_n, pixscale, out_n=None, weighting=NATURAL,
                 norm=NORM_WEIGHTS, gains=None, chunk_images=0, cols_per_wg=0, rows_wg=0,
                 kernel_support=0, kernel_beta=-1.0, phase_lm=(0.0, 0.0), cable_m=None,
                 reproject=False) -> Problem:
    if vis.dtype == torch.complex64:
        T, C, B = vis.shape
        vt = VIS_C64
    elif vis.dtype in (torch.float16, torch.bfloat16):
        T, C, B, two = vis.shape
        if two != 2:
            raise ValueError("half-precision visibilities must be [T][C][B][2]")
        vt = VIS_F16 if vis.dtype == torch.float16 else VIS_BF16
    else:
        raise ValueError(f"unsupported visibility dtype {vis.dtype}")
    n_ant = gains.shape[0] if gains is not None else (cable_m.shape[0] if cable_m is not None else 0)
    return Problem(n_time=T, n_chan=C, n_bl=B, n_ant=n_ant,
                   grid_n=grid_n, out_n=grid_n if out_n is None else out_n,
                   pixscale=float(pixscale), weighting=int(weighting), norm=int(norm),
                   vis_type=vt, chunk_images=int(chunk_images), cols_per_wg=int(cols_per_wg),
                   rows_wg=int(rows_wg), kernel_support=int(kernel_support),
                   kernel_beta=float(kernel_beta), phase_l=float(phase_lm[0]), phase_m=float(phase_lm[1]),
                   reproject=int(bool(reproject)))


def make_inputs(p: Problem, vis, uvw_m, freq_hz, flags=None, vis_scale=None, ant1=None,
                ant2=None, gains=None, cable_m=None):
    T, C, B = p.n_time, p.n_chan, p.n_bl
    _dev(vis, "vis")
    _dev(uvw_m, "uvw_m", torch.float64, (T, B, 3))
    _dev(freq_hz, "freq_hz", torch.float64, (C,))
    _dev(flags, "flags", torch.uint8, (T, B))
    _dev(vis_scale, "vis_scale", torch.float32, (C,))
    _dev(ant1, "ant1", torch.int32, (B,))
    _dev(ant2, "ant2", torch.int32, (B,))
    _dev(gains, "gains", torch.complex64)
    _dev(cable_m, "cable_m", torch.float64, (p.n_ant,) if cable_m is not None else None)
    if gains is not None and cable_m is not None and gains.shape[0] != cable_m.shape[0]:
        raise ValueError("gains and cable_m must cover the same antennas")
    keep = (vis, uvw_m, freq_hz, flags, vis_scale, ant1, ant2, gains, cable_m)
    inp = Inputs(vis=_ptr(vis), vis_scale=_ptr(vis_scale), uvw_m=_ptr(uvw_m), freq_hz=_ptr(freq_hz),
                 flags=_ptr(flags), ant1=_ptr(ant1), ant2=_ptr(ant2), gains=_ptr(gains),
                 cable_m=_ptr(cable_m))
    return inp, keep


def workspace(p: Problem, call: int, device) -> torch.Tensor:
    n = load_library().blink_workspace_size(ctypes.byref(p), int(call))
    if n == 0:
        return torch.empty(0, dtype=torch.uint8, device=device)
    return torch.empty(n, dtype=torch.uint8, device=device)


# ---------------------------------------------------------------- calls
def tuning_for(grid_n, out_n, n_bl, weighting, vis_type, chunk_images=None, cols_per_wg=None,
               rows_wg=None):
    """Tunables for a shape: explicit values win, then the autotuner's cache, then 0 (defaults)."""
    from . import autotune
    t = autotune.lookup(grid_n, out_n, n_bl, weighting, vis_type) or {}
    pick = lambda v, k: int(v) if v is not None else int(t.get(k, 0))
    return dict(chunk_images=pick(chunk_images, "chunk_images"), cols_per_wg=pick(cols_per_wg, "cols_per_wg"),
                rows_wg=pick(rows_wg, "rows_wg"))


def _vis_type(vis):
    return {torch.complex64: VIS_C64, torch.float16: VIS_F16, torch.bfloat16: VIS_BF16}.get(vis.dtype, -1)


def image_batch(vis, uvw_m, freq_hz, *, grid_n, pixscale, out_n=None, weighting=NATURAL,
                norm=NORM_WEIGHTS, flags=None, vis_scale=None, ant1=None, ant2=None, gains=None,
                chunk_images=None, cols_per_wg=None, rows_wg=None, images=None, weight_sum=None,
                ws=None, stream=None, times=None, kernel_support=0, kernel_beta=-1.0, phase_lm=(0.0, 0.0),
                cable_m=None, reproject=False):
    """Dirty images [T*C][M][M] float32 of the cube (blink_image_batch).

    Tunables left as None come from the autotuner's cache for this shape.
    ``kernel_support`` W >= 1 grids with a Kaiser-Bessel kernel of W cells
    (shape ``kernel_beta``, < 0 for the default) and corrects the image for it.
    ``phase_lm`` = (l0, m0) rotates the phase centre from zenith to that direction;
    with ``reproject`` the image lies on the tangent plane at (l0, m0).
    ``cable_m`` [A] float64 electrical cable lengths (with ``ant1``/``ant2``)
    applies the cable correction exp(+2 pi i nu (l_ant1 - l_ant2) / c).
    With ``times`` (a KernelTimes) the instrumented twin blink_image_batch_timed
    runs instead: same results, per-kernel-class event timings, host waits.
    """
    lib = load_library()
    M = grid_n if out_n is None else out_n
    tun = tuning_for(grid_n, M, vis.shape[2], weighting, _vis_type(vis), chunk_images, cols_per_wg, rows_wg)
    p = make_problem(vis, uvw_m, freq_hz, grid_n, pixscale, out_n, weighting, norm, gains, **tun,
                     kernel_support=kernel_support, kernel_beta=kernel_beta, phase_lm=phase_lm,
                     cable_m=cable_m, reproject=reproject)
    inp, _keep = make_inputs(p, vis, uvw_m, freq_hz, flags, vis_scale, ant1, ant2, gains, cable_m)
    n_img, M = p.n_time * p.n_chan, p.out_n
    if images is None:
        images = torch.empty((n_img, M, M), dtype=torch.float32, device=vis.device)
    _dev(images, "images", torch.float32, (n_img, M, M))
    _dev(weight_sum, "weight_sum", torch.float32, (n_img,))
    if ws is None:
        ws = workspace(p, CALL_IMAGE, vis.device)
    args = (ctypes.byref(p), ctypes.byref(inp), _ptr(images), _ptr(weight_sum),
            _ptr(ws) if ws.numel() else None, ws.numel(), _stream(stream))
    if times is None:
        _check(lib.blink_image_batch(*args), "blink_image_batch")
    else:
        _check(lib.blink_image_batch_timed(*args, ctypes.byref(times)), "blink_image_batch_timed")
    return images


def image_batch_noalloc(images, vis, uvw_m, freq_hz, *, grid_n, pixscale, out_n=None,
                        weighting=NATURAL, norm=NORM_WEIGHTS, flags=None, vis_scale=None, ant1=None,
                        ant2=None, gains=None, chunk_images=0, cols_per_wg=0, rows_wg=0,
                        weight_sum=None, stream=None):
    """blink_image_batch_noalloc into caller-allocated ``images`` [T*C][M][M]
    (and ``weight_sum`` [T*C]): the library allocates nothing; its scratch is a
    fixed per-GPU array. Tunables are passed as given (0 = library default)."""
    lib = load_library()
    p = make_problem(vis, uvw_m, freq_hz, grid_n, pixscale, out_n, weighting, norm, gains,
                     chunk_images, cols_per_wg, rows_wg)
    inp, _keep = make_inputs(p, vis, uvw_m, freq_hz, flags, vis_scale, ant1, ant2, gains)
    n_img, M = p.n_time * p.n_chan, p.out_n
    _dev(images, "images", torch.float32, (n_img, M, M))
    _dev(weight_sum, "weight_sum", torch.float32, (n_img,))
    _check(lib.blink_image_batch_noalloc(ctypes.byref(p), ctypes.byref(inp), _ptr(images),
                                         _ptr(weight_sum), _stream(stream)),
           "blink_image_batch_noalloc")
    return images


def grid(vis, uvw_m, freq_hz, *, grid_n, pixscale, weighting=NATURAL, flags=None, vis_scale=None,
         ant1=None, ant2=None, gains=None, counts=True, chunk_images=0, stream=None,
         kernel_support=0, kernel_beta=-1.0, phase_lm=(0.0, 0.0), cable_m=None, reproject=False):
    """(weighted grid [T*C][N][N] c64, counts int32 or None, W float32, n_dropped int32)."""
    lib = load_library()
    p = make_problem(vis, uvw_m, freq_hz, grid_n, pixscale, grid_n, weighting, NORM_NONE, gains,
                     chunk_images, kernel_support=kernel_support, kernel_beta=kernel_beta, phase_lm=phase_lm,
                     cable_m=cable_m, reproject=reproject)
    inp, _keep = make_inputs(p, vis, uvw_m, freq_hz, flags, vis_scale, ant1, ant2, gains, cable_m)
    n_img, N, dev = p.n_time * p.n_chan, grid_n, vis.device
    g = torch.empty((n_img, N, N), dtype=torch.complex64, device=dev)
    c = torch.empty((n_img, N, N), dtype=torch.int32, device=dev) if counts else None
    w = torch.empty((n_img,), dtype=torch.float32, device=dev)
    d = torch.empty((n_img,), dtype=torch.int32, device=dev)
    ws = workspace(p, CALL_GRID, dev)
    code = lib.blink_grid(ctypes.byref(p), ctypes.byref(inp), _ptr(g), _ptr(c), _ptr(w), _ptr(d),
                          _ptr(ws) if ws.numel() else None, ws.numel(), _stream(stream))
    _check(code, "blink_grid")
    return g, c, w, d


def fft2d(x, sign=+1, out=None, stream=None):
    """Batched unnormalised 2D C2C transform of [batch][n][n] complex64 (blink_fft2d)."""
    lib = load_library()
    _dev(x, "x", torch.complex64)
    if x.dim() != 3 or x.shape[1] != x.shape[2]:
        raise ValueError("x must be [batch][n][n]")
    if out is None:
        out = torch.empty_like(x)
    _dev(out, "out", torch.complex64, tuple(x.shape))
    code = lib.blink_fft2d(_ptr(x), _ptr(out), int(x.shape[0]), int(x.shape[1]), int(sign),
                           _stream(stream))
    _check(code, "blink_fft2d")
    return out


def degrid_adjoint(image_grad, vis, uvw_m, freq_hz, *, grid_n, pixscale, out_n=None,
                   weighting=NATURAL, norm=NORM_WEIGHTS, flags=None, ant1=None, ant2=None,
                   gains=None, want_gain_grad=True, chunk_images=0, stream=None, weight_sum=None,
                   vis_scale=None, phase_lm=(0.0, 0.0), cable_m=None, reproject=False,
                   kernel_support=0, kernel_beta=-1.0):
    """(vis_grad [T][C][B] c64, gain_grad [A] c64 or None) of a loss with dL/dimages = image_grad.

    ``weight_sum`` [T*C] float32: the forward call's weight sums (skips
    counting them again). With FP16/BF16 ``vis`` (and ``vis_scale``) the
    gradient is with respect to the dequantised visibilities. ``phase_lm``,
    ``cable_m``, ``reproject`` and the gridding kernel must be those of the
    forward call.
    """
    lib = load_library()
    p = make_problem(vis, uvw_m, freq_hz, grid_n, pixscale, out_n, weighting, norm, gains, chunk_images,
                     phase_lm=phase_lm, cable_m=cable_m, reproject=reproject,
                     kernel_support=kernel_support, kernel_beta=kernel_beta)
    inp, _keep = make_inputs(p, vis, uvw_m, freq_hz, flags, vis_scale, ant1, ant2, gains, cable_m)
    n_img, M = p.n_time * p.n_chan, p.out_n
    T, C, B = p.n_time, p.n_chan, p.n_bl
    _dev(image_grad, "image_grad", torch.float32, (n_img, M, M))
    _dev(weight_sum, "weight_sum", torch.float32, (n_img,))
    vg = torch.empty((T, C, B), dtype=torch.complex64, device=vis.device)
    gg = None
    if gains is not None and want_gain_grad:
        gg = torch.empty(gains.shape, dtype=torch.complex64, device=vis.device)
    ws = workspace(p, CALL_ADJOINT, vis.device)
    code = lib.blink_degrid_adjoint(ctypes.byref(p), ctypes.byref(inp), _ptr(image_grad), _ptr(weight_sum),
                                    _ptr(vg), _ptr(gg), _ptr(ws) if ws.numel() else None, ws.numel(),
                                    _stream(stream))
    _check(code, "blink_degrid_adjoint")
    return vg, gg


def dynamic_spectra(images, ref_mode=REF_NONE, ref_len=1, ref_image=None, out=None, stream=None):
    """Per-pixel time series [P][C][T] of an image cube [T][C][M][M] (blink_dynamic_spectra).

    ``ref_mode`` REF_NONE transposes; REF_MEAN subtracts the mean of the
    ``ref_len`` preceding images (0 at t = 0); REF_MODEL subtracts
    ``ref_image`` [C][M][M].
    """
    lib = load_library()
    _dev(images, "images", torch.float32)
    if images.dim() != 4 or images.shape[2] != images.shape[3]:
        raise ValueError("images must be [T][C][M][M]")
    T, C, M = images.shape[0], images.shape[1], images.shape[2]
    P = M * M
    if ref_mode == REF_MODEL:
        _dev(ref_image, "ref_image", torch.float32, (C, M, M))
    if out is None:
        out = torch.empty((P, C, T), dtype=torch.float32, device=images.device)
    _dev(out, "out", torch.float32, (P, C, T))
    code = lib.blink_dynamic_spectra(_ptr(images), T, C, P, int(ref_mode), int(ref_len),
                                     _ptr(ref_image) if ref_mode == REF_MODEL else None, _ptr(out),
                                     _stream(stream))
    _check(code, "blink_dynamic_spectra")
    return out


def correlate(volt, vis=None, autos=False, stream=None):
    """X-engine (blink_correlate): int8 voltages [T][C][A][S][2] -> (vis [T][C][B] c64, autos or None)."""
    lib = load_library()
    _dev(volt, "volt", torch.int8)
    if volt.dim() != 5 or volt.shape[4] != 2:
        raise ValueError("volt must be [T][C][A][S][2] int8")
    T, C, A, S = (int(d) for d in volt.shape[:4])
    B = A * (A - 1) // 2
    if vis is None:
        vis = torch.empty((T, C, B), dtype=torch.complex64, device=volt.device)
    _dev(vis, "vis", torch.complex64, (T, C, B))
    au = torch.empty((T, C, A), dtype=torch.float32, device=volt.device) if autos else None
    code = lib.blink_correlate(_ptr(volt), T, C, A, S, _ptr(vis), _ptr(au), _stream(stream))
    _check(code, "blink_correlate")
    return vis, au


class BlinkImage(torch.autograd.Function):
    """Differentiable dirty imaging: images = blink_image_batch(g[a1] conj(g[a2]) V).

    Gradients flow to the complex64 visibilities and the per-antenna gains
    through the hand-written adjoint (degridding + forward transforms), which
    reuses the forward call's weight sums.
    """

    @staticmethod
    def forward(ctx, vis, gains, uvw_m, freq_hz, ant1, ant2, flags, grid_n, pixscale, out_n,
                weighting, norm, phase_lm=(0.0, 0.0), cable_m=None, reproject=False,
                kernel_support=0, kernel_beta=-1.0):
        wsum = torch.empty((vis.shape[0] * vis.shape[1],), dtype=torch.float32, device=vis.device)
        img = image_batch(vis, uvw_m, freq_hz, grid_n=grid_n, pixscale=pixscale, out_n=out_n,
                          weighting=weighting, norm=norm, flags=flags, ant1=ant1, ant2=ant2,
                          gains=gains, weight_sum=wsum, phase_lm=phase_lm, cable_m=cable_m,
                          reproject=reproject, kernel_support=kernel_support, kernel_beta=kernel_beta)
        ctx.save_for_backward(vis, gains, uvw_m, freq_hz, ant1, ant2, flags, wsum, cable_m)
        ctx.cfg = (grid_n, pixscale, out_n, weighting, norm, phase_lm, reproject, kernel_support, kernel_beta)
        return img

    @staticmethod
    def backward(ctx, grad_images):
        vis, gains, uvw_m, freq_hz, ant1, ant2, flags, wsum, cable_m = ctx.saved_tensors
        grid_n, pixscale, out_n, weighting, norm, phase_lm, reproject, ksup, kbeta = ctx.cfg
        vg, gg = degrid_adjoint(grad_images.contiguous().float(), vis, uvw_m, freq_hz,
                                grid_n=grid_n, pixscale=pixscale, out_n=out_n,
                                weighting=weighting, norm=norm, flags=flags, ant1=ant1,
                                ant2=ant2, gains=gains,
                                want_gain_grad=gains is not None and ctx.needs_input_grad[1],
                                weight_sum=wsum, phase_lm=phase_lm, cable_m=cable_m, reproject=reproject,
                                kernel_support=ksup, kernel_beta=kbeta)
        return (vg if ctx.needs_input_grad[0] else None, gg, None, None, None, None, None,
                None, None, None, None, None, None, None, None, None, None)


def blink_image(vis, gains, uvw_m, freq_hz, ant1, ant2, *, grid_n, pixscale, out_n=None,
                weighting=NATURAL, norm=NORM_WEIGHTS, flags=None, phase_lm=(0.0, 0.0), cable_m=None,
                reproject=False, kernel_support=0, kernel_beta=-1.0):
    """Functional form of BlinkImage."""
    return BlinkImage.apply(vis, gains, uvw_m, freq_hz, ant1, ant2, flags, grid_n, pixscale,
                            grid_n if out_n is None else out_n, weighting, norm, phase_lm, cable_m, reproject,
                            kernel_support, kernel_beta)
