"""CPU checks of the C ABI: the library loads, exports what include/blink.h
declares, and rejects invalid arguments on the host with the documented
status codes. Every call here fails validation before anything would be
enqueued, so no GPU is touched."""
import ctypes
import os
import re

import pytest

import paper_2405_13478_amd as blink
from paper_2405_13478_amd import blink as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
E_OK, E_ARG, E_SIZE, E_UNSUP, E_WS, E_HIP = 0, -1, -2, -3, -4, -5
FAKE = ctypes.c_void_p(0x100000)   # never dereferenced: validation fails first


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return blink.load_library()


def _declared():
    text = open(os.path.join(ROOT, "include", "blink.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(blink_[a-z0-9_]+)\s*\(", text)))


def test_exports_every_declared_symbol(lib):
    decl = _declared()
    assert decl == sorted(B.EXPORTS)
    for name in decl:
        assert hasattr(lib, name), name


def test_status_strings(lib):
    for code in (E_OK, E_ARG, E_SIZE, E_UNSUP, E_WS, E_HIP):
        assert lib.blink_status_string(code).decode()
    assert lib.blink_status_string(E_OK).decode() == "ok"


def test_supported_sizes(lib):
    sup = [n for n in range(1, 5000) if lib.blink_supported_n(n)]
    assert {128, 180, 1024, 2048}.issubset(sup)
    assert all(n % 2 == 0 for n in sup)


def _prob(**kw):
    d = dict(n_time=2, n_chan=3, n_bl=10, n_ant=5, grid_n=64, out_n=32, pixscale=1e-2,
             weighting=0, norm=1, vis_type=0, chunk_images=0)
    d.update(kw)
    return B.Problem(**d)


def _inputs(**kw):
    d = dict(vis=FAKE, vis_scale=None, uvw_m=FAKE, freq_hz=FAKE, flags=None, ant1=None,
             ant2=None, gains=None, cable_m=None)
    d.update(kw)
    return B.Inputs(**d)


def _image(lib, p, inp, images=FAKE, ws=None, nbytes=0):
    return lib.blink_image_batch(ctypes.byref(p) if p is not None else None,
                                 ctypes.byref(inp) if inp is not None else None,
                                 images, None, ws, nbytes, None)


@pytest.mark.parametrize("kw,code", [
    (dict(grid_n=63), E_SIZE), (dict(grid_n=0), E_SIZE), (dict(out_n=33), E_SIZE),
    (dict(out_n=128), E_SIZE), (dict(out_n=0), E_SIZE), (dict(n_time=-1), E_SIZE),
    (dict(grid_n=1000), E_UNSUP), (dict(grid_n=14, out_n=8), E_UNSUP),
    (dict(pixscale=0.0), E_ARG), (dict(pixscale=float("nan")), E_ARG),
    (dict(pixscale=float("inf")), E_ARG), (dict(pixscale=-1.0), E_ARG),
    (dict(weighting=2), E_ARG), (dict(norm=5), E_ARG), (dict(vis_type=3), E_ARG),
    (dict(chunk_images=-2), E_ARG), (dict(cols_per_wg=3), E_ARG), (dict(cols_per_wg=16), E_ARG),
    (dict(rows_wg=-1), E_ARG),
    (dict(kernel_support=-1), E_ARG), (dict(kernel_support=17), E_ARG),
    (dict(kernel_support=1, kernel_beta=-1.0), E_ARG),        # default shape needs W >= 2
    (dict(kernel_support=4, kernel_beta=float("nan")), E_ARG),
    (dict(kernel_support=4, kernel_beta=float("inf")), E_ARG),
    (dict(kernel_support=4, kernel_beta=80.5), E_ARG),              # I0(beta) beyond FP32
    (dict(phase_l=float("nan")), E_ARG), (dict(phase_l=0.8, phase_m=0.6), E_ARG),   # needs l^2 + m^2 < 1
    (dict(phase_m=float("inf")), E_ARG),
    (dict(phase_l=0.1, reproject=2), E_ARG), (dict(reproject=-1), E_ARG),
])
def test_problem_validation(lib, kw, code):
    assert _image(lib, _prob(**kw), _inputs()) == code
    assert lib.blink_workspace_size(ctypes.byref(_prob(**kw)), 1) == 0


def test_null_and_input_validation(lib):
    assert _image(lib, None, _inputs()) == E_ARG
    assert _image(lib, _prob(), None) == E_ARG
    assert _image(lib, _prob(), _inputs(vis=None)) == E_ARG
    assert _image(lib, _prob(), _inputs(uvw_m=None)) == E_ARG
    assert _image(lib, _prob(), _inputs(freq_hz=None)) == E_ARG
    assert _image(lib, _prob(), _inputs(), images=None) == E_ARG
    # half-precision storage needs the per-channel scale
    assert _image(lib, _prob(vis_type=1), _inputs()) == E_ARG
    assert _image(lib, _prob(vis_type=2), _inputs()) == E_ARG
    # gains need both antenna index arrays and n_ant >= 1
    assert _image(lib, _prob(), _inputs(gains=FAKE)) == E_ARG
    assert _image(lib, _prob(), _inputs(gains=FAKE, ant1=FAKE)) == E_ARG
    assert _image(lib, _prob(n_ant=0), _inputs(gains=FAKE, ant1=FAKE, ant2=FAKE)) == E_ARG


def test_workspace_validation(lib):
    p = _prob()
    need = lib.blink_workspace_size(ctypes.byref(p), 1)
    assert need > 0
    assert _image(lib, p, _inputs(), ws=None, nbytes=need) == E_WS
    assert _image(lib, p, _inputs(), ws=FAKE, nbytes=need - 1) == E_WS
    assert _image(lib, p, _inputs(), ws=ctypes.c_void_p(0x100010), nbytes=need) == E_WS


def test_empty_problem_is_a_no_op(lib):
    # zero images: nothing to do, no workspace needed, nothing enqueued
    assert _image(lib, _prob(n_time=0), _inputs(vis=None, uvw_m=None, freq_hz=None)) == E_OK
    assert _image(lib, _prob(n_chan=0), _inputs()) == E_OK


def test_fft2d_validation(lib):
    f = lib.blink_fft2d
    assert f(None, FAKE, 1, 64, 1, None) == E_ARG
    assert f(FAKE, None, 1, 64, 1, None) == E_ARG
    assert f(FAKE, FAKE, 1, 64, 0, None) == E_ARG
    assert f(FAKE, FAKE, 1, 64, 2, None) == E_ARG
    assert f(FAKE, FAKE, -1, 64, 1, None) == E_SIZE
    assert f(FAKE, FAKE, 1, 1000, 1, None) == E_UNSUP
    assert f(FAKE, FAKE, 0, 64, 1, None) == E_OK


def test_grid_and_adjoint_validation(lib):
    p = _prob()
    inp = _inputs()
    g = lib.blink_grid
    assert g(ctypes.byref(p), ctypes.byref(inp), None, None, None, None, None, 0, None) == E_ARG
    assert g(ctypes.byref(_prob(grid_n=7)), ctypes.byref(inp), FAKE, None, None, None, None, 0,
             None) == E_SIZE
    a = lib.blink_degrid_adjoint
    # FP16 storage passes validation (and then needs a workspace); without its scale it is refused
    assert a(ctypes.byref(_prob(vis_type=1)), ctypes.byref(_inputs(vis_scale=FAKE)), FAKE, None, FAKE,
             None, None, 0, None) == E_WS
    assert a(ctypes.byref(_prob(vis_type=1)), ctypes.byref(inp), FAKE, None, FAKE, None, None, 0,
             None) == E_ARG
    # a gain gradient needs gains
    assert a(ctypes.byref(p), ctypes.byref(inp), FAKE, None, FAKE, FAKE, None, 0, None) == E_ARG
    assert a(ctypes.byref(p), ctypes.byref(inp), None, None, FAKE, None, None, 0, None) == E_ARG
    # the forward weight sums are optional
    assert a(ctypes.byref(p), ctypes.byref(inp), FAKE, FAKE, FAKE, None, None, 0, None) == E_WS


def test_workspace_sizes_scale(lib):
    c3 = B.Problem(n_time=10, n_chan=768, n_bl=8128, n_ant=128, grid_n=1024, out_n=512,
                   pixscale=8.3e-5, weighting=0, norm=1, vis_type=0, chunk_images=0)
    s_grid = lib.blink_workspace_size(ctypes.byref(c3), 0)
    s_img = lib.blink_workspace_size(ctypes.byref(c3), 1)
    s_adj = lib.blink_workspace_size(ctypes.byref(c3), 2)
    assert 0 < s_grid < s_img < s_adj
    # an explicit chunk sets the half-spectrum share: chunk * N/2 * M * 8 bytes
    c3.chunk_images = 4
    s4 = lib.blink_workspace_size(ctypes.byref(c3), 1)
    c3.chunk_images = 8
    s8 = lib.blink_workspace_size(ctypes.byref(c3), 1)
    assert s8 - s4 >= 4 * 512 * 512 * 8


def test_uniform_kernel_gridding_sizes_its_density_table(lib):
    # uniform weighting with a gridding kernel passes validation and takes
    # one int per (image of a chunk, baseline) for the cell occupancy
    for call in (0, 1):
        nat = _prob(kernel_support=4, kernel_beta=-1.0, chunk_images=3)
        uni = _prob(kernel_support=4, kernel_beta=-1.0, chunk_images=3, weighting=1)
        s_nat = lib.blink_workspace_size(ctypes.byref(nat), call)
        s_uni = lib.blink_workspace_size(ctypes.byref(uni), call)
        assert s_uni - s_nat == -(-3 * 10 * 4 // 256) * 256
        assert _image(lib, uni, _inputs(), ws=None, nbytes=0) == E_WS
    # nearest-cell uniform weighting needs no such table
    assert lib.blink_workspace_size(ctypes.byref(_prob(weighting=1)), 1) == \
        lib.blink_workspace_size(ctypes.byref(_prob()), 1)


def test_kernel_gridding_adjoint_sizes_its_column_buffer(lib):
    # the adjoint with a gridding kernel passes validation, needs a workspace,
    # and that workspace holds every transformed half-spectrum column of a
    # chunk ([chunk][N/2][N] complex64) on top of the nearest-cell adjoint's
    p = _prob(kernel_support=6, kernel_beta=-1.0, chunk_images=2)
    a = lib.blink_degrid_adjoint
    assert a(ctypes.byref(p), ctypes.byref(_inputs()), FAKE, None, FAKE, None, None, 0, None) == E_WS
    p0 = _prob(chunk_images=2)
    assert a(ctypes.byref(p0), ctypes.byref(_inputs()), FAKE, None, FAKE, None, None, 0, None) == E_WS
    s_kb = lib.blink_workspace_size(ctypes.byref(p), 2)
    s_nc = lib.blink_workspace_size(ctypes.byref(p0), 2)
    assert s_kb - s_nc == 2 * 32 * 64 * 8


def test_dynamic_spectra_validation(lib):
    d = lib.blink_dynamic_spectra
    assert d(FAKE, -1, 2, 16, 0, 1, None, FAKE, None) == E_SIZE
    assert d(FAKE, 4, 70000, 16, 0, 1, None, FAKE, None) == E_SIZE        # channels on grid.z
    assert d(FAKE, 4, 2, 16, 3, 1, None, FAKE, None) == E_ARG              # unknown mode
    assert d(FAKE, 4, 2, 16, 1, 0, None, FAKE, None) == E_ARG              # window 0
    assert d(FAKE, 4, 2, 16, 1, B.REF_MAX_LEN + 1, None, FAKE, None) == E_ARG
    assert d(FAKE, 4, 2, 16, 2, 1, None, FAKE, None) == E_ARG              # model without image
    assert d(None, 4, 2, 16, 0, 1, None, FAKE, None) == E_ARG
    assert d(FAKE, 4, 2, 16, 0, 1, None, None, None) == E_ARG
    assert d(None, 0, 2, 16, 0, 1, None, None, None) == E_OK               # empty: nothing to do


def test_correlate_validation(lib):
    c = lib.blink_correlate
    assert c(FAKE, -1, 2, 8, 32, FAKE, None, None) == E_SIZE
    assert c(FAKE, 1, 1, 1, 32, FAKE, None, None) == E_SIZE            # one antenna: no pairs
    assert c(FAKE, 1, 1, 8, 24, FAKE, None, None) == E_SIZE            # samples not a multiple of 16
    assert c(FAKE, 1, 1, 8, 65536, FAKE, None, None) == E_SIZE         # int32 sums could overflow
    assert c(None, 1, 1, 8, 32, FAKE, None, None) == E_ARG
    assert c(FAKE, 1, 1, 8, 32, None, None, None) == E_ARG
    assert c(ctypes.c_void_p(0x100008), 1, 1, 8, 32, FAKE, None, None) == E_ARG   # misaligned
    assert c(None, 0, 4, 8, 32, None, None, None) == E_OK                # empty


def test_problem_struct_layout_matches_the_header():
    # the binding's ctypes layout of blink_problem: 8-byte doubles aligned, the
    # trailing reproject flag after phase_m, padded to a multiple of 8
    assert B.Problem.reproject.offset == B.Problem.phase_m.offset + 8
    assert ctypes.sizeof(B.Problem) == B.Problem.reproject.offset + 8


def test_phase_rotation_adjoint_passes_validation(lib):
    # a rotated problem's adjoint is built: it passes validation and then needs a workspace
    p = _prob(phase_l=0.1, phase_m=-0.2)
    a = lib.blink_degrid_adjoint
    assert a(ctypes.byref(p), ctypes.byref(_inputs()), FAKE, None, FAKE, None, None, 0, None) == E_WS
    assert lib.blink_workspace_size(ctypes.byref(p), 2) > 0


def test_workspace_holds_the_delay_table(lib):
    # image, grid and adjoint calls reserve the [T][B] delay table of the phase rotation
    # and the cable correction whether or not one is applied (cable lengths are
    # an input, which the size query does not see); with the two sort key
    # buffers, two index buffers, sorted u, v and order that is 52 B per
    # baseline and timestep
    p0 = _prob(n_bl=1000)
    p1 = _prob(n_bl=1000, phase_l=0.1)
    for call in (0, 1, 2):
        s0 = lib.blink_workspace_size(ctypes.byref(p0), call)
        assert s0 == lib.blink_workspace_size(ctypes.byref(p1), call)
        assert s0 >= 2 * 1000 * 52


def test_cable_correction_validation(lib):
    # cable lengths need both antenna index arrays and n_ant >= 1
    assert _image(lib, _prob(), _inputs(cable_m=FAKE)) == E_ARG
    assert _image(lib, _prob(), _inputs(cable_m=FAKE, ant1=FAKE)) == E_ARG
    assert _image(lib, _prob(n_ant=0), _inputs(cable_m=FAKE, ant1=FAKE, ant2=FAKE)) == E_ARG
    a = lib.blink_degrid_adjoint
    inp = _inputs(cable_m=FAKE, ant1=FAKE, ant2=FAKE)
    assert a(ctypes.byref(_prob()), ctypes.byref(inp), FAKE, None, FAKE, None, None, 0, None) == E_WS
    assert a(ctypes.byref(_prob()), ctypes.byref(_inputs(cable_m=FAKE)), FAKE, None, FAKE, None, None, 0,
             None) == E_ARG


def _noalloc(lib, p, inp, images=FAKE):
    return lib.blink_image_batch_noalloc(ctypes.byref(p) if p is not None else None,
                                         ctypes.byref(inp) if inp is not None else None,
                                         images, None, None)


def test_noalloc_validation(lib):
    # the entry point without a workspace: the same argument checks as
    # blink_image_batch, all on the host before the scratch array is touched
    assert _noalloc(lib, None, _inputs()) == E_ARG
    assert _noalloc(lib, _prob(), None) == E_ARG
    assert _noalloc(lib, _prob(), _inputs(vis=None)) == E_ARG
    assert _noalloc(lib, _prob(), _inputs(), images=None) == E_ARG
    assert _noalloc(lib, _prob(grid_n=63), _inputs()) == E_SIZE
    assert _noalloc(lib, _prob(grid_n=1000), _inputs()) == E_UNSUP
    assert _noalloc(lib, _prob(n_time=0), _inputs(vis=None, uvw_m=None, freq_hz=None)) == E_OK
    # one image whose workspace exceeds the 64 MiB array: its half spectrum
    # alone is 2048 x 4096 x 8 B = 64 MiB
    assert B.NOALLOC_SCRATCH_BYTES == 64 << 20
    assert _noalloc(lib, _prob(n_time=1, n_chan=1, grid_n=4096, out_n=4096), _inputs()) == E_WS
