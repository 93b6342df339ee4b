"""Geometric phase rotation at visibility load against the FP64 oracle.

Images with the phase centre rotated away from zenith (with a non-zero w
term) match oracle.phase_rotation within the FP32 bound, for the one-kernel
sort (8128 baselines) and the multi-run sort (32,640 baselines), natural and
uniform weighting and kernel gridding; a source placed at the new centre
images at the image centre with its flux. The cable-length correction, alone
and with a rotation and gains, matches the oracle the same way, and
visibilities correlated from cable-delayed voltages of a zenith source image
at the centre with its flux once corrected. With re-projection onto the new
centre's tangent plane, images (nearest-cell and kernel gridding, one-kernel
and multi-run sorts, the single-image path) match the oracle, re-projection at
zenith changes no bit, and a source at a pixel of the new tangent plane images
there.
"""
import numpy as np
import pytest
import torch

from oracle import phase_rotation as opr
from oracle import kernel_gridding as kg
import paper_2405_13478_amd as blink
from paper_2405_13478_amd import synth

from _gpu_util import REL_L2_FP32, device, inputs, per_image_rel_l2

pytestmark = pytest.mark.gpu


def _with_w(w, seed, scale):
    rng = np.random.default_rng(seed)
    w.uvw_m = w.uvw_m.copy()
    w.uvw_m[..., 2] = rng.uniform(-scale, scale, size=w.uvw_m.shape[:2])
    return w


@pytest.mark.parametrize("name,lm", [("wide512", (0.012, -0.02)), ("allsky180", (0.3, 0.25)),
                                     ("plain128", (-0.2, 0.1))])
def test_rotated_images_match_oracle(name, lm):
    print(f"\n[gpu] phase rotation {name} to {lm}", flush=True)
    if name == "wide512":
        w = synth.widefield(n_time=1, n_chan=2, chan_stride=300)
        w.grid_n, w.out_n = 512, 256
        w.pixscale = synth.oversampled_pixscale(3000.0, float(w.freq_hz.max()))
        w = _with_w(w, 1, 40.0)
    elif name == "allsky180":
        w = _with_w(synth.station_allsky(n_time=1, n_chan=2), 2, 3.0)
    else:
        w = _with_w(synth.plain_single(), 3, 5.0)
    d = inputs(w)
    img = blink.image_batch(d["vis"], d["uvw_m"], d["freq_hz"], grid_n=w.grid_n, pixscale=w.pixscale,
                            out_n=w.out_n, weighting=w.weighting, norm=w.norm, flags=d["flags"], phase_lm=lm)
    torch.cuda.synchronize()
    ref, _ = opr.image_batch_rotated(d["vis"].cpu().numpy(), w.uvw_m, w.freq_hz, w.grid_n, w.pixscale, w.out_n,
                                     w.weighting, w.norm, lm[0], lm[1], w.flags)
    errs = per_image_rel_l2(img.cpu().numpy(), ref)
    print(f"  rel-L2 {max(errs):.2e}", flush=True)
    assert max(errs) <= REL_L2_FP32


def test_rotation_with_kernel_gridding():
    w = _with_w(synth.plain_single(), 4, 5.0)
    w.out_n = 64
    lm = (0.15, -0.05)
    d = inputs(w)
    img = blink.image_batch(d["vis"], d["uvw_m"], d["freq_hz"], grid_n=w.grid_n, pixscale=w.pixscale,
                            out_n=w.out_n, weighting=0, norm=w.norm, kernel_support=6, phase_lm=lm)
    torch.cuda.synchronize()
    v = d["vis"].cpu().numpy()
    rot = np.stack([[opr.rotate(v[t, c], w.uvw_m[t], w.freq_hz[c], *lm) for c in range(w.n_chan)]
                    for t in range(w.n_time)])
    ref, _ = kg.image_batch_conv(rot, w.uvw_m, w.freq_hz, w.grid_n, w.pixscale, w.out_n, w.norm, 6)
    assert max(per_image_rel_l2(img.cpu().numpy(), ref)) <= REL_L2_FP32


def test_source_at_new_centre_images_at_centre():
    w = _with_w(synth.plain_single(), 5, 5.0)
    l0, m0 = 0.23, -0.11
    n0 = np.sqrt(1 - l0 ** 2 - m0 ** 2)
    lam = synth.C_LIGHT / w.freq_hz[0]
    uvw = w.uvw_m[0]
    v = 2.5 * np.exp(-2j * np.pi * (uvw[:, 0] * l0 + uvw[:, 1] * m0 + uvw[:, 2] * (n0 - 1)) / lam)
    dev = device()
    img = blink.image_batch(torch.from_numpy(v.astype(np.complex64)[None, None]).to(dev),
                            torch.from_numpy(w.uvw_m).to(dev), torch.from_numpy(w.freq_hz).to(dev),
                            grid_n=w.grid_n, pixscale=w.pixscale, out_n=w.out_n, weighting=0, norm=1,
                            phase_lm=(l0, m0))
    torch.cuda.synchronize()
    im = img[0].cpu().numpy()
    n = w.out_n
    assert np.unravel_index(np.argmax(im), im.shape) == (n // 2, n // 2)
    assert abs(im[n // 2, n // 2] - 2.5) <= 1e-5 * 2.5


# ------------------------------------------------------------ cable correction
def _cables(w, seed):
    return np.random.default_rng(seed).uniform(0.0, 400.0, w.n_ant)


@pytest.mark.parametrize("name,lm", [("wide512", (0.012, -0.02)), ("allsky180", (0.0, 0.0)),
                                     ("plain128", (-0.2, 0.1))])
def test_cable_corrected_images_match_oracle(name, lm):
    """Cable lengths alone (all-sky: multi-run sort, uniform weighting, flags)
    and together with a rotation (512^2 also with per-antenna gains)."""
    print(f"\n[gpu] cable correction {name}, rotation {lm}", flush=True)
    if name == "wide512":
        w = synth.widefield(n_time=1, n_chan=2, chan_stride=300)
        w.grid_n, w.out_n = 512, 256
        w.pixscale = synth.oversampled_pixscale(3000.0, float(w.freq_hz.max()))
        w = _with_w(w, 11, 40.0)
    elif name == "allsky180":
        w = synth.station_allsky(n_time=1, n_chan=2)
    else:
        w = _with_w(synth.plain_single(), 13, 5.0)
    gains = name == "wide512"
    d = inputs(w, with_gains=gains)
    dev = device()
    cab = _cables(w, 17)
    ant1 = d.get("ant1", torch.from_numpy(w.ant1).to(dev))
    ant2 = d.get("ant2", torch.from_numpy(w.ant2).to(dev))
    img = blink.image_batch(d["vis"], d["uvw_m"], d["freq_hz"], grid_n=w.grid_n, pixscale=w.pixscale,
                            out_n=w.out_n, weighting=w.weighting, norm=w.norm, flags=d["flags"],
                            gains=d.get("gains"), ant1=ant1, ant2=ant2, phase_lm=lm,
                            cable_m=torch.from_numpy(cab).to(dev))
    torch.cuda.synchronize()
    ref, _ = opr.image_batch_rotated(d["vis"].cpu().numpy(), w.uvw_m, w.freq_hz, w.grid_n, w.pixscale,
                                     w.out_n, w.weighting, w.norm, lm[0], lm[1], w.flags,
                                     w.gains if gains else None, w.ant1, w.ant2, cable_m=cab)
    errs = per_image_rel_l2(img.cpu().numpy(), ref)
    print(f"  rel-L2 {max(errs):.2e}", flush=True)
    assert max(errs) <= REL_L2_FP32, errs


def test_cable_delayed_voltages_image_at_centre():
    # visibilities correlated from cable-delayed voltages of a zenith source:
    # corrected on the GPU, the source images at the centre with its flux
    w = synth.plain_single()
    cab = _cables(w, 19)
    freq = float(w.freq_hz[0])
    x = 1.5 * np.exp(-2j * np.pi * freq * cab / synth.C_LIGHT)
    v = (x[w.ant1] * np.conj(x[w.ant2])).astype(np.complex64)
    dev = device()
    img = blink.image_batch(torch.from_numpy(v[None, None]).to(dev), torch.from_numpy(w.uvw_m).to(dev),
                            torch.from_numpy(w.freq_hz).to(dev), grid_n=w.grid_n, pixscale=w.pixscale,
                            out_n=w.out_n, weighting=0, norm=1, ant1=torch.from_numpy(w.ant1).to(dev),
                            ant2=torch.from_numpy(w.ant2).to(dev), cable_m=torch.from_numpy(cab).to(dev))
    torch.cuda.synchronize()
    im = img[0].cpu().numpy()
    n = w.out_n
    assert np.unravel_index(np.argmax(im), im.shape) == (n // 2, n // 2)
    assert abs(im[n // 2, n // 2] - 2.25) <= 1e-5 * 2.25


# ------------------------------------------------------------ re-projection
@pytest.mark.parametrize("name,lm", [("wide512", (0.3, -0.2)), ("allsky180", (0.45, 0.3)),
                                     ("plain128", (-0.5, 0.4))])
def test_reprojected_images_match_oracle(name, lm):
    print(f"\n[gpu] re-projection {name} to {lm}", flush=True)
    if name == "wide512":
        w = synth.widefield(n_time=1, n_chan=2, chan_stride=300)
        w.grid_n, w.out_n = 512, 256
        w.pixscale = synth.oversampled_pixscale(3000.0, float(w.freq_hz.max()))
        w = _with_w(w, 6, 40.0)
    elif name == "allsky180":
        w = _with_w(synth.station_allsky(n_time=1, n_chan=2), 7, 3.0)
    else:
        w = _with_w(synth.plain_single(), 8, 5.0)
    d = inputs(w)
    img = blink.image_batch(d["vis"], d["uvw_m"], d["freq_hz"], grid_n=w.grid_n, pixscale=w.pixscale,
                            out_n=w.out_n, weighting=w.weighting, norm=w.norm, flags=d["flags"], phase_lm=lm,
                            reproject=True)
    torch.cuda.synchronize()
    ref, _ = opr.image_batch_rotated(d["vis"].cpu().numpy(), w.uvw_m, w.freq_hz, w.grid_n, w.pixscale, w.out_n,
                                     w.weighting, w.norm, lm[0], lm[1], w.flags, reproject=True)
    errs = per_image_rel_l2(img.cpu().numpy(), ref)
    print(f"  rel-L2 {max(errs):.2e}", flush=True)
    assert max(errs) <= REL_L2_FP32


def test_reprojection_with_kernel_gridding():
    w = _with_w(synth.plain_single(), 9, 5.0)
    w.out_n = 64
    lm = (0.35, -0.15)
    d = inputs(w)
    img = blink.image_batch(d["vis"], d["uvw_m"], d["freq_hz"], grid_n=w.grid_n, pixscale=w.pixscale,
                            out_n=w.out_n, weighting=1, norm=w.norm, kernel_support=6, phase_lm=lm,
                            reproject=True)
    torch.cuda.synchronize()
    v = d["vis"].cpu().numpy()
    rot = np.stack([[opr.rotate(v[t, c], w.uvw_m[t], w.freq_hz[c], *lm) for c in range(w.n_chan)]
                    for t in range(w.n_time)])
    uvw_p = np.stack([opr.plane_uvw(w.uvw_m[t], lm[0], lm[1], True) for t in range(w.n_time)])
    ref, _ = kg.image_batch_conv(rot, uvw_p, w.freq_hz, w.grid_n, w.pixscale, w.out_n, w.norm, 6,
                                 weighting=1)
    assert max(per_image_rel_l2(img.cpu().numpy(), ref)) <= REL_L2_FP32


def test_reprojection_at_zenith_changes_no_bit():
    w = _with_w(synth.station_allsky(n_time=1, n_chan=2), 10, 3.0)
    d = inputs(w)
    kw = dict(grid_n=w.grid_n, pixscale=w.pixscale, out_n=w.out_n, weighting=w.weighting, norm=w.norm,
              flags=d["flags"], phase_lm=(0.0, 0.0))
    a = blink.image_batch(d["vis"], d["uvw_m"], d["freq_hz"], reproject=True, **kw)
    b = blink.image_batch(d["vis"], d["uvw_m"], d["freq_hz"], **kw)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_reprojected_source_images_at_its_tangent_plane_pixel():
    # baselines perpendicular to s0 (w' = 0; w != 0 in the zenith frame): a
    # source at a pixel of the new tangent plane peaks at that pixel
    n, pix = 64, 1.0 / (3 * 24.0)
    l0, m0 = 0.45, 0.3
    R = opr.reprojection_matrix(l0, m0)
    rng = np.random.default_rng(11)
    xy = rng.uniform(-12, 12, size=(400, 2))
    uvw = xy[:, :1] * R[:, 0] + xy[:, 1:] * R[:, 1]
    lp, mp = 18 * pix, -12 * pix
    s = R @ np.array([lp, mp, np.sqrt(1 - lp ** 2 - mp ** 2)])
    v = 2.5 * np.exp(-2j * np.pi * (uvw @ (s - np.array([0.0, 0.0, 1.0]))))
    dev = device()
    img = blink.image_batch(torch.from_numpy(v.astype(np.complex64)[None, None]).to(dev),
                            torch.from_numpy(uvw[None]).to(dev),
                            torch.tensor([synth.C_LIGHT], dtype=torch.float64, device=dev),
                            grid_n=n, pixscale=pix, out_n=n, weighting=0, norm=1, phase_lm=(l0, m0),
                            reproject=True)
    torch.cuda.synchronize()
    im = img[0].cpu().numpy()
    assert np.unravel_index(np.argmax(im), im.shape) == (n // 2 - 12, n // 2 + 18)
