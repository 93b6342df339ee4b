"""Correlator X-engine on the matrix cores against the integer oracle.

Sums of 8-bit products are exact integers on both sides, so visibilities and
autocorrelations must equal the oracle's values rounded to float bit for bit,
including blocks of antennas and samples that are only partly filled, the
most negative 8-bit value and sums beyond 2^24. Voltages of a plane wave,
correlated and then imaged by the library, must peak at the wave's direction.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import correlator as xc
import paper_2405_13478_amd as blink

from _gpu_util import device

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("T,C,A,S", [(2, 3, 37, 48), (1, 1, 2, 16), (2, 2, 64, 1024), (1, 1, 256, 256),
                                     (1, 2, 33, 32), (3, 1, 100, 0), (1, 1, 130, 208), (2, 1, 17, 80)])
def test_correlate_matches_oracle(T, C, A, S):
    print(f"\n[gpu] correlate T={T} C={C} A={A} S={S}", flush=True)
    rng = np.random.default_rng(A * 1000 + S + T)
    volt = rng.integers(-128, 128, size=(T, C, A, S, 2)).astype(np.int8)
    vis, autos = blink.correlate(torch.from_numpy(volt).to(device()), autos=True)
    torch.cuda.synchronize()
    rv, ra = xc.correlate(volt)
    got = vis.cpu().numpy()
    assert np.array_equal(got.real, rv.real.astype(np.float32))
    assert np.array_equal(got.imag, rv.imag.astype(np.float32))
    assert np.array_equal(autos.cpu().numpy(), ra.astype(np.float32))


def test_correlate_extremes_beyond_float_precision():
    # -128 everywhere: Re V = 2 * 16384 * S = 33,554,432 for S = 1024 (> 2^24), Im V = 0
    volt = np.full((1, 1, 40, 1024, 2), -128, dtype=np.int8)
    volt[0, 0, 5, :, 1] = 127
    vis, autos = blink.correlate(torch.from_numpy(volt).to(device()), autos=True)
    torch.cuda.synchronize()
    rv, ra = xc.correlate(volt)
    got = vis.cpu().numpy()
    assert np.array_equal(got.real, rv.real.astype(np.float32))
    assert np.array_equal(got.imag, rv.imag.astype(np.float32))
    assert np.array_equal(autos.cpu().numpy(), ra.astype(np.float32))


def test_correlate_largest_sample_count_stays_exact():
    # -128 everywhere at the largest accepted count: RR + QQ = 2 * 16384 * 65520,
    # just below 2^31, so the int32 sums must not wrap
    S = 65520
    volt = np.full((1, 1, 20, S, 2), -128, dtype=np.int8)
    volt[0, 0, 3, ::7, 0] = 127
    vis, autos = blink.correlate(torch.from_numpy(volt).to(device()), autos=True)
    torch.cuda.synchronize()
    rv, ra = xc.correlate(volt)
    assert ra.max() == 2 * 16384 * S
    got = vis.cpu().numpy()
    assert np.array_equal(got.real, rv.real.astype(np.float32))
    assert np.array_equal(got.imag, rv.imag.astype(np.float32))
    assert np.array_equal(autos.cpu().numpy(), ra.astype(np.float32))


def test_correlated_plane_wave_images_at_its_direction():
    rng = np.random.default_rng(12)
    A, S, n = 48, 512, 64
    xy = rng.uniform(-10, 10, size=(A, 2))
    pix = 1.0 / (3 * 40.0)
    ql, qm = 9, -6
    l, m = ql * pix, qm * pix
    sig = rng.normal(size=S) + 1j * rng.normal(size=S)
    x = sig[None, :] * np.exp(2j * np.pi * (xy[:, 0] * l + xy[:, 1] * m))[:, None]
    volt = np.stack([np.round(20 * x.real), np.round(20 * x.imag)], axis=-1).astype(np.int8)[None, None]
    dev = device()
    vis, _ = blink.correlate(torch.from_numpy(volt).to(dev))
    a1, a2 = np.triu_indices(A, k=1)
    d = xy[a2] - xy[a1]
    uvw = np.zeros((1, len(a1), 3))
    uvw[0, :, :2] = d
    img = blink.image_batch(vis, torch.from_numpy(uvw).to(dev), torch.tensor([oracle.C_LIGHT], dtype=torch.float64,
                            device=dev), grid_n=n, pixscale=pix, out_n=n, weighting=0, norm=1)
    torch.cuda.synchronize()
    im = img[0].cpu().numpy()
    assert np.unravel_index(np.argmax(im), im.shape) == (n // 2 + qm, n // 2 + ql)
