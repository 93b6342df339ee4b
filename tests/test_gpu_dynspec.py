"""Dynamic spectra with reference subtraction on the GPU against the FP64 oracle.

Transposition and the model / preceding-image references are one rounding
of the exact value, so they must match the oracle rounded to FP32 bit for bit;
a mean over several preceding images is evaluated in double on both sides and
may differ by one unit in the last place. Sizes cover ragged tiles in time
and pixels, windows up to the maximum, and a cube of real dirty images.
"""
import numpy as np
import pytest
import torch

from oracle import dynamic_spectra as ods
import paper_2405_13478_amd as blink
from paper_2405_13478_amd import synth

from _gpu_util import device

pytestmark = pytest.mark.gpu


def _cube(T, C, M, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(T, C, M, M)).astype(np.float32)


def _check(got, ref64, exact):
    ref = ref64.astype(np.float32)
    if exact:
        assert np.array_equal(got, ref)
    else:
        assert np.all(np.abs(got - ref) <= np.spacing(np.abs(ref)))


# (T, P) multiples of 4 take the 16-byte path: (64, 2, 8), (132, 2, 12), (256, 1, 10)
@pytest.mark.parametrize("T,C,M", [(70, 3, 10), (64, 2, 8), (5, 4, 16), (130, 1, 6), (132, 2, 12),
                                   (256, 1, 10)])
@pytest.mark.parametrize("mode,K", [(0, 1), (1, 1), (1, 5), (1, 64), (1, 128), (2, 1)])
def test_dynspec_matches_oracle(T, C, M, mode, K):
    print(f"\n[gpu] dynspec T={T} C={C} M={M} mode={mode} K={K}", flush=True)
    dev = device()
    I = _cube(T, C, M, 100 + T + C + M)
    R = _cube(1, C, M, 7)[0] if mode == 2 else None
    got = blink.dynamic_spectra(torch.from_numpy(I).to(dev), mode, K,
                                None if R is None else torch.from_numpy(R).to(dev))
    torch.cuda.synchronize()
    ref = ods.dynamic_spectra(I, mode, K, R)
    _check(got.cpu().numpy(), ref, exact=(mode != 1 or K == 1))


def test_dynspec_of_dirty_images():
    print("\n[gpu] dynspec of widefield dirty images, 72 timesteps x 8 channels, 512^2", flush=True)
    dev = device()
    w = synth.widefield(n_time=72, n_chan=8, chan_stride=96)
    vis = synth.visibilities(w, device=dev)
    img = blink.image_batch(vis, torch.from_numpy(w.uvw_m).to(dev), torch.from_numpy(w.freq_hz).to(dev),
                            grid_n=w.grid_n, pixscale=w.pixscale, out_n=w.out_n, weighting=w.weighting,
                            norm=w.norm)
    cube = img.view(w.n_time, w.n_chan, w.out_n, w.out_n)
    S = blink.dynamic_spectra(cube, blink.REF_MEAN, 8)
    torch.cuda.synchronize()
    rows = [0, 255, 256, 511]
    sub = cube[:, :, rows, :].cpu().numpy()                           # [T][C][4][512]
    ref = ods.dynamic_spectra(sub.reshape(w.n_time, w.n_chan, -1), ods.REF_MEAN, 8)   # [4*512][C][T]
    got = S.view(w.out_n, w.out_n, w.n_chan, w.n_time)[rows].reshape(-1, w.n_chan, w.n_time)
    _check(got.cpu().numpy(), ref, exact=False)
    # the transposition alone moves every value unchanged
    S0 = blink.dynamic_spectra(cube, blink.REF_NONE)
    torch.cuda.synchronize()
    assert torch.equal(S0.view(w.out_n * w.out_n, w.n_chan, w.n_time).permute(2, 1, 0).reshape(cube.shape), cube)
