"""GPU check of blink_image_batch_noalloc, the entry point that allocates
nothing (its scratch is a fixed per-GPU array in the library): on the same
inputs it gives the same images and weight sums as blink_image_batch, bit
for bit, on two calls in a row (the second on a smaller input, which finds
the first call's data still in the array), including a cube that is imaged
in several timestep blocks. The images also match the FP64 oracle on
sampled images."""
import numpy as np
import pytest
import torch

import paper_2405_13478_amd as blink
from paper_2405_13478_amd import synth

from _gpu_util import REL_L2_FP32, inputs, oracle_images, rel_l2, run_image

pytestmark = pytest.mark.gpu


def _noalloc(w, d, images, ws):
    blink.image_batch_noalloc(images, d["vis"], d["uvw_m"], d["freq_hz"], grid_n=w.grid_n,
                              pixscale=w.pixscale, out_n=w.out_n, weighting=w.weighting, norm=w.norm,
                              flags=d.get("flags"), weight_sum=ws)
    torch.cuda.synchronize()


def _check(w, d, sample):
    ref_img, ref_w = run_image(w, d)
    n_img, M = w.n_img, w.out_n
    # outputs pre-filled with garbage: every element must be written
    img = torch.full((n_img, M, M), float("nan"), dtype=torch.float32, device=d["vis"].device)
    ws = torch.full((n_img,), float("nan"), dtype=torch.float32, device=d["vis"].device)
    _noalloc(w, d, img, ws)
    assert torch.equal(img, ref_img)
    assert torch.equal(ws, ref_w)
    vis_np = d["vis"].cpu().numpy()
    orc, orc_w = oracle_images(w, vis_np, sample)
    got = img.cpu().numpy()
    for k, i in enumerate(sample):
        assert rel_l2(got[i], orc[k]) <= REL_L2_FP32
        assert ws[i].item() == orc_w[k]


def test_noalloc_two_calls_second_smaller():
    # 1: all-sky 180^2, uniform, flags, 40 timesteps x 2 channels: the sorted
    #    lists of 40 timesteps of 32640 baselines exceed the 64 MiB array, so
    #    the cube is imaged in blocks of 20 timesteps
    w1 = synth.station_allsky(n_time=40, n_chan=2)
    d1 = inputs(w1)
    print(f"\n[gpu] noalloc call 1: all-sky 40 x 2 images of 180^2", flush=True)
    _check(w1, d1, [0, 41, 79])
    # 2: widefield 1024^2 -> 512^2, 1 timestep x 40 channels (smaller input;
    #    several 2 MiB half spectra per chunk)
    w2 = synth.widefield(n_time=1, n_chan=40, chan_stride=19)
    d2 = inputs(w2)
    print(f"[gpu] noalloc call 2: widefield 1 x 40 images of 1024^2 -> 512^2", flush=True)
    _check(w2, d2, [0, 39])


def test_noalloc_repeat_and_chunk_bound():
    # the same input twice more, with a chunk bound of 3 images: same bits
    w = synth.widefield(n_time=1, n_chan=8, chan_stride=90)
    d = inputs(w)
    ref, ref_w = run_image(w, d)
    for chunk in (0, 3):
        img = torch.empty_like(ref)
        ws = torch.empty_like(ref_w)
        blink.image_batch_noalloc(img, d["vis"], d["uvw_m"], d["freq_hz"], grid_n=w.grid_n,
                                  pixscale=w.pixscale, out_n=w.out_n, weighting=w.weighting,
                                  norm=w.norm, chunk_images=chunk, weight_sum=ws)
        torch.cuda.synchronize()
        assert torch.equal(img, ref) and torch.equal(ws, ref_w)
