"""Kaiser-Bessel kernel gridding on the GPU against the FP64 kernel oracle.

Images (including the taper correction), weight sums and the gridded cells
are compared with oracle.kernel_gridding on the same seeded inputs; the box
kernel of width one must reproduce nearest-cell gridding (natural and
uniform weighting); results are bitwise repeatable and independent of the
chunking. Uniform weighting with a kernel follows oracle.kernel_gridding's
reading: each baseline's weights are divided by the number of kept entries at
its nearest cell.
"""
import numpy as np
import pytest
import torch

from oracle import kernel_gridding as kg
import paper_2405_13478_amd as blink
from paper_2405_13478_amd import synth

from _gpu_util import REL_L2_FP32, device, inputs, per_image_rel_l2

pytestmark = pytest.mark.gpu


def _case(name):
    if name == "plain128":
        w = synth.plain_single()
        w.out_n = 64
    elif name == "allsky180":
        w = synth.station_allsky(n_time=2, n_chan=2)
        w.weighting = 0
    elif name == "wide512":
        w = synth.widefield(n_time=1, n_chan=2, chan_stride=300)
        w.grid_n, w.out_n = 512, 256
        w.pixscale = synth.oversampled_pixscale(3000.0, float(w.freq_hz.max()))
    else:
        raise ValueError(name)
    return w


def _run(w, d, support, beta=-1.0, weighting=0, **kw):
    ws = torch.empty(w.n_img, dtype=torch.float32, device=d["vis"].device)
    img = blink.image_batch(d["vis"], d["uvw_m"], d["freq_hz"], grid_n=w.grid_n, pixscale=w.pixscale,
                            out_n=w.out_n, weighting=weighting, norm=w.norm, flags=d.get("flags"),
                            weight_sum=ws, kernel_support=support, kernel_beta=beta, **kw)
    torch.cuda.synchronize()
    return img, ws


# W <= 8 takes the short footprint form, W = 12 the long one
@pytest.mark.parametrize("name,support", [("plain128", 4), ("plain128", 6), ("plain128", 12),
                                          ("allsky180", 4), ("wide512", 6), ("wide512", 8)])
def test_kernel_image_parity(name, support):
    print(f"\n[gpu] kernel gridding {name} W={support}", flush=True)
    w = _case(name)
    d = inputs(w)
    img, ws = _run(w, d, support)
    ref, W = kg.image_batch_conv(d["vis"].cpu().numpy(), w.uvw_m, w.freq_hz, w.grid_n, w.pixscale,
                                 w.out_n, w.norm, support, None, w.flags)
    errs = per_image_rel_l2(img.cpu().numpy(), ref)
    print(f"  rel-L2 {max(errs):.2e}", flush=True)
    assert max(errs) <= REL_L2_FP32, errs
    assert np.allclose(ws.cpu().numpy(), W, rtol=2e-6, atol=0), (ws.cpu().numpy(), W)


def test_explicit_beta_and_unnormalised():
    w = _case("plain128")
    w.norm = 0
    d = inputs(w)
    img, _ = _run(w, d, 5, beta=7.5)
    ref, _ = kg.image_batch_conv(d["vis"].cpu().numpy(), w.uvw_m, w.freq_hz, w.grid_n, w.pixscale,
                                 w.out_n, 0, 5, 7.5, w.flags)
    assert max(per_image_rel_l2(img.cpu().numpy(), ref)) <= REL_L2_FP32


def test_very_sharp_kernel_takes_the_bessel_routine():
    # beta = 80 (the largest accepted) needs more polynomial terms than the
    # library keeps, so the weights come from cyl_bessel_i0f: same parity bar
    w = _case("plain128")
    d = inputs(w)
    img, ws = _run(w, d, 12, beta=80.0)
    ref, W = kg.image_batch_conv(d["vis"].cpu().numpy(), w.uvw_m, w.freq_hz, w.grid_n, w.pixscale,
                                 w.out_n, w.norm, 12, 80.0, w.flags)
    assert max(per_image_rel_l2(img.cpu().numpy(), ref)) <= REL_L2_FP32
    assert np.allclose(ws.cpu().numpy(), W, rtol=2e-6, atol=0)


def test_box_kernel_of_width_one_grids_like_nearest_cell():
    w = _case("allsky180")
    d = inputs(w)
    kw = dict(grid_n=w.grid_n, pixscale=w.pixscale, weighting=0, flags=d["flags"])
    g0, c0, w0, n0 = blink.grid(d["vis"], d["uvw_m"], d["freq_hz"], **kw)
    g1, c1, w1, n1 = blink.grid(d["vis"], d["uvw_m"], d["freq_hz"], kernel_support=1, kernel_beta=0.0, **kw)
    torch.cuda.synchronize()
    assert torch.equal(c0, c1)
    assert torch.equal(n0, n1)
    assert torch.equal(w0, w1)
    # same entries added in the same order with weight 1.0 exactly
    assert torch.equal(g0, g1)


def test_kernel_grid_cells_match_oracle():
    w = _case("plain128")
    d = inputs(w)
    support = 6
    g, c, W, nd = blink.grid(d["vis"], d["uvw_m"], d["freq_hz"], grid_n=w.grid_n, pixscale=w.pixscale,
                             weighting=0, kernel_support=support, kernel_beta=-1.0)
    torch.cuda.synchronize()
    beta = kg.kb_default_beta(support)
    r = kg.image_one_conv(d["vis"].cpu().numpy()[0, 0], w.uvw_m[0, :, 0], w.uvw_m[0, :, 1], w.freq_hz[0],
                          w.grid_n, w.pixscale, w.grid_n, 0, support, beta)
    assert np.array_equal(c.cpu().numpy()[0], r["counts"])
    S = r["S"]
    got = g.cpu().numpy()[0].astype(np.complex128)
    assert np.linalg.norm(got - S) <= 2e-6 * np.linalg.norm(S)
    assert abs(float(W.cpu()[0]) - r["W"]) <= 2e-6 * r["W"]
    assert int(nd.cpu()[0]) == int((~r["keep"]).sum())


def test_kernel_bitwise_repeatable_and_chunk_invariant():
    w = _case("allsky180")
    d = inputs(w)
    a, wa = _run(w, d, 4)
    b, wb = _run(w, d, 4)
    c, wc = _run(w, d, 4, chunk_images=1)
    assert torch.equal(a, b) and torch.equal(a, c)
    assert torch.equal(wa, wb) and torch.equal(wa, wc)


def test_kernel_widefield_fullsize_sampled():
    print("\n[gpu] kernel gridding widefield 1024 -> 512, W=6, sampled", flush=True)
    w = synth.widefield(n_time=1, n_chan=768)
    dev = device()
    vis = synth.visibilities(w, device=dev)
    uvw = torch.from_numpy(w.uvw_m).to(dev)
    freq = torch.from_numpy(w.freq_hz).to(dev)
    ws = torch.empty(w.n_img, dtype=torch.float32, device=dev)
    img = blink.image_batch(vis, uvw, freq, grid_n=w.grid_n, pixscale=w.pixscale, out_n=w.out_n,
                            weighting=0, norm=w.norm, weight_sum=ws, kernel_support=6)
    torch.cuda.synchronize()
    assert torch.isfinite(img).all()
    sample = [0, 767]
    ref, W = kg.image_batch_conv(vis.cpu().numpy(), w.uvw_m, w.freq_hz, w.grid_n, w.pixscale, w.out_n,
                                 w.norm, 6, None, None, images=sample)
    errs = per_image_rel_l2(img[sample].cpu().numpy(), ref)
    print(f"  sampled rel-L2: {[f'{e:.2e}' for e in errs]}", flush=True)
    assert max(errs) <= REL_L2_FP32
    assert np.allclose(ws.cpu().numpy()[sample], W, rtol=2e-6, atol=0)


@pytest.mark.parametrize("name,support", [("plain128", 4), ("allsky180", 6), ("wide512", 6)])
def test_uniform_kernel_image_parity(name, support):
    print(f"\n[gpu] kernel gridding, uniform weighting, {name} W={support}", flush=True)
    w = _case(name)
    d = inputs(w)
    img, ws = _run(w, d, support, weighting=1)
    ref, W = kg.image_batch_conv(d["vis"].cpu().numpy(), w.uvw_m, w.freq_hz, w.grid_n, w.pixscale,
                                 w.out_n, w.norm, support, None, w.flags, weighting=1)
    errs = per_image_rel_l2(img.cpu().numpy(), ref)
    print(f"  rel-L2 {max(errs):.2e}", flush=True)
    assert max(errs) <= REL_L2_FP32, errs
    assert np.allclose(ws.cpu().numpy(), W, rtol=2e-6, atol=0), (ws.cpu().numpy(), W)


def test_uniform_kernel_grid_cells_match_oracle():
    w = _case("allsky180")
    d = inputs(w)
    support = 6
    g, c, W, nd = blink.grid(d["vis"], d["uvw_m"], d["freq_hz"], grid_n=w.grid_n, pixscale=w.pixscale,
                             weighting=1, flags=d["flags"], kernel_support=support, kernel_beta=-1.0)
    torch.cuda.synchronize()
    beta = kg.kb_default_beta(support)
    vis = d["vis"].cpu().numpy()
    for i in range(w.n_img):
        t, ch = divmod(i, w.n_chan)
        r = kg.image_one_conv(vis[t, ch], w.uvw_m[t, :, 0], w.uvw_m[t, :, 1], w.freq_hz[ch], w.grid_n,
                              w.pixscale, w.grid_n, 0, support, beta, flagged=w.flags[t], weighting=1)
        assert np.array_equal(c.cpu().numpy()[i], r["counts"])
        S = r["S"]
        got = g.cpu().numpy()[i].astype(np.complex128)
        assert np.linalg.norm(got - S) <= 2e-6 * np.linalg.norm(S)
        assert abs(float(W.cpu()[i]) - r["W"]) <= 2e-6 * r["W"]
        # dropped: unflagged baselines outside the grid
        assert int(nd.cpu()[i]) == int((~r["keep"] & ~w.flags[t]).sum())


def test_uniform_box_kernel_of_width_one_grids_like_nearest_cell_uniform():
    w = _case("allsky180")
    d = inputs(w)
    kw = dict(grid_n=w.grid_n, pixscale=w.pixscale, weighting=1, flags=d["flags"])
    g0, c0, w0, n0 = blink.grid(d["vis"], d["uvw_m"], d["freq_hz"], **kw)
    g1, c1, w1, n1 = blink.grid(d["vis"], d["uvw_m"], d["freq_hz"], kernel_support=1, kernel_beta=0.0, **kw)
    torch.cuda.synchronize()
    assert torch.equal(c0, c1)
    assert torch.equal(n0, n1)
    # W: occupied cells (nearest cell) against the sum of 1/n over the entries
    assert torch.allclose(w0, w1, rtol=1e-6, atol=0)
    # sum / n against the sum of V / n: equal up to rounding
    for i in range(w.n_img):
        a, b = g0[i].cpu().numpy(), g1[i].cpu().numpy()
        assert np.linalg.norm(a - b) <= 1e-6 * np.linalg.norm(a)


def test_uniform_kernel_bitwise_repeatable_and_chunk_invariant():
    w = _case("allsky180")
    d = inputs(w)
    a, wa = _run(w, d, 4, weighting=1)
    b, wb = _run(w, d, 4, weighting=1)
    c, wc = _run(w, d, 4, weighting=1, chunk_images=1)
    assert torch.equal(a, b) and torch.equal(a, c)
    assert torch.equal(wa, wb) and torch.equal(wa, wc)


def test_uniform_kernel_widefield_fullsize_sampled():
    print("\n[gpu] kernel gridding, uniform weighting, widefield 1024 -> 512, W=6, sampled", flush=True)
    w = synth.widefield(n_time=1, n_chan=768)
    dev = device()
    vis = synth.visibilities(w, device=dev)
    uvw = torch.from_numpy(w.uvw_m).to(dev)
    freq = torch.from_numpy(w.freq_hz).to(dev)
    ws = torch.empty(w.n_img, dtype=torch.float32, device=dev)
    img = blink.image_batch(vis, uvw, freq, grid_n=w.grid_n, pixscale=w.pixscale, out_n=w.out_n,
                            weighting=1, norm=w.norm, weight_sum=ws, kernel_support=6)
    torch.cuda.synchronize()
    assert torch.isfinite(img).all()
    sample = [383]
    ref, W = kg.image_batch_conv(vis.cpu().numpy(), w.uvw_m, w.freq_hz, w.grid_n, w.pixscale, w.out_n,
                                 w.norm, 6, None, None, images=sample, weighting=1)
    errs = per_image_rel_l2(img[sample].cpu().numpy(), ref)
    print(f"  sampled rel-L2: {[f'{e:.2e}' for e in errs]}", flush=True)
    assert max(errs) <= REL_L2_FP32
    assert np.allclose(ws.cpu().numpy()[sample], W, rtol=2e-6, atol=0)
