"""GPU parity of the adjoint (degridding + forward transforms) and of the
autograd wrapper against the FP64 oracle's adjoint, which is itself pinned by
the dot-product test and central finite differences."""
import numpy as np
import pytest
import torch

import oracle
import paper_2405_13478_amd as blink
from paper_2405_13478_amd import synth

from _gpu_util import device, inputs, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu] {request.node.name}", flush=True)
    yield


def _case(name):
    if name == "wide1024_gains":
        return synth.widefield(n_time=1, n_chan=2, chan_stride=383), True
    if name == "allsky180_uniform":
        return synth.station_allsky(n_time=2, n_chan=2), False
    if name == "subset64_gains":
        w = synth.subset_antennas(synth.widefield(n_time=1, n_chan=1), 16, 64)
        return w, True
    raise KeyError(name)


def _adjoint_both(w, d, use_g, gbar):
    vg, gg = blink.degrid_adjoint(gbar, d["vis"], d["uvw_m"], d["freq_hz"], grid_n=w.grid_n,
                                  pixscale=w.pixscale, out_n=w.out_n, weighting=w.weighting,
                                  norm=w.norm, flags=d["flags"], gains=d.get("gains"),
                                  ant1=d.get("ant1"), ant2=d.get("ant2"))
    torch.cuda.synchronize()
    vis = d["vis"].cpu().numpy()
    rv, rg = oracle.adjoint_batch(gbar.cpu().numpy().astype(np.float64), vis, w.uvw_m, w.freq_hz,
                                  w.grid_n, w.pixscale, w.weighting, w.norm, w.flags,
                                  w.gains if use_g else None, w.ant1, w.ant2)
    return vg, gg, rv, rg


@pytest.mark.parametrize("name", ["wide1024_gains", "allsky180_uniform", "subset64_gains"])
def test_adjoint_vs_oracle(name):
    w, use_g = _case(name)
    d = inputs(w, with_gains=use_g)
    rng = np.random.default_rng(17)
    gbar = torch.from_numpy(rng.normal(size=(w.n_img, w.out_n, w.out_n)).astype(np.float32)).to(device())
    vg, gg, rv, rg = _adjoint_both(w, d, use_g, gbar)
    e = rel_l2(vg.cpu().numpy().view(np.float32), rv.view(np.float64))
    print(f"  vis_grad rel-L2 {e:.2e}", flush=True)
    assert e <= 1e-5
    if use_g:
        eg = rel_l2(gg.cpu().numpy().view(np.float32), rg.view(np.float64))
        print(f"  gain_grad rel-L2 {eg:.2e}", flush=True)
        assert eg <= 1e-5


def test_adjoint_dot_product_on_gpu():
    w = synth.widefield(n_time=1, n_chan=2, chan_stride=200)
    d = inputs(w)
    img = blink.image_batch(d["vis"], d["uvw_m"], d["freq_hz"], grid_n=w.grid_n, pixscale=w.pixscale,
                            out_n=w.out_n, weighting=w.weighting, norm=w.norm)
    rng = np.random.default_rng(3)
    gbar = torch.from_numpy(rng.normal(size=img.shape).astype(np.float32)).to(device())
    vg, _ = blink.degrid_adjoint(gbar, d["vis"], d["uvw_m"], d["freq_hz"], grid_n=w.grid_n,
                                 pixscale=w.pixscale, out_n=w.out_n, weighting=w.weighting, norm=w.norm)
    lhs = (img.double() * gbar.double()).sum().item()
    v = d["vis"]
    rhs = (vg.real.double() * v.real.double() + vg.imag.double() * v.imag.double()).sum().item()
    assert abs(lhs - rhs) <= 1e-5 * max(abs(lhs), 1e-30)


def test_autograd_matches_oracle_gradient():
    w, _ = _case("subset64_gains")
    d = inputs(w, with_gains=True)
    vis = d["vis"].clone().requires_grad_(True)
    gains = d["gains"].clone().requires_grad_(True)
    rng = np.random.default_rng(8)
    target = torch.from_numpy(rng.normal(size=(w.n_img, w.out_n, w.out_n)).astype(np.float32)).to(device())
    img = blink.blink_image(vis, gains, d["uvw_m"], d["freq_hz"], d["ant1"], d["ant2"],
                            grid_n=w.grid_n, pixscale=w.pixscale, out_n=w.out_n,
                            weighting=w.weighting, norm=w.norm)
    loss = ((img - target) ** 2).sum()
    loss.backward()
    # the oracle gradient of the same loss; the oracle's adjoint is pinned on the CPU by
    # FP64 central finite differences on this same 16-antenna 64^2 subset
    vnp = d["vis"].cpu().numpy()
    ref_img, _ = oracle.image_batch(vnp, w.uvw_m, w.freq_hz, w.grid_n, w.pixscale, w.out_n,
                                    w.weighting, w.norm, None, w.gains, w.ant1, w.ant2)
    gbar = 2 * (ref_img - target.cpu().numpy())
    rv, rg = oracle.adjoint_batch(gbar, vnp, w.uvw_m, w.freq_hz, w.grid_n, w.pixscale, w.weighting,
                                  w.norm, None, w.gains, w.ant1, w.ant2)
    ev = rel_l2(vis.grad.cpu().numpy().view(np.float32), rv.view(np.float64))
    eg = rel_l2(gains.grad.cpu().numpy().view(np.float32), rg.view(np.float64))
    print(f"  autograd vs oracle: vis {ev:.2e} gains {eg:.2e}", flush=True)
    assert ev <= 1e-5 and eg <= 1e-5


def _rot_inputs(w, d, seed):
    rng = np.random.default_rng(seed)
    cab = rng.uniform(0.0, 300.0, w.n_ant)
    d = dict(d, cable_m=torch.from_numpy(cab).to(device()), ant1=torch.from_numpy(w.ant1).to(device()),
             ant2=torch.from_numpy(w.ant2).to(device()))
    return cab, d


@pytest.mark.parametrize("name", ["wide1024_gains", "subset64_gains", "allsky180_uniform"])
def test_adjoint_with_rotation_and_cables_vs_oracle(name):
    """The adjoint applies the conjugate of the rotation / cable factor: vis and
    gain gradients match the oracle's rotated adjoint (Sec. 4.2 (i), (iii))."""
    from oracle import phase_rotation as pr
    w, use_g = _case(name)
    d = inputs(w, with_gains=use_g)
    lm = (0.04, -0.03)
    cab, d = _rot_inputs(w, d, 11)
    rng = np.random.default_rng(23)
    gbar = torch.from_numpy(rng.normal(size=(w.n_img, w.out_n, w.out_n)).astype(np.float32)).to(device())
    g = d.get("gains")
    vg, gg = blink.degrid_adjoint(gbar, d["vis"], d["uvw_m"], d["freq_hz"], grid_n=w.grid_n,
                                  pixscale=w.pixscale, out_n=w.out_n, weighting=w.weighting, norm=w.norm,
                                  flags=d["flags"], gains=g, ant1=d["ant1"], ant2=d["ant2"],
                                  phase_lm=lm, cable_m=d["cable_m"])
    torch.cuda.synchronize()
    rv, rg = pr.adjoint_batch_rotated(gbar.cpu().numpy().astype(np.float64), d["vis"].cpu().numpy(), w.uvw_m,
                                      w.freq_hz, w.grid_n, w.pixscale, w.weighting, w.norm, lm[0], lm[1],
                                      w.flags, w.gains if use_g else None, w.ant1, w.ant2, cable_m=cab)
    e = rel_l2(vg.cpu().numpy().view(np.float32), rv.view(np.float64))
    print(f"  rotated vis_grad rel-L2 {e:.2e}", flush=True)
    assert e <= 1e-5
    if use_g:
        eg = rel_l2(gg.cpu().numpy().view(np.float32), rg.view(np.float64))
        print(f"  rotated gain_grad rel-L2 {eg:.2e}", flush=True)
        assert eg <= 1e-5


@pytest.mark.parametrize("name", ["wide1024_gains", "allsky180_uniform"])
def test_adjoint_reuses_forward_weight_sums(name):
    """With the forward call's weight sums the adjoint skips counting them and
    gives the same bits."""
    w, use_g = _case(name)
    d = inputs(w, with_gains=use_g)
    _, wsum = run_image_w(w, d)
    rng = np.random.default_rng(5)
    gbar = torch.from_numpy(rng.normal(size=(w.n_img, w.out_n, w.out_n)).astype(np.float32)).to(device())
    kw = dict(grid_n=w.grid_n, pixscale=w.pixscale, out_n=w.out_n, weighting=w.weighting, norm=w.norm,
              flags=d["flags"], gains=d.get("gains"), ant1=d.get("ant1"), ant2=d.get("ant2"))
    a = blink.degrid_adjoint(gbar, d["vis"], d["uvw_m"], d["freq_hz"], **kw)
    b = blink.degrid_adjoint(gbar, d["vis"], d["uvw_m"], d["freq_hz"], weight_sum=wsum, **kw)
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0])
    if use_g:
        assert torch.equal(a[1], b[1])


def run_image_w(w, d):
    ws = torch.empty(w.n_img, dtype=torch.float32, device=device())
    img = blink.image_batch(d["vis"], d["uvw_m"], d["freq_hz"], grid_n=w.grid_n, pixscale=w.pixscale,
                            out_n=w.out_n, weighting=w.weighting, norm=w.norm, flags=d.get("flags"),
                            gains=d.get("gains"), ant1=d.get("ant1"), ant2=d.get("ant2"), weight_sum=ws)
    return img, ws


@pytest.mark.parametrize("dt", [torch.float16, torch.bfloat16])
def test_adjoint_half_storage_vs_oracle(dt):
    """FP16/BF16 storage: the gradient with respect to the dequantised
    visibilities (and the gains) matches the oracle's adjoint on those values."""
    w, _ = _case("wide1024_gains")
    d = inputs(w, with_gains=True)
    q, sig = synth.quantize_vis(d["vis"], dt)
    rng = np.random.default_rng(29)
    gbar = torch.from_numpy(rng.normal(size=(w.n_img, w.out_n, w.out_n)).astype(np.float32)).to(device())
    vg, gg = blink.degrid_adjoint(gbar, q, d["uvw_m"], d["freq_hz"], grid_n=w.grid_n, pixscale=w.pixscale,
                                  out_n=w.out_n, weighting=w.weighting, norm=w.norm, gains=d["gains"],
                                  ant1=d["ant1"], ant2=d["ant2"], vis_scale=sig)
    torch.cuda.synchronize()
    qn = q.cpu()
    if dt == torch.bfloat16:
        bits = qn.view(torch.int16).numpy().view(np.uint16)
        re, im = bits[..., 0], bits[..., 1]
    else:
        re, im = qn[..., 0].numpy(), qn[..., 1].numpy()
    deq = oracle.dequantize(re, im, sig.cpu().numpy()[None, :, None].astype(np.float64))
    rv, rg = oracle.adjoint_batch(gbar.cpu().numpy().astype(np.float64), deq, w.uvw_m, w.freq_hz, w.grid_n,
                                  w.pixscale, w.weighting, w.norm, None, w.gains, w.ant1, w.ant2)
    e = rel_l2(vg.cpu().numpy().view(np.float32), rv.view(np.float64))
    eg = rel_l2(gg.cpu().numpy().view(np.float32), rg.view(np.float64))
    print(f"  {dt}: vis_grad {e:.2e} gain_grad {eg:.2e}", flush=True)
    assert e <= 1e-5 and eg <= 1e-5


@pytest.mark.parametrize("name", ["subset64_gains", "allsky180_uniform"])
def test_adjoint_with_reprojection_vs_oracle(name):
    """With re-projection the adjoint gathers at the re-projected cells: vis and
    gain gradients match the oracle's re-projected adjoint."""
    from oracle import phase_rotation as pr
    w, use_g = _case(name)
    d = inputs(w, with_gains=use_g)
    lm = (0.35, -0.25)
    cab, d = _rot_inputs(w, d, 12)
    rng = np.random.default_rng(24)
    gbar = torch.from_numpy(rng.normal(size=(w.n_img, w.out_n, w.out_n)).astype(np.float32)).to(device())
    vg, gg = blink.degrid_adjoint(gbar, d["vis"], d["uvw_m"], d["freq_hz"], grid_n=w.grid_n,
                                  pixscale=w.pixscale, out_n=w.out_n, weighting=w.weighting, norm=w.norm,
                                  flags=d["flags"], gains=d.get("gains"), ant1=d["ant1"], ant2=d["ant2"],
                                  phase_lm=lm, cable_m=d["cable_m"], reproject=True)
    torch.cuda.synchronize()
    rv, rg = pr.adjoint_batch_rotated(gbar.cpu().numpy().astype(np.float64), d["vis"].cpu().numpy(), w.uvw_m,
                                      w.freq_hz, w.grid_n, w.pixscale, w.weighting, w.norm, lm[0], lm[1],
                                      w.flags, w.gains if use_g else None, w.ant1, w.ant2, cable_m=cab,
                                      reproject=True)
    e = rel_l2(vg.cpu().numpy().view(np.float32), rv.view(np.float64))
    print(f"  re-projected vis_grad rel-L2 {e:.2e}", flush=True)
    assert e <= 1e-5
    if use_g:
        eg = rel_l2(gg.cpu().numpy().view(np.float32), rg.view(np.float64))
        print(f"  re-projected gain_grad rel-L2 {eg:.2e}", flush=True)
        assert eg <= 1e-5


def test_autograd_with_rotation_and_cables():
    from oracle import phase_rotation as pr
    w, _ = _case("subset64_gains")
    d = inputs(w, with_gains=True)
    lm = (0.02, 0.05)
    cab, d = _rot_inputs(w, d, 13)
    vis = d["vis"].clone().requires_grad_(True)
    gains = d["gains"].clone().requires_grad_(True)
    rng = np.random.default_rng(9)
    target = torch.from_numpy(rng.normal(size=(w.n_img, w.out_n, w.out_n)).astype(np.float32)).to(device())
    img = blink.blink_image(vis, gains, d["uvw_m"], d["freq_hz"], d["ant1"], d["ant2"], grid_n=w.grid_n,
                            pixscale=w.pixscale, out_n=w.out_n, weighting=w.weighting, norm=w.norm,
                            phase_lm=lm, cable_m=d["cable_m"])
    ((img - target) ** 2).sum().backward()
    vnp = d["vis"].cpu().numpy()
    ref, _ = pr.image_batch_rotated(vnp, w.uvw_m, w.freq_hz, w.grid_n, w.pixscale, w.out_n, w.weighting,
                                    w.norm, lm[0], lm[1], gains=w.gains, ant1=w.ant1, ant2=w.ant2, cable_m=cab)
    assert rel_l2(img.detach().cpu().numpy(), ref) <= 1e-5
    rv, rg = pr.adjoint_batch_rotated(2 * (ref - target.cpu().numpy()), vnp, w.uvw_m, w.freq_hz, w.grid_n,
                                      w.pixscale, w.weighting, w.norm, lm[0], lm[1], gains=w.gains,
                                      ant1=w.ant1, ant2=w.ant2, cable_m=cab)
    ev = rel_l2(vis.grad.cpu().numpy().view(np.float32), rv.view(np.float64))
    eg = rel_l2(gains.grad.cpu().numpy().view(np.float32), rg.view(np.float64))
    print(f"  rotated autograd vs oracle: vis {ev:.2e} gains {eg:.2e}", flush=True)
    assert ev <= 1e-5 and eg <= 1e-5


# ------------------------------------------------------------ kernel gridding
@pytest.mark.parametrize("name,support", [("subset64_gains", 6), ("allsky180_uniform", 4),
                                          ("wide1024_gains", 6)])
def test_kernel_gridding_adjoint_vs_oracle(name, support):
    """Degridding with the Kaiser-Bessel kernel (and its correction, 1/W and
    the gains): vis and gain gradients against the oracle's kernel adjoint."""
    from oracle import kernel_gridding as kg
    w, use_g = _case(name)
    d = inputs(w, with_gains=use_g)
    rng = np.random.default_rng(31)
    gbar = torch.from_numpy(rng.normal(size=(w.n_img, w.out_n, w.out_n)).astype(np.float32)).to(device())
    g = d.get("gains")
    kw = dict(grid_n=w.grid_n, pixscale=w.pixscale, out_n=w.out_n, weighting=w.weighting, norm=w.norm,
              flags=d["flags"], gains=g, ant1=d.get("ant1"), ant2=d.get("ant2"), kernel_support=support)
    vg, gg = blink.degrid_adjoint(gbar, d["vis"], d["uvw_m"], d["freq_hz"], **kw)
    torch.cuda.synchronize()
    rv, rg = kg.adjoint_batch_conv(gbar.cpu().numpy().astype(np.float64), d["vis"].cpu().numpy(), w.uvw_m,
                                   w.freq_hz, w.grid_n, w.pixscale, w.norm, support, None, w.flags,
                                   w.gains if use_g else None, w.ant1, w.ant2, weighting=w.weighting)
    e = rel_l2(vg.cpu().numpy().view(np.float32), rv.view(np.float64))
    print(f"  kernel adjoint vis_grad rel-L2 {e:.2e}", flush=True)
    assert e <= 1e-5
    if use_g:
        eg = rel_l2(gg.cpu().numpy().view(np.float32), rg.view(np.float64))
        print(f"  kernel adjoint gain_grad rel-L2 {eg:.2e}", flush=True)
        assert eg <= 1e-5
    # the forward call's weight sums give the same gradients to rounding
    ws = torch.empty(w.n_img, dtype=torch.float32, device=device())
    blink.image_batch(d["vis"], d["uvw_m"], d["freq_hz"], weight_sum=ws, **kw)
    vg2, _ = blink.degrid_adjoint(gbar, d["vis"], d["uvw_m"], d["freq_hz"], weight_sum=ws, **kw)
    torch.cuda.synchronize()
    assert rel_l2(vg2.cpu().numpy().view(np.float32), vg.cpu().numpy().view(np.float32)) <= 1e-6


def test_kernel_gridding_adjoint_dot_product_on_gpu():
    w = synth.widefield(n_time=1, n_chan=2, chan_stride=200)
    w.weighting = 1
    d = inputs(w)
    kw = dict(grid_n=w.grid_n, pixscale=w.pixscale, out_n=w.out_n, weighting=w.weighting, norm=w.norm,
              kernel_support=6)
    img = blink.image_batch(d["vis"], d["uvw_m"], d["freq_hz"], **kw)
    rng = np.random.default_rng(5)
    gbar = torch.from_numpy(rng.normal(size=img.shape).astype(np.float32)).to(device())
    vg, _ = blink.degrid_adjoint(gbar, d["vis"], d["uvw_m"], d["freq_hz"], **kw)
    lhs = (img.double() * gbar.double()).sum().item()
    v = d["vis"]
    rhs = (vg.real.double() * v.real.double() + vg.imag.double() * v.imag.double()).sum().item()
    assert abs(lhs - rhs) <= 1e-5 * max(abs(lhs), 1e-30)


def test_autograd_with_kernel_gridding():
    from oracle import kernel_gridding as kg
    w, _ = _case("subset64_gains")
    d = inputs(w, with_gains=True)
    vis = d["vis"].clone().requires_grad_(True)
    gains = d["gains"].clone().requires_grad_(True)
    rng = np.random.default_rng(10)
    target = torch.from_numpy(rng.normal(size=(w.n_img, w.out_n, w.out_n)).astype(np.float32)).to(device())
    img = blink.blink_image(vis, gains, d["uvw_m"], d["freq_hz"], d["ant1"], d["ant2"], grid_n=w.grid_n,
                            pixscale=w.pixscale, out_n=w.out_n, weighting=w.weighting, norm=w.norm,
                            flags=d["flags"], kernel_support=5)
    # (default beta: a much smaller one puts a near-zero of the correction
    # at the edge of this full-field 64^2 image, where dividing by it then
    # magnifies FP32 rounding of the uncorrected pixels)
    ((img - target) ** 2).sum().backward()
    vnp = d["vis"].cpu().numpy()
    ref, _ = kg.image_batch_conv(vnp, w.uvw_m, w.freq_hz, w.grid_n, w.pixscale, w.out_n, w.norm, 5, None,
                                 w.flags, w.gains, w.ant1, w.ant2, weighting=w.weighting)
    assert rel_l2(img.detach().cpu().numpy(), ref) <= 1e-5
    rv, rg = kg.adjoint_batch_conv(2 * (ref - target.cpu().numpy()), vnp, w.uvw_m, w.freq_hz, w.grid_n,
                                   w.pixscale, w.norm, 5, None, w.flags, w.gains, w.ant1, w.ant2,
                                   weighting=w.weighting)
    ev = rel_l2(vis.grad.cpu().numpy().view(np.float32), rv.view(np.float64))
    eg = rel_l2(gains.grad.cpu().numpy().view(np.float32), rg.view(np.float64))
    print(f"  kernel autograd vs oracle: vis {ev:.2e} gains {eg:.2e}", flush=True)
    assert ev <= 1e-5 and eg <= 1e-5


def test_kernel_gridding_adjoint_with_rotation_and_cables():
    """Degridding with the kernel after a phase rotation and cable correction:
    the gradient carries the conjugate of the per-visibility factor p, i.e.
    conj(p) times the kernel adjoint of the rotated visibilities."""
    from oracle import kernel_gridding as kg
    from oracle import phase_rotation as pr
    w, _ = _case("subset64_gains")
    d = inputs(w, with_gains=False)
    lm = (0.05, -0.04)
    cab, d = _rot_inputs(w, d, 14)
    rng = np.random.default_rng(33)
    gbar = torch.from_numpy(rng.normal(size=(w.n_img, w.out_n, w.out_n)).astype(np.float32)).to(device())
    vg, _ = blink.degrid_adjoint(gbar, d["vis"], d["uvw_m"], d["freq_hz"], grid_n=w.grid_n, pixscale=w.pixscale,
                                 out_n=w.out_n, weighting=w.weighting, norm=w.norm, flags=d["flags"],
                                 ant1=d["ant1"], ant2=d["ant2"], phase_lm=lm, cable_m=d["cable_m"],
                                 kernel_support=6)
    torch.cuda.synchronize()
    vis = d["vis"].cpu().numpy()
    ref = np.zeros(vis.shape, dtype=np.complex128)
    for t in range(w.n_time):
        for c in range(w.n_chan):
            p = pr.rotate(np.ones(vis.shape[2]), w.uvw_m[t], w.freq_hz[c], lm[0], lm[1], cab, w.ant1, w.ant2)
            gp, _ = kg.adjoint_one_conv(gbar.cpu().numpy()[t * w.n_chan + c].astype(np.float64), p * vis[t, c],
                                        w.uvw_m[t, :, 0], w.uvw_m[t, :, 1], w.freq_hz[c], w.grid_n, w.pixscale,
                                        w.norm, 6, None, None if w.flags is None else w.flags[t],
                                        weighting=w.weighting)
            ref[t, c] = np.conj(p) * gp
    e = rel_l2(vg.cpu().numpy().view(np.float32), ref.view(np.float64))
    print(f"  rotated kernel adjoint vis_grad rel-L2 {e:.2e}", flush=True)
    assert e <= 1e-5
