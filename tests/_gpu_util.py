"""Shared helpers of the GPU parity tests: seeded inputs on the device, oracle
runs on the same bytes, and the per-image error measures."""
import numpy as np
import torch

import oracle
import paper_2405_13478_amd as blink
from paper_2405_13478_amd import synth

REL_L2_FP32 = 1e-5     # per image, FP32 path against the FP64 oracle


def device():
    return torch.device("cuda:0")


def inputs(w: synth.Workload, with_gains=False, dev=None):
    dev = dev or device()
    vis = synth.visibilities(w, device=dev)
    d = dict(vis=vis,
             uvw_m=torch.from_numpy(np.ascontiguousarray(w.uvw_m)).to(dev),
             freq_hz=torch.from_numpy(np.ascontiguousarray(w.freq_hz)).to(dev),
             flags=None if w.flags is None else torch.from_numpy(w.flags).to(dev))
    if with_gains:
        d["gains"] = torch.from_numpy(w.gains).to(dev)
        d["ant1"] = torch.from_numpy(w.ant1).to(dev)
        d["ant2"] = torch.from_numpy(w.ant2).to(dev)
    return d


def run_image(w, d, **kw):
    ws = torch.empty(w.n_img, dtype=torch.float32, device=d["vis"].device)
    img = blink.image_batch(d["vis"], d["uvw_m"], d["freq_hz"], grid_n=w.grid_n, pixscale=w.pixscale,
                            out_n=w.out_n, weighting=w.weighting, norm=w.norm, flags=d.get("flags"),
                            vis_scale=d.get("vis_scale"), gains=d.get("gains"), ant1=d.get("ant1"),
                            ant2=d.get("ant2"), weight_sum=ws, **kw)
    torch.cuda.synchronize()
    return img, ws


def oracle_images(w, vis_np, images, gains=None, norm=None, out_n=None):
    return oracle.image_batch(vis_np, w.uvw_m, w.freq_hz, w.grid_n, w.pixscale,
                              w.out_n if out_n is None else out_n, w.weighting,
                              w.norm if norm is None else norm, w.flags,
                              gains, w.ant1 if gains is not None else None,
                              w.ant2 if gains is not None else None, images=images)


def rel_l2(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.linalg.norm(ref)
    if den == 0:
        return float(np.linalg.norm(got))
    return float(np.linalg.norm(got - ref) / den)


def per_image_rel_l2(got, ref):
    return [rel_l2(g, r) for g, r in zip(got, ref)]
