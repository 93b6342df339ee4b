"""HIP-graph capture of the whole image path.

blink_image_batch allocates nothing and never synchronises, so a call can be
captured once and replayed. Each replay is checked bit for bit against an
eager call, with eager library work and host synchronisation in between, and
after the inputs are overwritten in place.
"""
import pytest
import torch

import paper_2405_13478_amd as blink
from paper_2405_13478_amd import synth

from _gpu_util import device, inputs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", ["allsky180", "wide1024"])
def test_graph_replay_matches_eager(name):
    print(f"\n[gpu] graph replay {name}", flush=True)
    w = (synth.station_allsky(n_time=2, n_chan=3) if name == "allsky180"
         else synth.widefield(n_time=1, n_chan=4, chan_stride=100))
    d = inputs(w)
    dev = device()
    kw = dict(grid_n=w.grid_n, pixscale=w.pixscale, out_n=w.out_n, weighting=w.weighting,
              norm=w.norm, flags=d["flags"])
    p = blink.blink.make_problem(d["vis"], d["uvw_m"], d["freq_hz"], w.grid_n, w.pixscale, w.out_n,
                                 w.weighting, w.norm)
    ws = blink.workspace(p, blink.CALL_IMAGE, dev)
    out = torch.empty((w.n_img, w.out_n, w.out_n), dtype=torch.float32, device=dev)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        blink.image_batch(d["vis"], d["uvw_m"], d["freq_hz"], images=out, ws=ws, **kw)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()

    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        blink.image_batch(d["vis"], d["uvw_m"], d["freq_hz"], images=out, ws=ws, **kw)
    torch.cuda.synchronize()

    for rep in range(4):
        if rep == 2:   # new visibilities, written in place into the captured input
            d["vis"].mul_(0.5).add_(1.0 + 0.25j)
        ref = blink.image_batch(d["vis"], d["uvw_m"], d["freq_hz"], **kw)   # eager, own workspace
        torch.cuda.synchronize()
        out.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref), f"replay {rep} differs from the eager call"
