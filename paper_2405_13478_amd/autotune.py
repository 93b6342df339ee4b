"""Autotuner for the image path's launch shapes, with a JSON cache.

The tunables of blink_image_batch - u-cell columns per workgroup of the
column kernel, the persistent row-pass grid size and the images per chunk -
are timed on synthetic inputs of the target shape (HIP events, median of a
few calls): first every tile width x row grid at the default chunk, then the
chunk sizes at the best of those (a smaller chunk keeps the half-spectrum
intermediate resident in the 256 MB Infinity Cache between the two passes, a
larger one means fewer, longer launches with less time in their tails).
The fastest combination is stored under a key of the shape (grid size,
cutout, baselines, weighting, storage type). image_batch looks
the key up when the caller leaves a tunable unset.
"""
from __future__ import annotations

import argparse
import itertools
import json
import os
import statistics

_PKG = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(_PKG, "tuned.json")
_cache = None

COLS_PER_WG = (2, 4, 8)
ROWS_WG = (0, 512, 1024, 2048)
# images per chunk besides the default: small ones keep the half spectrum in
# the Infinity Cache, large ones (several GiB of half spectrum) shorten the
# launch tails; chunks beyond the call's image count are skipped
CHUNKS = (0, 16, 32, 64, 128, 256, 384, 512, 768, 1024, 1536, 2048, 3072)


def key(grid_n, out_n, n_bl, weighting, vis_type) -> str:
    return f"gfx950/N{int(grid_n)}/M{int(out_n)}/B{int(n_bl)}/w{int(weighting)}/v{int(vis_type)}"


def _load():
    global _cache
    if _cache is None:
        try:
            with open(CACHE) as f:
                _cache = json.load(f)
        except (OSError, ValueError):
            _cache = {}
    return _cache


def lookup(grid_n, out_n, n_bl, weighting, vis_type):
    return _load().get(key(grid_n, out_n, n_bl, weighting, vis_type))


def tune_workload(w, vis, uvw, freq, flags=None, vis_scale=None, steps=5, candidates=None, log=print):
    """Time every candidate on the given device inputs; returns (best dict, all results)."""
    import torch
    from . import blink as B
    M = w.out_n
    n_img = vis.shape[0] * vis.shape[1]
    images = torch.empty((n_img, M, M), dtype=torch.float32, device=vis.device)
    vt = B._vis_type(vis)
    results = []

    def run(cands):
        for cpw, rwg, chunk in cands:
            r = _time_one(B, w, vis, uvw, freq, flags, vis_scale, images, n_img, cpw, rwg, chunk, steps, log)
            if r is not None:
                results.append(r)

    if candidates:
        run(candidates)
    else:
        run(itertools.product(COLS_PER_WG, ROWS_WG, (0,)))
        b = min(results, key=lambda r: r["ms"])
        run((b["cols_per_wg"], b["rows_wg"], c) for c in CHUNKS if c != 0 and c <= n_img)
    best = min(results, key=lambda r: r["ms"])
    return {**best, "key": key(w.grid_n, M, w.n_bl, w.weighting, vt)}, results


def _time_one(B, w, vis, uvw, freq, flags, vis_scale, images, n_img, cpw, rwg, chunk, steps, log):
    import torch
    M = w.out_n
    kw = dict(grid_n=w.grid_n, pixscale=w.pixscale, out_n=M, weighting=w.weighting, norm=w.norm,
              flags=flags, vis_scale=vis_scale, chunk_images=chunk, cols_per_wg=cpw, rows_wg=rwg)
    p = B.make_problem(vis, uvw, freq, w.grid_n, w.pixscale, M, w.weighting, w.norm, None, chunk, cpw, rwg)
    ws = B.workspace(p, B.CALL_IMAGE, vis.device)
    try:
        B.image_batch(vis, uvw, freq, images=images, ws=ws, **kw)
    except B.BlinkError as e:          # e.g. a tile width whose workgroup exceeds LDS
        log(json.dumps({"cols_per_wg": cpw, "rows_wg": rwg, "chunk_images": chunk, "skipped": str(e)}))
        return None
    torch.cuda.synchronize()
    ts = []
    for _ in range(steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        B.image_batch(vis, uvw, freq, images=images, ws=ws, **kw)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    ms = statistics.median(ts)
    r = {"cols_per_wg": cpw, "rows_wg": rwg, "chunk_images": chunk, "ms": ms,
         "images_per_s": n_img / (ms / 1e3)}
    log(json.dumps(r))
    return r


def main():
    ap = argparse.ArgumentParser(description="tune the image path's launch shapes")
    ap.add_argument("--workload", nargs="+", default=["widefield", "allsky", "precision", "plain"])
    ap.add_argument("--out", default=CACHE, help="cache file to update")
    args = ap.parse_args()
    import torch
    from . import synth
    dev = torch.device("cuda:0")
    shapes = {
        "widefield": lambda: synth.widefield(n_time=10, n_chan=768),
        "allsky": lambda: synth.station_allsky(n_time=250, n_chan=32),
        "precision": lambda: synth.precision_station(n_time=1, n_chan=384),
        "plain": lambda: synth.plain_single(n_time=1),
    }
    try:
        with open(args.out) as f:
            cache = json.load(f)
    except (OSError, ValueError):
        cache = {}
    for name in args.workload:
        w = shapes[name]()
        vis = synth.visibilities(w, device=dev)
        uvw = torch.from_numpy(w.uvw_m).to(dev)
        freq = torch.from_numpy(w.freq_hz).to(dev)
        flags = None if w.flags is None else torch.from_numpy(w.flags).to(dev)
        forms = [(vis, None)]
        if name == "precision":
            forms.append(synth.quantize_vis(vis, torch.float16))
        for v, sc in forms:
            best, _ = tune_workload(w, v, uvw, freq, flags, sc, log=lambda m: print(f"[{name}] {m}", flush=True))
            cache[best.pop("key")] = {**best, "workload": name}
            print(f"[{name}] best {json.dumps(best)}", flush=True)
        del vis
        with open(args.out, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
