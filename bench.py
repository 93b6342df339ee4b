#!/usr/bin/env python3
"""Throughput of the dirty-imaging path on one MI355X.

Workload: the widefield array case - 128 tiles (64 in a 300 m core, 64 in a
3 km disc, 8128 baselines), 768 channels of 40 kHz centred at 185 MHz, 100
timesteps (76,800 images), 1024 x 1024 grid, natural weighting, images cut to
the central 512 x 512. Visibilities are synthetic (200 power-law point
sources plus noise), generated into HBM before timing.

One step = one call of the whole path (sort by u, cell bounds, gridding +
column inverse transform, row inverse transform + shift / 1/W / cutout) over
a batch of 10 timesteps x 768 channels = 7,680 images; consecutive steps walk
through the 100 timesteps, so 10 steps image the whole job once.

Prints ONE JSON line (images/s = value) with the roofline of the dominant
kernel (per-launch HIP-event durations from the same timed steps) and the
FP64 CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E peak, GB/s
METRIC = "dirty images/s and visibilities/s at 128 tiles, 1024² grid; % HBM roofline"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_grid_cols_rows_widefield1024.json")
CSRC = os.path.join(ROOT, "paper_2405_13478_amd", "csrc")


def _csrc_digest():
    h = hashlib.sha256()
    for f in sorted(os.listdir(CSRC)):
        if f.endswith((".hip", ".hpp", ".py")):
            with open(os.path.join(CSRC, f), "rb") as fh:
                h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


# ---------------------------------------------------------------- CPU baseline
def _oracle_one(job):
    """One image with the FP64 oracle (runs in a worker process)."""
    import oracle
    vis, u, v, f, n, dx, m, wt, nm = job
    return oracle.image_one(vis, u, v, f, n, dx, m, wt, nm)["image"].shape[0]


def cpu_baseline(w, vis_cpu, sample, cores):
    import multiprocessing as mp
    ctx = mp.get_context("spawn")
    jobs = []
    for i in sample:
        t, c = divmod(i, w.n_chan)
        jobs.append((vis_cpu[t, c], w.uvw_m[t, :, 0], w.uvw_m[t, :, 1], float(w.freq_hz[c]),
                     w.grid_n, w.pixscale, w.out_n, w.weighting, w.norm))
    env_keep = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in env_keep:
        os.environ[k] = "1"
    try:
        with ctx.Pool(cores) as pool:
            pool.map(_oracle_one, jobs[:cores], chunksize=1)     # start-up and imports, untimed
            t0 = time.perf_counter()
            pool.map(_oracle_one, jobs, chunksize=1)
            dt = time.perf_counter() - t0
    finally:
        for k, v in env_keep.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    return len(jobs) / dt, dt


# ---------------------------------------------------------------- main
def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--timesteps-per-step", type=int, default=10)
    ap.add_argument("--chunk", type=int, default=0, help="images per internal chunk (0 = library default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=64)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (counter calibration for profiling)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "images shard across GPUs with no exchange, see DESIGN.md", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    sys.path.insert(0, ROOT)
    import paper_2405_13478_amd as blink
    from paper_2405_13478_amd import synth

    dev = torch.device("cuda:0")
    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)   # 1 GiB
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": a.numel() * 4, "repeats": 5}))
        return

    blink.load_library()
    TT = args.timesteps_per_step
    w = synth.widefield(n_time=100, n_chan=768)
    n_batches = w.n_time // TT
    t_gen = time.perf_counter()
    vis = synth.visibilities(w, device=dev)                                # [100][768][8128] c64, 5.0 GB
    uvw = torch.from_numpy(w.uvw_m).to(dev)
    freq = torch.from_numpy(w.freq_hz).to(dev)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t_gen

    n_img = TT * w.n_chan
    M = w.out_n
    images = torch.empty((n_img, M, M), dtype=torch.float32, device=dev)   # reused per step
    p = blink.blink.make_problem(vis[:TT], uvw[:TT], freq, w.grid_n, w.pixscale, M, w.weighting,
                                 w.norm, None, args.chunk)
    ws = blink.workspace(p, blink.CALL_IMAGE, dev)
    times = blink.KernelTimes()

    def step(k, tm=None):
        b = k % n_batches
        sl = slice(b * TT, (b + 1) * TT)
        blink.image_batch(vis[sl], uvw[sl], freq, grid_n=w.grid_n, pixscale=w.pixscale, out_n=M,
                          weighting=w.weighting, norm=w.norm, chunk_images=args.chunk,
                          images=images, ws=ws, times=tm)

    for k in range(args.warmup):
        step(k)
    torch.cuda.synchronize()

    acc_ms = [0.0] * 4
    acc_n = [0] * 4
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    for k in range(args.steps):
        step(k, times)
        for c in range(4):
            acc_ms[c] += times.ms[c]
            acc_n[c] += times.launches[c]
    ev1.record()
    torch.cuda.synchronize()
    total_ms = ev0.elapsed_time(ev1)
    ms_per_step = total_ms / args.steps
    img_per_s = n_img * args.steps / (total_ms / 1e3)
    vis_per_s = img_per_s * w.n_bl

    # ---- roofline of the dominant kernel (algorithmic bytes per launch / mean launch time)
    H, N, B = w.grid_n // 2, w.grid_n, w.n_bl
    per_image = {
        "grid_cols": B * 8 + H * M * 8,            # visibilities in, half spectrum (cut rows) out
        "rows": H * M * 8 + M * M * 4,             # half spectrum in, float image cutout out
    }
    classes = blink.KCLASS
    dom = max(range(4), key=lambda c: acc_ms[c])
    name = classes[dom]
    imgs_timed = n_img * args.steps
    mean_ms = acc_ms[dom] / max(acc_n[dom], 1)
    bytes_per_launch = per_image.get(name, 0) * imgs_timed / max(acc_n[dom], 1)
    achieved = bytes_per_launch / (mean_ms * 1e-3) / 1e9
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        tr = json.load(open(TRAFFIC_FILE))
        if tr.get("csrc_digest") == _csrc_digest() and tr.get("kernel") == name:
            traffic = tr.get("hbm_bytes_per_launch")
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": name, "mean_launch_ms": round(mean_ms, 5),
            "algorithmic_bytes_per_launch": int(bytes_per_launch),
            "images_per_launch": round(imgs_timed / max(acc_n[dom], 1), 2)}
    path_bytes = per_image["grid_cols"] + per_image["rows"]
    kernel_ms = {classes[c]: round(acc_ms[c] / args.steps, 4) for c in range(4)}

    out = {
        "metric": METRIC, "value": round(img_per_s, 1), "unit": "images/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "widefield 128 tiles (8128 baselines), 768 ch x 100 timesteps, "
                               "1024^2 grid -> 512^2 cutout, natural weighting",
                   "images_per_step": n_img, "timesteps_per_step": TT, "grid_n": N, "out_n": M,
                   "baselines": B, "channels": w.n_chan, "chunk_images": args.chunk},
        "visibilities_per_s": round(vis_per_s, 1),
        "path_hbm_frac_model_iii": round(path_bytes * img_per_s / 1e9 / HBM_PEAK_GBS, 4),
        "path_hbm_frac_model_i": round((B * 8 + 2 * N * N * 8 + M * M * 4) * img_per_s / 1e9 / HBM_PEAK_GBS, 4),
        "kernel_ms_per_step": kernel_ms,
        "roofline": roof,
        "input_generation_s": round(t_gen, 2),
    }

    if not args.no_cpu_baseline:
        cores = max(1, min(16, os.cpu_count() or 1))
        S = max(1, args.cpu_sample)
        stride = max(1, w.n_chan // S)
        sample = [(k * stride) % w.n_chan + (k * stride // w.n_chan) * w.n_chan for k in range(S)]
        vis_cpu = vis[:2].cpu().numpy()
        rate, dt = cpu_baseline(w, vis_cpu, sample, cores)
        out["cpu_baseline"] = {"value": round(rate, 3), "unit": "images/s", "cores": cores,
                               "kind": "oracle",
                               "sample": f"{S} images of timestep 0 (channels every {stride}) of "
                                         f"the same workload, FP64 numpy oracle, {cores}-process "
                                         f"pool, {dt:.1f} s wall"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
