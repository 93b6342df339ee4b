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


def nonzero_columns(w, t_slice):
    """Per image (t, c) of the slice: the number of half-spectrum u columns that
    can hold data, min(N/2, max |rint(u s_c)| + 1) over the usable baselines.
    The column kernels transform and store only these columns and the row
    kernel reads only these, so they set the algorithmic bytes per image."""
    import numpy as np
    H = w.grid_n // 2
    s = (w.freq_hz * (np.float64(w.grid_n) * np.float64(w.pixscale))) / 299792458.0
    out = []
    for t in range(t_slice.start, t_slice.stop):
        u = w.uvw_m[t, :, 0]
        ok = np.isfinite(u) & np.isfinite(w.uvw_m[t, :, 1])
        if w.flags is not None:
            ok &= w.flags[t] == 0
        umax = np.abs(u[ok]).max() if ok.any() else None
        if umax is None:
            out.append(np.zeros(len(s), dtype=np.int64))
            continue
        cmax = np.abs(np.rint(np.outer(s, u[ok]))).max(axis=1)
        out.append(np.minimum(H, cmax + 1).astype(np.int64))
    return np.concatenate(out)


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


# ---------------------------------------------------------------- rocprof summaries
PROFILE_CMDS = {
    "stats": "rocprofv3 --kernel-trace --stats --output-format csv -d OUT/stats -o bench -- "
             "python3 bench.py --steps 5 --warmup 1 --no-cpu-baseline",
    "fetch": "rocprofv3 --pmc FETCH_SIZE --kernel-include-regex 'blink|copyBuffer' --output-format csv "
             "-d OUT/pmc_FETCH_SIZE -o bench -- python3 bench.py --timesteps 10 --steps 1 --warmup 0 --no-cpu-baseline",
    "write": "rocprofv3 --pmc WRITE_SIZE --kernel-include-regex 'blink|copyBuffer' --output-format csv "
             "-d OUT/pmc_WRITE_SIZE -o bench -- python3 bench.py --timesteps 10 --steps 1 --warmup 0 --no-cpu-baseline",
    "copy_fetch": "rocprofv3 --pmc FETCH_SIZE --kernel-include-regex 'blink|copyBuffer' --output-format csv "
                  "-d OUT/pmc_copy_FETCH_SIZE -o copy -- python3 bench.py --copy-calibration",
    "copy_write": "rocprofv3 --pmc WRITE_SIZE --kernel-include-regex 'blink|copyBuffer' --output-format csv "
                  "-d OUT/pmc_copy_WRITE_SIZE -o copy -- python3 bench.py --copy-calibration",
}
KERNEL_KEYS = {"grid_cols": "k_grid_cols<1024, 0", "rows": "k_rows<1024>"}


def _csv(path):
    import csv
    import glob
    files = glob.glob(path)
    if not files:
        raise SystemExit(f"missing rocprof output: {path}")
    with open(files[0]) as f:
        return list(csv.DictReader(f))


def _counter_mean(rows, key, counter):
    v = [float(r["Counter_Value"]) for r in rows if key in r["Kernel_Name"] and r["Counter_Name"] == counter]
    return (sum(v) / len(v), len(v)) if v else (None, 0)


def summarize(out_dir):
    """Write profiles/ summaries from the rocprofv3 outputs under out_dir (CPU only)."""
    prof = os.path.join(ROOT, "profiles")
    os.makedirs(prof, exist_ok=True)
    digest = _csrc_digest()
    stats = _csv(os.path.join(out_dir, "stats", "*_kernel_stats.csv"))
    tot = sum(float(r["TotalDurationNs"]) for r in stats if "blink" in r["Name"])
    lines = ["# rocprofv3 kernel statistics: widefield 1024^2 -> 512^2 image batches", "",
             "Workload: 128 tiles (8128 baselines), 768 channels x 10 timesteps per step (7,680 images), "
             "natural weighting; 5 timed steps + 1 warm-up.", "",
             "Command (from the repository root, with OUT the output folder):", "",
             "    " + PROFILE_CMDS["stats"], "",
             f"Library sources digest: `{digest}`", "",
             "| kernel | calls | avg us | min us | max us | share of blink time |",
             "|---|---|---|---|---|---|"]
    for r in sorted(stats, key=lambda r: -float(r["TotalDurationNs"])):
        if "blink" not in r["Name"]:
            continue
        lines.append(f"| `{r['Name'].replace('|', '/')}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | "
                     f"{100 * float(r['TotalDurationNs']) / tot:.1f}% |")
    with open(os.path.join(prof, "k_grid_cols_k_rows_widefield1024_kernel_stats.md"), "w") as f:
        f.write("\n".join(lines) + "\n")

    fe = _csv(os.path.join(out_dir, "pmc_FETCH_SIZE", "*_counter_collection.csv"))
    wr = _csv(os.path.join(out_dir, "pmc_WRITE_SIZE", "*_counter_collection.csv"))
    cfe = _csv(os.path.join(out_dir, "pmc_copy_FETCH_SIZE", "*_counter_collection.csv"))
    cwr = _csv(os.path.join(out_dir, "pmc_copy_WRITE_SIZE", "*_counter_collection.csv"))
    copy_bytes = 1 << 30
    cf, _ = _counter_mean(cfe, "copyBuffer", "FETCH_SIZE")
    cw, _ = _counter_mean(cwr, "copyBuffer", "WRITE_SIZE")
    f_fetch = copy_bytes / (cf * 1024.0)
    f_write = copy_bytes / (cw * 1024.0)
    imgs = 512
    res = {"workload": "widefield 1024^2 -> 512^2, 8128 baselines, 512 images per launch",
           "csrc_digest": digest, "copy_calibration": {"bytes": copy_bytes, "FETCH_SIZE_KiB": cf,
                                                      "WRITE_SIZE_KiB": cw, "fetch_scale": f_fetch,
                                                      "write_scale": f_write},
           "kernels": {}}
    md = ["# HBM traffic per dispatch (rocprofv3 FETCH_SIZE / WRITE_SIZE)", "",
          "Counters in KiB per dispatch, scaled by what the same counter reads for a plain 1 GiB "
          "device copy (`__amd_rocclr_copyBuffer`).", "", "Commands (from the repository root):", ""]
    md += ["    " + PROFILE_CMDS[k] for k in ("fetch", "write", "copy_fetch", "copy_write")]
    md += ["", f"Copy calibration: FETCH_SIZE {cf:.1f} KiB and WRITE_SIZE {cw:.1f} KiB for 1 GiB moved "
           f"-> scale {f_fetch:.4f} (fetch), {f_write:.4f} (write).", "",
           f"Library sources digest: `{digest}`", "",
           "| kernel | dispatches | FETCH KiB | WRITE KiB | HBM bytes / launch (scaled) | per image | algorithmic per image |",
           "|---|---|---|---|---|---|---|"]
    alg = {"grid_cols": 8128 * 8 + 512 * 512 * 8, "rows": 512 * 512 * 8 + 512 * 512 * 4}
    for name, key in KERNEL_KEYS.items():
        fm, n = _counter_mean(fe, key, "FETCH_SIZE")
        wm, _ = _counter_mean(wr, key, "WRITE_SIZE")
        tb = (fm * f_fetch + wm * f_write) * 1024.0
        res["kernels"][name] = {"FETCH_SIZE_KiB": fm, "WRITE_SIZE_KiB": wm, "dispatches": n,
                                "hbm_bytes_per_launch": tb, "images_per_launch": imgs}
        md.append(f"| {name} (`{key}`) | {n} | {fm:.1f} | {wm:.1f} | {tb:.4g} | {tb / imgs:.4g} | {alg[name]} |")
    dom = "grid_cols"
    res["kernel"] = dom
    res["hbm_bytes_per_launch"] = res["kernels"][dom]["hbm_bytes_per_launch"]
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(res, f, indent=1)
    with open(TRAFFIC_FILE.replace(".json", ".md"), "w") as f:
        f.write("\n".join(md) + "\n")
    print(json.dumps(res))


# ---------------------------------------------------------------- main
def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--timesteps-per-step", type=int, default=10)
    ap.add_argument("--timesteps", type=int, default=100,
                    help="timesteps of the job generated into HBM (100 = the whole workload)")
    ap.add_argument("--chunk", type=int, default=0, help="images per internal chunk (0 = library default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=64)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (counter calibration for profiling)")
    ap.add_argument("--summarize", metavar="ROCPROF_OUT",
                    help="write the profiles/ summaries from rocprofv3 output (no GPU needed)")
    args = ap.parse_args()
    if args.summarize:
        summarize(args.summarize)
        return

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
    w = synth.widefield(n_time=max(TT, args.timesteps), n_chan=768)
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
    ncz_mean = float(np.mean([nonzero_columns(w, slice((k % n_batches) * TT, (k % n_batches + 1) * TT)).mean()
                              for k in range(min(args.steps, n_batches))]))
    per_image = {
        "grid_cols": B * 8 + ncz_mean * M * 8,     # visibilities in, non-empty half-spectrum columns out
        "rows": ncz_mean * M * 8 + M * M * 4,      # those columns in, float image cutout out
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
        "nonzero_half_spectrum_columns_mean": round(ncz_mean, 2),
        "path_hbm_frac_algorithmic": round(path_bytes * img_per_s / 1e9 / HBM_PEAK_GBS, 4),
        "path_hbm_frac_model_iii": round((B * 8 + H * M * 8 * 2 + M * M * 4) * img_per_s / 1e9 / HBM_PEAK_GBS, 4),
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
