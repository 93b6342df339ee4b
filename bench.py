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
import glob
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E peak, GB/s
KB_SUPPORT = 6                 # Kaiser-Bessel support (cells) of the kernel-gridding workload
ROT_LM = (0.05, 0.03)          # phase centre of the rotation workload (direction cosines)
CABLE_MAX_M = 500.0            # rotation workload: electrical cable lengths uniform in [0, 500) m
METRIC = "dirty images/s and visibilities/s at 128 tiles, 1024² grid; % HBM roofline"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_grid_cols_half_k_rows_half_widefield1024.json")
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
    vis, u, v, f, n, dx, m, wt, nm, ksup = job
    if ksup > 0:
        return oracle.kernel_gridding.image_one_conv(vis, u, v, f, n, dx, m, nm, ksup)["image"].shape[0]
    return oracle.image_one(vis, u, v, f, n, dx, m, wt, nm)["image"].shape[0]


def cpu_baseline(w, vis_cpu, sample, cores, ksup=0):
    import multiprocessing as mp
    ctx = mp.get_context("spawn")
    jobs = []
    for i in sample:
        t, c = divmod(i, w.n_chan)
        jobs.append((vis_cpu[t, c], w.uvw_m[t, :, 0], w.uvw_m[t, :, 1], float(w.freq_hz[c]),
                     w.grid_n, w.pixscale, w.out_n, w.weighting, w.norm, ksup))
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
             "python3 bench.py --steps 5 --warmup 1 --no-cpu-baseline --plain-loop 0",
    "fetch": "rocprofv3 --pmc FETCH_SIZE --kernel-include-regex 'blink|copyBuffer' --output-format csv "
             "-d OUT/pmc_FETCH_SIZE -o bench -- python3 bench.py --timesteps 10 --steps 1 --warmup 0 "
             "--no-cpu-baseline --plain-loop 0",
    "write": "rocprofv3 --pmc WRITE_SIZE --kernel-include-regex 'blink|copyBuffer' --output-format csv "
             "-d OUT/pmc_WRITE_SIZE -o bench -- python3 bench.py --timesteps 10 --steps 1 --warmup 0 "
             "--no-cpu-baseline --plain-loop 0",
    "copy_fetch": "rocprofv3 --pmc FETCH_SIZE --kernel-include-regex 'blink|copyBuffer' --output-format csv "
                  "-d OUT/pmc_copy_FETCH_SIZE -o copy -- python3 bench.py --copy-calibration",
    "copy_write": "rocprofv3 --pmc WRITE_SIZE --kernel-include-regex 'blink|copyBuffer' --output-format csv "
                  "-d OUT/pmc_copy_WRITE_SIZE -o copy -- python3 bench.py --copy-calibration",
}
# kernel statistics of the other workloads: (output folder, bench flags, summary file, title)
EXTRA_STATS = {
    "widefield_kb": ("stats_widefield_kb", "--workload widefield_kb --steps 3 --warmup 1 --no-cpu-baseline",
                     "k_grid_cols_kb_k_rows_half_kb_widefield1024_kernel_stats.md",
                     "widefield 1024^2 -> 512^2 with a 6-cell Kaiser-Bessel gridding kernel, 7,680-image steps"),
    "dynspec": ("stats_dynspec", "--workload dynspec --steps 5 --warmup 1 --no-cpu-baseline",
                "k_dynspec_100x96_512sq_mean8_kernel_stats.md",
                "dynamic spectra of 100 timesteps x 96 channels of 512^2 images, mean of 8 preceding images"),
    "xengine": ("stats_xengine", "--workload xengine --steps 5 --warmup 1 --no-cpu-baseline",
                "k_xengine_256ant_4096samp_kernel_stats.md",
                "X-engine, 256 antennas, 32 channels x 64 integrations of 4096 int8 samples"),
    "diff": ("stats_diff", "--workload diff --steps 5 --warmup 2 --no-cpu-baseline",
             "k_rows_adj_k_cols_adj_diff_widefield1024_320img_kernel_stats.md",
             "forward + hand-written adjoint (autograd step) of 320 widefield images, 1024^2 -> 512^2, "
             "with antenna gains"),
    "allsky": ("stats_allsky", "--workload allsky --steps 3 --warmup 1 --no-cpu-baseline",
               "k_grid_cols_k_rows_allsky180_uniform_kernel_stats.md",
               "station all-sky, 32640 baselines, 32,000 images of 180^2 per step, uniform weighting, "
               "2-10% flagged"),
}


def extra_stats_cmd(k):
    d, flags, _, _ = EXTRA_STATS[k]
    return f"rocprofv3 --kernel-trace --stats --output-format csv -d OUT/{d} -o bench -- python3 bench.py {flags}"
KERNEL_KEYS = {"grid_cols": "k_grid_cols_half<1024", "rows": "k_rows_half<1024"}


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
    with open(os.path.join(prof, "k_grid_cols_half_k_rows_half_widefield1024_kernel_stats.md"), "w") as f:
        f.write("\n".join(lines) + "\n")
    for k, (d, _, fname, title) in EXTRA_STATS.items():
        if not glob.glob(os.path.join(out_dir, d, "*_kernel_stats.csv")):
            continue
        st = _csv(os.path.join(out_dir, d, "*_kernel_stats.csv"))
        tt = sum(float(r["TotalDurationNs"]) for r in st if "blink" in r["Name"]) or 1.0
        ln = [f"# rocprofv3 kernel statistics: {title}", "",
              "Command (from the repository root, with OUT the output folder):", "",
              "    " + extra_stats_cmd(k), "", f"Library sources digest: `{digest}`", "",
              "| kernel | calls | avg us | min us | max us | share of blink time |", "|---|---|---|---|---|---|"]
        for r in sorted(st, key=lambda r: -float(r["TotalDurationNs"])):
            if "blink" not in r["Name"]:
                continue
            ln.append(f"| `{r['Name'].replace('|', '/')}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                      f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | "
                      f"{100 * float(r['TotalDurationNs']) / tt:.1f}% |")
        with open(os.path.join(prof, fname), "w") as f:
            f.write("\n".join(ln) + "\n")

    fe = _csv(os.path.join(out_dir, "pmc_FETCH_SIZE", "*_counter_collection.csv"))
    wr = _csv(os.path.join(out_dir, "pmc_WRITE_SIZE", "*_counter_collection.csv"))
    cfe = _csv(os.path.join(out_dir, "pmc_copy_FETCH_SIZE", "*_counter_collection.csv"))
    cwr = _csv(os.path.join(out_dir, "pmc_copy_WRITE_SIZE", "*_counter_collection.csv"))
    copy_bytes = 1 << 30
    cf, _ = _counter_mean(cfe, "copyBuffer", "FETCH_SIZE")
    cw, _ = _counter_mean(cwr, "copyBuffer", "WRITE_SIZE")
    f_fetch = copy_bytes / (cf * 1024.0)
    f_write = copy_bytes / (cw * 1024.0)
    _, n_launch = _counter_mean(fe, KERNEL_KEYS["grid_cols"], "FETCH_SIZE")
    imgs = 10 * 768 // max(n_launch, 1)          # the counter runs image 10 timesteps x 768 channels
    sys.path.insert(0, ROOT)
    from paper_2405_13478_amd import synth
    ncz = float(nonzero_columns(synth.widefield(n_time=10, n_chan=768), slice(0, 10)).mean())
    alg = {"grid_cols": 8128 * 8 + ncz * 512 * 8, "rows": ncz * 512 * 8 + 512 * 512 * 4}
    res = {"workload": f"widefield 1024^2 -> 512^2, 8128 baselines, {imgs} images per launch",
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
           "Algorithmic bytes per image count the visibilities and the non-empty half-spectrum columns "
           f"(mean {ncz:.1f} of 512 for this batch) that the kernels must move.", "",
           "| kernel | dispatches | FETCH KiB | WRITE KiB | HBM bytes / launch (scaled) | per image | algorithmic per image |",
           "|---|---|---|---|---|---|---|"]
    for name, key in KERNEL_KEYS.items():
        fm, n = _counter_mean(fe, key, "FETCH_SIZE")
        wm, _ = _counter_mean(wr, key, "WRITE_SIZE")
        tb = (fm * f_fetch + wm * f_write) * 1024.0
        res["kernels"][name] = {"FETCH_SIZE_KiB": fm, "WRITE_SIZE_KiB": wm, "dispatches": n,
                                "hbm_bytes_per_launch": tb, "images_per_launch": imgs}
        md.append(f"| {name} (`{key}`) | {n} | {fm:.1f} | {wm:.1f} | {tb:.4g} | {tb / imgs:.4g} | {alg[name]:.4g} |")
    dom = "grid_cols"
    res["kernel"] = dom
    res["hbm_bytes_per_launch"] = res["kernels"][dom]["hbm_bytes_per_launch"]
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(res, f, indent=1)
    with open(TRAFFIC_FILE.replace(".json", ".md"), "w") as f:
        f.write("\n".join(md) + "\n")
    print(json.dumps(res))


# ---------------------------------------------------------------- workloads
def _setup(args, synth):
    """(workload, timesteps per step, channels per step) for --workload."""
    k = args.workload
    if k in ("widefield", "widefield_kb", "widefield_rot"):
        TT = args.timesteps_per_step or 10
        return synth.widefield(n_time=max(TT, args.timesteps or 100), n_chan=768), TT
    if k == "plain":
        return synth.plain_single(n_time=1), 1
    if k == "allsky":
        T = args.timesteps or 1000
        return synth.station_allsky(n_time=T, n_chan=32), args.timesteps_per_step or T
    if k == "precision":
        TT = args.timesteps_per_step or 1
        return synth.precision_station(n_time=max(TT, args.timesteps or 5), n_chan=384), TT
    raise SystemExit(f"unknown workload {k}")


DESCRIPTION = {
    "widefield": "widefield 128 tiles (8128 baselines), 768 ch x 100 timesteps, 1024^2 grid -> 512^2 cutout, natural weighting",
    "widefield_rot": "widefield 128 tiles (8128 baselines), 768 ch x 100 timesteps, 1024^2 grid -> 512^2 cutout, natural weighting, phase centre rotated to (l, m) = (0.05, 0.03) and per-antenna cable lengths (uniform 0-500 m) corrected at load",
    "widefield_kb": "widefield 128 tiles (8128 baselines), 768 ch x 100 timesteps, 1024^2 grid -> 512^2 cutout, natural weighting, Kaiser-Bessel gridding kernel of 6 cells with taper correction",
    "plain": "plain single image, 32 antennas (496 baselines), 1 ch at 160 MHz, 128^2, natural weighting",
    "allsky": "station all-sky, 256 antennas (32640 baselines), 32 ch x 1000 timesteps (32,000 images), 180^2, uniform weighting, 2-10% flagged per timestep",
    "precision": "precision, 256 tiles in 5 km (32640 baselines), 384 ch x 50 timesteps, 2048^2, uniform weighting",
    "diff": "differentiation, widefield layout, 32 ch x 10 timesteps (320 images) 1024^2 -> 512^2, gains, loss ||I - I_model||^2",
}


def _timed_steps(blink, torch, args, run):
    """Warm-up, then K timed calls of run(k, times); returns (total ms, per-class ms and launches)."""
    times = blink.KernelTimes()
    for k in range(args.warmup):
        run(k, None)
    torch.cuda.synchronize()
    acc_ms, acc_n = [0.0] * 4, [0] * 4
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    for k in range(args.steps):
        run(k, times)
        for c in range(4):
            acc_ms[c] += times.ms[c]
            acc_n[c] += times.launches[c]
    ev1.record()
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1), acc_ms, acc_n


def _roofline(blink, acc_ms, acc_n, per_image, imgs_timed, digest_ok_kernel=None):
    classes = blink.KCLASS
    dom = max(range(4), key=lambda c: acc_ms[c])
    name = classes[dom]
    mean_ms = acc_ms[dom] / max(acc_n[dom], 1)
    bytes_per_launch = per_image.get(name, 0) * imgs_timed / max(acc_n[dom], 1)
    achieved = bytes_per_launch / (mean_ms * 1e-3) / 1e9 if mean_ms > 0 else 0.0
    traffic = None
    if digest_ok_kernel and os.path.exists(TRAFFIC_FILE):
        tr = json.load(open(TRAFFIC_FILE))
        ipl = imgs_timed / max(acc_n[dom], 1)
        if (tr.get("csrc_digest") == _csrc_digest() and name in tr.get("kernels", {})
                and abs(tr["kernels"][name].get("images_per_launch", 0) - ipl) < 0.5):
            traffic = tr["kernels"][name].get("hbm_bytes_per_launch")
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": name, "mean_launch_ms": round(mean_ms, 5),
            "algorithmic_bytes_per_launch": int(bytes_per_launch),
            "images_per_launch": round(imgs_timed / max(acc_n[dom], 1), 2)}


def bench_images(args, np, torch, blink, synth, dev):
    w, TT = _setup(args, synth)
    n_batches = w.n_time // TT
    t_gen = time.perf_counter()
    vis = synth.visibilities(w, device=dev)
    uvw = torch.from_numpy(w.uvw_m).to(dev)
    freq = torch.from_numpy(w.freq_hz).to(dev)
    flags = None if w.flags is None else torch.from_numpy(w.flags).to(dev)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t_gen
    n_img = TT * w.n_chan
    M, N, H, B = w.out_n, w.grid_n, w.grid_n // 2, w.n_bl
    ksup = KB_SUPPORT if args.workload == "widefield_kb" else 0
    plm = ROT_LM if args.workload == "widefield_rot" else (0.0, 0.0)
    cable = ant1 = ant2 = None
    if args.workload == "widefield_rot":
        cable = torch.from_numpy(np.random.default_rng(2405).uniform(0.0, CABLE_MAX_M, w.n_ant)).to(dev)
        ant1 = torch.from_numpy(w.ant1).to(dev)
        ant2 = torch.from_numpy(w.ant2).to(dev)
    images = torch.empty((n_img, M, M), dtype=torch.float32, device=dev)   # reused per step
    ws_cache = {}

    tunings = {}

    def make_run(v, scale, vbytes):
        # launch shapes: explicit flags win, else the autotuner's cache for this shape
        tun = blink.blink.tuning_for(N, M, B, w.weighting, blink.blink._vis_type(v), args.chunk,
                                     args.cols_per_wg, args.rows_wg)
        tunings[vbytes] = tun
        p = blink.blink.make_problem(v[:TT], uvw[:TT], freq, N, w.pixscale, M, w.weighting, w.norm,
                                     None, **tun, kernel_support=ksup, phase_lm=plm, cable_m=cable)
        ws_cache[vbytes] = ws = blink.workspace(p, blink.CALL_IMAGE, dev)

        def run(k, tm):
            b = k % n_batches
            sl = slice(b * TT, (b + 1) * TT)
            blink.image_batch(v[sl], uvw[sl], freq, grid_n=N, pixscale=w.pixscale, out_n=M,
                              weighting=w.weighting, norm=w.norm, flags=None if flags is None else flags[sl],
                              vis_scale=scale, images=images, ws=ws, times=tm, **tun, kernel_support=ksup,
                              phase_lm=plm, ant1=ant1, ant2=ant2, cable_m=cable)
        return run

    ncz = np.concatenate([nonzero_columns(w, slice(b * TT, (b + 1) * TT))
                          for b in range(min(args.steps, n_batches))])
    unflagged = (B if w.flags is None else
                 float(np.mean([(w.flags[t] == 0).sum() for t in range(min(args.steps, n_batches) * TT)])))
    if ksup:   # a kernel reaches up to floor(W/2 + 1/2) columns beyond the outermost baseline's
        ncz = np.minimum(ncz + (ksup + 1) // 2, H)
    ncz_mean = float(ncz.mean())

    def measure(v, scale, vbytes):
        total_ms, acc_ms, acc_n = _timed_steps(blink, torch, args, make_run(v, scale, vbytes))
        per_image = {"grid_cols": unflagged * vbytes + ncz_mean * M * 8,
                     "rows": ncz_mean * M * 8 + M * M * 4}
        img_per_s = n_img * args.steps / (total_ms / 1e3)
        roof = _roofline(blink, acc_ms, acc_n, per_image, n_img * args.steps,
                         digest_ok_kernel=args.workload == "widefield" and vbytes == 8)
        path_bytes = per_image["grid_cols"] + per_image["rows"]
        return {"images_per_s": img_per_s, "ms_per_step": total_ms / args.steps, "roofline": roof,
                "kernel_ms_per_step": {blink.KCLASS[c]: round(acc_ms[c] / args.steps, 4) for c in range(4)},
                "path_hbm_frac_algorithmic": round(path_bytes * img_per_s / 1e9 / HBM_PEAK_GBS, 4)}

    res = measure(vis, None, 8)
    dtype = "f32"
    extra = {}
    if args.workload == "precision":
        # FP16 and BF16 storage (per-channel scale), FP32 accumulation; FP16 is the headline
        forms = {"f32": res}
        errs = {}
        sample = [0, w.n_chan // 2]
        import oracle
        ref64, _ = oracle.image_batch(vis[:1].cpu().numpy(), w.uvw_m[:1], w.freq_hz, N, w.pixscale, M,
                                      w.weighting, w.norm, images=sample)
        blink.image_batch(vis[:1], uvw[:1], freq, grid_n=N, pixscale=w.pixscale, out_n=M,
                          weighting=w.weighting, norm=w.norm, images=images[:w.n_chan])
        f32img = images[sample].cpu().double().numpy()
        errs["f32"] = [float(np.linalg.norm(a - r) / np.linalg.norm(r)) for a, r in zip(f32img, ref64)]
        for name, dt in (("f16", torch.float16), ("bf16", torch.bfloat16)):
            q, sig = synth.quantize_vis(vis, dt)
            forms[name] = measure(q, sig, 4)
            blink.image_batch(q[:1], uvw[:1], freq, grid_n=N, pixscale=w.pixscale, out_n=M,
                              weighting=w.weighting, norm=w.norm, vis_scale=sig, images=images[:w.n_chan])
            got = images[sample].cpu().double().numpy()
            errs[name] = {"rel_l2_vs_fp64_oracle": [float(np.linalg.norm(a - r) / np.linalg.norm(r)) for a, r in zip(got, ref64)],
                          "rel_l2_vs_fp32_gpu": [float(np.linalg.norm(a - r) / np.linalg.norm(r)) for a, r in zip(got, f32img)],
                          "peak_abs_err_vs_fp64": [float(np.abs(a - r).max()) for a, r in zip(got, ref64)]}
            del q
        res = forms["f16"]
        dtype = "f16 storage, f32 arithmetic"
        extra["forms"] = {k: {"images_per_s": round(v["images_per_s"], 1), "ms_per_step": round(v["ms_per_step"], 4),
                              "kernel_ms_per_step": v["kernel_ms_per_step"], "roofline_frac": v["roofline"]["frac"]}
                          for k, v in forms.items()}
        extra["errors_sampled_images"] = errs

    if args.workload == "widefield" and args.plain_loop > 0:
        # the plain per-image path on the same GPU: one library call per image
        p1 = blink.blink.make_problem(vis[:1, :1], uvw[:1], freq[:1], N, w.pixscale, M, w.weighting, w.norm)
        ws1 = blink.workspace(p1, blink.CALL_IMAGE, dev)
        one = torch.empty((1, M, M), dtype=torch.float32, device=dev)
        idx = [(i // w.n_chan, i % w.n_chan) for i in range(args.plain_loop)]

        def single(t, c):
            blink.image_batch(vis[t:t + 1, c:c + 1], uvw[t:t + 1], freq[c:c + 1], grid_n=N, pixscale=w.pixscale,
                              out_n=M, weighting=w.weighting, norm=w.norm, images=one, ws=ws1)
        for t, c in idx[:8]:
            single(t, c)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for t, c in idx:
            single(t, c)
        e1.record()
        torch.cuda.synchronize()
        extra["plain_per_image_loop"] = {"images_per_s": round(len(idx) / (e0.elapsed_time(e1) / 1e3), 1),
                                         "images": len(idx), "us_per_image": round(e0.elapsed_time(e1) * 1e3 / len(idx), 2)}

    img_per_s = res["images_per_s"]
    out = {
        "metric": METRIC if args.workload == "widefield" else f"dirty images/s ({args.workload})",
        "value": round(img_per_s, 1), "unit": "images/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(res["ms_per_step"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": DESCRIPTION[args.workload], "images_per_step": n_img,
                   "timesteps_per_step": TT, "grid_n": N, "out_n": M, "baselines": B,
                   "channels": w.n_chan, "launch": tunings.get(8)},
        "visibilities_per_s": round(img_per_s * unflagged, 1),
        "nonzero_half_spectrum_columns_mean": round(ncz_mean, 2),
        "path_hbm_frac_algorithmic": res["path_hbm_frac_algorithmic"],
        "path_hbm_frac_model_iii": round((unflagged * 8 + H * M * 8 * 2 + M * M * 4) * img_per_s / 1e9 / HBM_PEAK_GBS, 4),
        "path_hbm_frac_model_i": round((unflagged * 8 + 2 * N * N * 8 + M * M * 4) * img_per_s / 1e9 / HBM_PEAK_GBS, 4),
        "kernel_ms_per_step": res["kernel_ms_per_step"],
        "roofline": res["roofline"],
        "input_generation_s": round(t_gen, 2),
    }
    out.update(extra)
    if args.workload == "plain":
        # the instrumented call above waits on an event pair around every launch;
        # the plain path's own costs: back-to-back calls (the host enqueues the
        # next while the GPU runs) and one call waited for on its own
        one = torch.empty((1, M, M), dtype=torch.float32, device=dev)
        p1 = blink.blink.make_problem(vis, uvw, freq, N, w.pixscale, M, w.weighting, w.norm)
        ws1 = blink.workspace(p1, blink.CALL_IMAGE, dev)

        def call():
            blink.image_batch(vis, uvw, freq, grid_n=N, pixscale=w.pixscale, out_n=M, weighting=w.weighting,
                              norm=w.norm, images=one, ws=ws1)
        for _ in range(20):
            call()
        torch.cuda.synchronize()
        nl = 500
        t0 = time.perf_counter()
        for _ in range(nl):
            call()
        torch.cuda.synchronize()
        loop_us = (time.perf_counter() - t0) / nl * 1e6
        lat = []
        for _ in range(200):
            t0 = time.perf_counter()
            call()
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - t0)
        lat.sort()
        out["latency_us_per_image"] = round(res["ms_per_step"] * 1e3, 2)
        out["back_to_back_us_per_call"] = round(loop_us, 2)
        out["single_call_latency_us_median"] = round(lat[len(lat) // 2] * 1e6, 2)
        out["latency_note"] = ("latency_us_per_image times the instrumented entry point (an event pair and a "
                               "host wait around every launch); back_to_back_us_per_call is the plain "
                               "call in a loop, single_call_latency_us_median one call and a synchronisation")

    sample_n = args.cpu_sample if args.cpu_sample is not None else {"widefield": 128, "widefield_kb": 32, "widefield_rot": 0, "plain": 64, "allsky": 4096, "precision": 16}[args.workload]
    if not args.no_cpu_baseline and sample_n > 0:
        cores = max(1, min(16, os.cpu_count() or 1))
        S = min(sample_n, w.n_img)
        stride = max(1, w.n_chan // S)
        sample = [(k * stride) % w.n_chan + ((k * stride) // w.n_chan) * w.n_chan for k in range(S)]
        tmax = max(sample) // w.n_chan + 1
        vis_cpu = vis[:tmax].cpu().numpy()
        rate, dt = cpu_baseline(w, vis_cpu, sample, cores, ksup)
        out["cpu_baseline"] = {"value": round(rate, 3), "unit": "images/s", "cores": cores, "kind": "oracle",
                               "sample": f"{S} images (timesteps < {tmax}, channels every {stride}) of the same "
                                         f"workload, FP64 numpy oracle, {cores}-process pool, {dt:.1f} s wall"}
    print(json.dumps(out), flush=True)


def bench_diff(args, np, torch, blink, synth, dev):
    """Forward + backward (hand-written adjoint) of ||I - I_model||^2 w.r.t. vis and gains."""
    w = synth.widefield(n_time=10, n_chan=32, chan_stride=24)
    vis0 = synth.visibilities(w, device=dev)
    uvw = torch.from_numpy(w.uvw_m).to(dev)
    freq = torch.from_numpy(w.freq_hz).to(dev)
    gains0 = torch.from_numpy(w.gains).to(dev)
    a1 = torch.from_numpy(w.ant1).to(dev)
    a2 = torch.from_numpy(w.ant2).to(dev)
    rng = np.random.default_rng(20240521 + 4)
    model = np.zeros((w.n_img, w.out_n, w.out_n), np.float32)
    for i in range(w.n_img):
        idx = rng.integers(0, w.out_n, size=(2, 50))
        model[i, idx[0], idx[1]] = rng.uniform(1, 10, 50)
    target = torch.from_numpy(model).to(dev)

    def step():
        vis = vis0.clone().requires_grad_(True)
        g = gains0.clone().requires_grad_(True)
        img = blink.blink_image(vis, g, uvw, freq, a1, a2, grid_n=w.grid_n, pixscale=w.pixscale,
                                out_n=w.out_n, weighting=w.weighting, norm=w.norm)
        loss = ((img - target) ** 2).sum()
        loss.backward()
        return vis.grad, g.grad

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(args.steps):
        step()
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    # forward alone, for the split
    fw0, fw1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fw0.record()
    for _ in range(args.steps):
        blink.image_batch(vis0, uvw, freq, grid_n=w.grid_n, pixscale=w.pixscale, out_n=w.out_n,
                          weighting=w.weighting, norm=w.norm, gains=gains0, ant1=a1, ant2=a2)
    fw1.record()
    torch.cuda.synchronize()
    fwd_ms = fw0.elapsed_time(fw1) / args.steps
    # the library's adjoint alone (degridding + forward transforms + gain
    # gradient, reusing the forward weight sums), for the backward / forward ratio
    img0 = blink.image_batch(vis0, uvw, freq, grid_n=w.grid_n, pixscale=w.pixscale, out_n=w.out_n,
                             weighting=w.weighting, norm=w.norm, gains=gains0, ant1=a1, ant2=a2)
    wsum = torch.empty(w.n_img, dtype=torch.float32, device=dev)
    blink.image_batch(vis0, uvw, freq, grid_n=w.grid_n, pixscale=w.pixscale, out_n=w.out_n,
                      weighting=w.weighting, norm=w.norm, gains=gains0, ant1=a1, ant2=a2, weight_sum=wsum)
    gbar = (2 * (img0 - target)).contiguous()
    torch.cuda.synchronize()
    ad0, ad1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ad0.record()
    for _ in range(args.steps):
        blink.degrid_adjoint(gbar, vis0, uvw, freq, grid_n=w.grid_n, pixscale=w.pixscale, out_n=w.out_n,
                             weighting=w.weighting, norm=w.norm, gains=gains0, ant1=a1, ant2=a2,
                             weight_sum=wsum)
    ad1.record()
    torch.cuda.synchronize()
    adj_ms = ad0.elapsed_time(ad1) / args.steps
    out = {"metric": "dirty images/s forward + backward (diff)", "value": round(w.n_img / (ms / 1e3), 1),
           "unit": "images/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": DESCRIPTION["diff"], "images_per_step": w.n_img, "grid_n": w.grid_n,
                      "out_n": w.out_n, "baselines": w.n_bl, "antennas": w.n_ant},
           "forward_ms_per_step": round(fwd_ms, 4), "backward_ms_per_step": round(ms - fwd_ms, 4),
           "adjoint_call_ms_per_step": round(adj_ms, 4),
           "adjoint_over_forward": round(adj_ms / fwd_ms, 3),
           "backward_note": "backward_ms_per_step is the autograd step (torch's loss-gradient kernels "
                            "over the 320 images plus the adjoint call); adjoint_call_ms_per_step times "
                            "blink_degrid_adjoint alone",
           "roofline": None, "cpu_baseline": None}
    print(json.dumps(out), flush=True)


def bench_dynspec(args, np, torch, blink, synth, dev):
    """Dynamic spectra of a cube of widefield dirty images, mean of 8 preceding images subtracted."""
    T, C, K = 100, 96, 8
    w = synth.widefield(n_time=T, n_chan=C, chan_stride=8)
    vis = synth.visibilities(w, device=dev)
    M = w.out_n
    cube = blink.image_batch(vis, torch.from_numpy(w.uvw_m).to(dev), torch.from_numpy(w.freq_hz).to(dev),
                             grid_n=w.grid_n, pixscale=w.pixscale, out_n=M, weighting=w.weighting,
                             norm=w.norm).view(T, C, M, M)
    del vis
    out = torch.empty((M * M, C, T), dtype=torch.float32, device=dev)
    for _ in range(args.warmup):
        blink.dynamic_spectra(cube, blink.REF_MEAN, K, out=out)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()       # the library launches on the caller's current stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(args.steps):
        blink.dynamic_spectra(cube, blink.REF_MEAN, K, out=out)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    # the plain transposition (no reference) on the same cube, for comparison
    e0.record(st)
    for _ in range(args.steps):
        blink.dynamic_spectra(cube, blink.REF_NONE, out=out)
    e1.record(st)
    torch.cuda.synchronize()
    ms_none = e0.elapsed_time(e1) / args.steps
    n_img = T * C
    alg = 2.0 * n_img * M * M * 4                 # every pixel read once and written once
    achieved = alg / (ms * 1e-3) / 1e9
    out_line = {
        "metric": "dirty images/s (dynspec)", "value": round(n_img / (ms / 1e3), 1), "unit": "images/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32 (f64 window sums)",
        "data": "synthetic",
        "config": {"workload": f"dynamic spectra of {T} timesteps x {C} channels of 512^2 widefield dirty "
                               f"images ({alg / 2e9:.1f} GB), mean of the {K} preceding images subtracted",
                   "images_per_step": n_img, "out_n": M, "ref_len": K},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": "dynspec",
                     "mean_launch_ms": round(ms, 5), "algorithmic_bytes_per_launch": int(alg),
                     "images_per_launch": n_img},
        "transpose_only_ms_per_step": round(ms_none, 4),
    }
    if not args.no_cpu_baseline:
        import oracle
        sub = cube[:, :4].cpu().numpy()
        t0 = time.perf_counter()
        oracle.dynamic_spectra.dynamic_spectra(sub, 1, K)
        dt = time.perf_counter() - t0
        out_line["cpu_baseline"] = {"value": round(T * 4 / dt, 3), "unit": "images/s", "cores": 1,
                                    "kind": "oracle",
                                    "sample": f"{T} timesteps x 4 channels of the same cube (numpy, one thread), "
                                              f"{dt:.1f} s"}
    print(json.dumps(out_line), flush=True)


INT8_PEAK_TOPS = 5000.0         # MI355X dense int8 matrix peak, TOP/s


def bench_xengine(args, np, torch, blink, dev):
    """Correlator X-engine: 256 antennas, 32 channels, 64 integrations of 4096 int8 samples."""
    T, C, A, S = 64, 32, 256, 4096
    g = torch.Generator(device=dev)
    g.manual_seed(20240521 + 6)
    volt = torch.randint(-128, 128, (T, C, A, S, 2), dtype=torch.int8, device=dev, generator=g)
    B = A * (A - 1) // 2
    vis = torch.empty((T, C, B), dtype=torch.complex64, device=dev)
    for _ in range(args.warmup):
        blink.correlate(volt, vis=vis)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(args.steps):
        blink.correlate(volt, vis=vis)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    n = T * C
    ops = 8.0 * (A * (A + 1) / 2) * S * n          # 4 real multiply-adds per complex product, pairs incl. autos
    hbm = n * (A * S * 2 + B * 8)
    out = {
        "metric": "integrations x channels correlated/s (xengine)", "value": round(n / (ms / 1e3), 1),
        "unit": "spectra/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "i8 (i32 accumulation)",
        "data": "synthetic",
        "config": {"workload": f"X-engine: {A} antennas ({B} baselines), {C} channels x {T} integrations of "
                               f"{S} complex int8 samples", "antennas": A, "samples": S, "spectra_per_step": n},
        "roofline": {"bound": "mfma", "achieved": round(ops / (ms * 1e-3) / 1e12, 1), "peak": INT8_PEAK_TOPS,
                     "unit": "TOP/s", "frac": round(ops / (ms * 1e-3) / 1e12 / INT8_PEAK_TOPS, 4), "traffic": None,
                     "kernel": "xengine", "mean_launch_ms": round(ms, 5), "algorithmic_ops_per_launch": ops,
                     "hbm_gbs_algorithmic": round(hbm / (ms * 1e-3) / 1e9, 1)},
    }
    if not args.no_cpu_baseline:
        import oracle
        from threadpoolctl import threadpool_info
        sub = volt[:1, :16].cpu().numpy()
        t0 = time.perf_counter()
        oracle.correlator.correlate(sub)
        dt = time.perf_counter() - t0
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
        out["cpu_baseline"] = {"value": round(16 / dt, 3), "unit": "spectra/s", "cores": threads, "kind": "oracle",
                               "sample": f"1 integration x 16 channels of the same data (numpy complex matmul), "
                                         f"{dt:.2f} s"}
    print(json.dumps(out), flush=True)


# ---------------------------------------------------------------- main
def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", default="widefield",
                    choices=("widefield", "widefield_kb", "widefield_rot", "plain", "allsky", "diff", "precision",
                             "dynspec", "xengine"))
    ap.add_argument("--timesteps-per-step", type=int, default=None)
    ap.add_argument("--timesteps", type=int, default=None,
                    help="timesteps of the job generated into HBM (default: the whole widefield job)")
    ap.add_argument("--chunk", type=int, default=None, help="images per internal chunk (default: tuned)")
    ap.add_argument("--cols-per-wg", type=int, default=None, help="column kernel tile width (default: tuned)")
    ap.add_argument("--rows-wg", type=int, default=None, help="persistent row-pass grid (default: tuned)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=None)
    ap.add_argument("--plain-loop", type=int, default=256,
                    help="widefield: also time this many single-image calls (0 = skip)")
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
    defaults = {"widefield": (20, 3), "widefield_kb": (10, 2), "widefield_rot": (20, 3), "plain": (500, 20),
                "allsky": (3, 1),
                "diff": (5, 2), "precision": (5, 1), "dynspec": (10, 2), "xengine": (10, 2)}
    ds, dw = defaults[args.workload]
    args.steps = ds if args.steps is None else args.steps
    args.warmup = dw if args.warmup is None else args.warmup

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
    if args.workload == "diff":
        bench_diff(args, np, torch, blink, synth, dev)
    elif args.workload == "dynspec":
        bench_dynspec(args, np, torch, blink, synth, dev)
    elif args.workload == "xengine":
        bench_xengine(args, np, torch, blink, dev)
    else:
        bench_images(args, np, torch, blink, synth, dev)


if __name__ == "__main__":
    main()
