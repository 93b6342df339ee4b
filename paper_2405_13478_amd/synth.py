"""Seeded synthetic workloads: array layouts, sky models, visibilities, flags.

This module produces inputs only. It holds none of the imaging arithmetic
(no cell indexing, gridding, weighting or transforms); it is shared by the
tests, the benchmark and the CPU baseline so that the HIP path and the
oracle see exactly the same bytes.

Visibilities follow the paper's forward model (Sec. 4.3, Eq. 5, w = 0):
V_b(nu) = sum_s S_s(nu) exp(-2 pi i (u_b l_s + v_b m_s) nu / c) + noise,
with (u_b, v_b) in metres and noise ~ sigma (N(0,1) + i N(0,1)).

The five workloads stand in for the paper's EDA2 / MWA observations (which
are not available): they take the instrument shapes of Sec. 3 and Sec. 6
(a 256-antenna station imaged at 180^2 with 32 channels of 100 ms
integrations, a 128-tile array at 1024^2, and larger grids).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import torch

C_LIGHT = 299792458.0          # m/s
OMEGA_EARTH = 7.2921e-5        # rad/s, sidereal rotation rate
DT = 0.1                       # s, integration time of the production runs
BASE_SEED = 20240521

NATURAL, UNIFORM = 0, 1
NORM_NONE, NORM_WEIGHTS = 0, 1


@dataclasses.dataclass
class Workload:
    """One imaging problem: geometry, sky, and the parameters of the imager."""
    name: str
    n_ant: int
    n_time: int
    n_chan: int
    grid_n: int
    out_n: int
    pixscale: float
    weighting: int
    norm: int
    freq_hz: np.ndarray            # [C] float64
    ant_xy: np.ndarray             # [A][2] float64 metres (E, N)
    ant1: np.ndarray               # [B] int32
    ant2: np.ndarray               # [B] int32
    uvw_m: np.ndarray              # [T][B][3] float64
    flags: np.ndarray | None       # [T][B] uint8 or None
    src_l: np.ndarray              # [S]
    src_m: np.ndarray              # [S]
    src_flux: np.ndarray           # [S][C] Jy at each channel
    noise_sigma: float
    vis_seed: int
    gains: np.ndarray | None = None    # [A] complex64

    @property
    def n_bl(self) -> int:
        return int(self.ant1.shape[0])

    @property
    def n_img(self) -> int:
        return self.n_time * self.n_chan


# ---------------------------------------------------------------------------
# geometry
# ---------------------------------------------------------------------------
def disc_positions(n: int, radius: float, rng) -> np.ndarray:
    """n points uniform by area in a disc: r = R sqrt(U), theta = 2 pi U'."""
    r = radius * np.sqrt(rng.random(n))
    th = 2.0 * np.pi * rng.random(n)
    return np.stack([r * np.cos(th), r * np.sin(th)], axis=1)


def baseline_pairs(n_ant: int):
    """All antenna pairs i < j (no autocorrelations): N(N-1)/2 baselines."""
    a1, a2 = np.triu_indices(n_ant, k=1)
    return a1.astype(np.int32), a2.astype(np.int32)


def baseline_uvw(ant_xy, ant1, ant2, n_time: int, t0: int = 0) -> np.ndarray:
    """uvw in metres per timestep for a coplanar array phased to zenith.

    The (E, N) baseline vectors are rotated by omega_earth * t * dt so that
    every timestep has its own cell indices (a synthetic stand-in for the
    slow uv-track motion; w = 0).
    """
    d = ant_xy[ant2] - ant_xy[ant1]              # [B][2]
    out = np.zeros((n_time, d.shape[0], 3), dtype=np.float64)
    for t in range(n_time):
        th = OMEGA_EARTH * (t0 + t) * DT
        c, s = math.cos(th), math.sin(th)
        out[t, :, 0] = d[:, 0] * c - d[:, 1] * s
        out[t, :, 1] = d[:, 0] * s + d[:, 1] * c
    return out


def oversampled_pixscale(max_baseline_m: float, freq_max_hz: float, os: float = 3.0) -> float:
    """dx = 1 / (os * u_max): the synthesised beam sampled `os` times (Sec. 4.4.1)."""
    u_max = max_baseline_m * freq_max_hz / C_LIGHT
    return 1.0 / (os * u_max)


def random_flags(n_time: int, n_bl: int, rng, lo=0.02, hi=0.10) -> np.ndarray:
    """Per timestep a fraction f ~ U[lo, hi] of baselines, drawn without replacement."""
    fl = np.zeros((n_time, n_bl), dtype=np.uint8)
    for t in range(n_time):
        k = int(round(rng.uniform(lo, hi) * n_bl))
        fl[t, rng.choice(n_bl, size=k, replace=False)] = 1
    return fl


# ---------------------------------------------------------------------------
# visibilities
# ---------------------------------------------------------------------------
def visibilities(w: Workload, device="cpu", t_range=None, c_range=None,
                 src_chunk: int = 8) -> torch.Tensor:
    """complex64 vis[T][C][B] from the point-source sky plus Gaussian noise.

    Phases are formed and reduced to [0, 1) turns in float64, then the
    exponentials are summed in complex128 and cast to complex64 once.
    """
    dev = torch.device(device)
    t0, t1 = (0, w.n_time) if t_range is None else t_range
    c0, c1 = (0, w.n_chan) if c_range is None else c_range
    T, C, B = t1 - t0, c1 - c0, w.n_bl
    uv = torch.from_numpy(np.ascontiguousarray(w.uvw_m[t0:t1, :, :2])).to(dev)      # [T][B][2]
    lam_inv = torch.from_numpy(w.freq_hz[c0:c1] / C_LIGHT).to(dev)               # [C]
    l = torch.from_numpy(w.src_l).to(dev)
    m = torch.from_numpy(w.src_m).to(dev)
    flux = torch.from_numpy(np.ascontiguousarray(w.src_flux[:, c0:c1])).to(dev)  # [S][C]
    out = torch.empty((T, C, B), dtype=torch.complex64, device=dev)
    gen = torch.Generator(device=dev)
    for t in range(T):
        acc = torch.zeros((C, B), dtype=torch.complex128, device=dev)
        for s0 in range(0, l.numel(), src_chunk):
            s1 = min(s0 + src_chunk, l.numel())
            # path difference in metres for each (source, baseline)
            pd = uv[t, :, 0][None, :] * l[s0:s1, None] + uv[t, :, 1][None, :] * m[s0:s1, None]
            turns = pd[:, None, :] * lam_inv[None, :, None]            # [s][C][B]
            turns = turns - torch.floor(turns)
            ph = torch.polar(torch.ones_like(turns), -2.0 * math.pi * turns)
            acc += (flux[s0:s1, :, None] * ph).sum(0)
        gen.manual_seed(w.vis_seed * 1000003 + t0 + t)
        nre = torch.randn((C, B), generator=gen, device=dev, dtype=torch.float64)
        nim = torch.randn((C, B), generator=gen, device=dev, dtype=torch.float64)
        acc += w.noise_sigma * torch.complex(nre, nim)
        out[t] = acc.to(torch.complex64)
    return out


def quantize_vis(vis: torch.Tensor, dtype: torch.dtype):
    """Per-channel scaled half-precision storage of vis[T][C][B].

    sigma_c = max over (t, b) of max(|Re V|, |Im V|) (as float32); the stored
    pair is round-to-nearest-even of (Re V / sigma_c, Im V / sigma_c) in
    ``dtype`` (float16 or bfloat16), interleaved as [T][C][B][2].
    Returns (stored, sigma[C] float32).
    """
    re = vis.real.float()
    im = vis.imag.float()
    sig = torch.maximum(re.abs().amax(dim=(0, 2)), im.abs().amax(dim=(0, 2)))
    sig = torch.where(sig > 0, sig, torch.ones_like(sig))
    q = torch.stack([re / sig[None, :, None], im / sig[None, :, None]], dim=-1).to(dtype)
    return q.contiguous(), sig.contiguous()


# ---------------------------------------------------------------------------
# the five workloads
# ---------------------------------------------------------------------------
def _streams(k: int):
    ss = np.random.SeedSequence(BASE_SEED + k)
    return [np.random.default_rng(s) for s in ss.spawn(5)]  # pos, src, noise, flags, gains


def plain_single(n_time: int = 1) -> Workload:
    """32 antennas in a 35 m disc, 496 baselines, 1 channel at 160 MHz, 128^2, natural."""
    r_pos, r_src, r_noise, _, _ = _streams(1)
    xy = disc_positions(32, 35.0, r_pos)
    a1, a2 = baseline_pairs(32)
    freq = np.array([160e6])
    ns = 3
    return Workload(
        name="plain single image, 32 antennas, 128x128", n_ant=32, n_time=n_time,
        n_chan=1, grid_n=128, out_n=128,
        pixscale=oversampled_pixscale(70.0, 160e6), weighting=NATURAL,
        norm=NORM_WEIGHTS, freq_hz=freq, ant_xy=xy, ant1=a1, ant2=a2,
        uvw_m=baseline_uvw(xy, a1, a2, n_time), flags=None,
        src_l=r_src.uniform(-0.5, 0.5, ns), src_m=r_src.uniform(-0.5, 0.5, ns),
        src_flux=np.repeat(r_src.uniform(1, 10, ns)[:, None], 1, axis=1),
        noise_sigma=0.1, vis_seed=int(r_noise.integers(1 << 30)))


def station_allsky(n_time: int = 1000, n_chan: int = 32) -> Workload:
    """256 antennas in a 35 m disc (32640 baselines), 150-180 MHz, 180^2, uniform, 2-10% flags."""
    r_pos, r_src, r_noise, r_flag, _ = _streams(2)
    xy = disc_positions(256, 35.0, r_pos)
    a1, a2 = baseline_pairs(256)
    freq = np.linspace(150e6, 180e6, 32)[:n_chan]
    ns = 20
    rr = np.sqrt(r_src.random(ns))
    th = 2 * np.pi * r_src.random(ns)
    return Workload(
        name="station all-sky, 256 antennas, 180x180, uniform", n_ant=256,
        n_time=n_time, n_chan=len(freq), grid_n=180, out_n=180, pixscale=2.0 / 180,
        weighting=UNIFORM, norm=NORM_WEIGHTS, freq_hz=freq, ant_xy=xy, ant1=a1,
        ant2=a2, uvw_m=baseline_uvw(xy, a1, a2, n_time),
        flags=random_flags(n_time, len(a1), r_flag),
        src_l=rr * np.cos(th), src_m=rr * np.sin(th),
        src_flux=np.repeat(r_src.uniform(1, 10, ns)[:, None], len(freq), axis=1),
        noise_sigma=0.1, vis_seed=int(r_noise.integers(1 << 30)))


def _widefield_freqs(n_chan_total=768, centre=185e6, width=40e3):
    return centre + (np.arange(n_chan_total) - (n_chan_total - 1) / 2.0) * width


def widefield(n_time: int = 100, n_chan: int = 768, chan_stride: int = 1,
              t0: int = 0) -> Workload:
    """128 tiles (64 in a 300 m core, 64 in a 3 km disc), 8128 baselines,
    768 x 40 kHz channels centred at 185 MHz, 1024^2 grid cut to 512^2, natural.

    ``n_chan``/``chan_stride`` select channels [0, n_chan*stride, stride) of
    the 768; ``t0`` offsets the timesteps (for benchmark batches).
    """
    r_pos, r_src, r_noise, _, r_gain = _streams(3)
    xy = np.concatenate([disc_positions(64, 300.0, r_pos), disc_positions(64, 3000.0, r_pos)])
    a1, a2 = baseline_pairs(128)
    fall = _widefield_freqs()
    freq = fall[: n_chan * chan_stride: chan_stride]
    dx = oversampled_pixscale(6000.0, fall.max())
    ns = 200
    half = 512 * dx / 2
    s0 = r_src.uniform(1, 10, ns)
    flux = s0[:, None] * (freq[None, :] / 185e6) ** -0.8
    gains = (1 + r_gain.normal(0, 0.05, 128) + 1j * r_gain.normal(0, 0.05, 128)).astype(np.complex64)
    return Workload(
        name="widefield, 128 tiles, 1024x1024 -> 512x512, natural", n_ant=128,
        n_time=n_time, n_chan=len(freq), grid_n=1024, out_n=512, pixscale=dx,
        weighting=NATURAL, norm=NORM_WEIGHTS, freq_hz=freq, ant_xy=xy, ant1=a1,
        ant2=a2, uvw_m=baseline_uvw(xy, a1, a2, n_time, t0), flags=None,
        src_l=r_src.uniform(-half, half, ns), src_m=r_src.uniform(-half, half, ns),
        src_flux=flux, noise_sigma=0.1, vis_seed=int(r_noise.integers(1 << 30)),
        gains=gains)


def precision_station(n_time: int = 50, n_chan: int = 384) -> Workload:
    """256 tiles in a 5 km disc (32640 baselines), 384 x 40 kHz at 200 MHz, 2048^2, uniform."""
    r_pos, r_src, r_noise, _, _ = _streams(5)
    xy = disc_positions(256, 5000.0, r_pos)
    a1, a2 = baseline_pairs(256)
    fall = 200e6 + (np.arange(384) - 191.5) * 40e3
    freq = fall[:n_chan]
    dx = oversampled_pixscale(10000.0, fall.max())
    ns = 200
    half = 2048 * dx / 2
    s0 = r_src.uniform(1, 10, ns)
    flux = s0[:, None] * (freq[None, :] / 200e6) ** -0.8
    return Workload(
        name="precision, 256 tiles, 2048x2048, uniform", n_ant=256, n_time=n_time,
        n_chan=len(freq), grid_n=2048, out_n=2048, pixscale=dx, weighting=UNIFORM,
        norm=NORM_WEIGHTS, freq_hz=freq, ant_xy=xy, ant1=a1, ant2=a2,
        uvw_m=baseline_uvw(xy, a1, a2, n_time), flags=None,
        src_l=r_src.uniform(-half, half, ns), src_m=r_src.uniform(-half, half, ns),
        src_flux=flux, noise_sigma=0.1, vis_seed=int(r_noise.integers(1 << 30)))


def subset_antennas(w: Workload, n_keep: int, grid_n: int, seed: int = 4) -> Workload:
    """A seeded antenna subset of ``w`` on its own grid (os = 3 on its longest baseline)."""
    rng = np.random.default_rng(BASE_SEED + 100 + seed)
    keep = np.sort(rng.choice(w.n_ant, size=n_keep, replace=False))
    xy = w.ant_xy[keep]
    a1, a2 = baseline_pairs(n_keep)
    d = xy[a2] - xy[a1]
    bmax = float(np.sqrt((d ** 2).sum(1)).max())
    dx = oversampled_pixscale(bmax, float(w.freq_hz.max()))
    out = dataclasses.replace(
        w, name=w.name + f" ({n_keep}-antenna subset, {grid_n}^2)", n_ant=n_keep,
        grid_n=grid_n, out_n=grid_n, pixscale=dx, ant_xy=xy, ant1=a1, ant2=a2,
        uvw_m=baseline_uvw(xy, a1, a2, w.n_time), flags=None,
        gains=None if w.gains is None else w.gains[keep])
    return out
