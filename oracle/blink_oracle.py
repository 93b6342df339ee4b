"""Plain FP64 CPU oracle of the BLINK dirty-imaging path (grid + 2D inverse FFT).

TEST INFRASTRUCTURE ONLY. This module is the slow, obviously correct reference
that the HIP library is checked against. Only the test suite, the smoke check
of the package entry point and the CPU-baseline leg of the benchmark may
import it; the product path never calls into it, and it shares no code,
table or constant generator with the HIP sources.

Everything is numpy in float64 / complex128. No FFT library is used inside
the oracle: the inverse transform is a self-written recursive mixed-radix
decimation-in-time FFT (``fft_last_axis``) and, as a second independent
form, a separable DFT-matrix product (``dft2_matrix``).

What is computed, per image (timestep t, channel c), following the paper:

* Sec. 4.3, Eqs. 4-6: visibilities and the sky form a Fourier pair with
  kernel exp(-2 pi i (u l + v m)); the dirty image is the inverse transform
  of the sampled visibilities, so the image side uses exp(+2 pi i ...).
* Sec. 4.4.1, Eq. 9: the uv cell is du = dv = 1 / (N dx); a baseline of
  u metres lies at u * nu / c wavelengths, i.e. at u * s_c cells with
  s_c = nu_c * (N dx) / c.  Frequencies and wavelengths are handled in
  double precision (Sec. 5.2.4, multi-channel gridding kernel).
* Sec. 5.2.1: each visibility is added to the cell holding its (u, v)
  (nearest cell; no convolution kernel, Sec. 4.4.1), DC placed at the FFT
  origin, and a per-cell counter is incremented for weighting.
* Sec. 4.4.2: natural weighting sums the visibilities of a cell; uniform
  weighting weights by uv area so every occupied cell counts equally.
* Sec. 5.2.2: unnormalised 2D C2C inverse FFT, real part, then the FFT
  shift that moves the phase centre from the corner to the image centre.

Readings where the paper is silent (each is listed with its reason in the
design notes of the repository):

* rounding to a cell is round-half-to-even of the FP64 product (numpy rint);
* the keep range is symmetric, |i_u| < N/2 and |i_v| < N/2, so the grid is
  exactly Hermitian (the Nyquist row/column stays empty) and the image real;
* the input holds each baseline once; the library grids V at +k and its
  conjugate at -k (the full correlation matrix without autocorrelations);
* uniform weighting: cell value = cell sum / cell count; W = number of
  occupied cells. Natural: W = sum of counts;
* ``norm=1`` divides the image by W (a unit source at the phase centre gives
  a peak of 1; W = 0 gives an all-zero image), ``norm=0`` keeps the raw
  unnormalised transform;
* image layout [m][l]: row index follows v/m, column index follows u/l, both
  increasing, phase centre at [N/2][N/2]; the M x M cutout keeps rows and
  columns [N/2 - M/2, N/2 + M/2);
* gains: V' = g[a1] * conj(g[a2]) * V (one complex gain per antenna,
  Sec. 4.2 item (ii), applied post-correlation);
* reduced-precision storage: V = float(q) * sigma_c with q the stored
  fp16/bf16 value and sigma_c the per-channel scale.
"""
from __future__ import annotations

import math

import numpy as np

# Speed of light in m/s (SI exact value). The paper's kernel divides by a
# constant it does not print; the SI value is the only sensible reading.
C_LIGHT = 299792458.0

NATURAL = 0
UNIFORM = 1
NORM_NONE = 0
NORM_WEIGHTS = 1


# --------------------------------------------------------------------------
# Cell indexing (Sec. 4.4.1 Eq. 9; Sec. 5.2.1 step 1; Sec. 5.2.4)
# --------------------------------------------------------------------------
def uv_scale(freq_hz, grid_n: int, pixscale: float) -> np.ndarray:
    """Cells per metre for each channel: s_c = (nu_c * (N * dx)) / c.

    Eq. 9 gives du = 1 / (N dx) wavelengths per cell, and a baseline of u
    metres is u * nu / c wavelengths long, hence u * nu * N dx / c cells.
    Evaluated in IEEE double in exactly this order: N*dx, times nu, over c.
    """
    nf = np.asarray(freq_hz, dtype=np.float64)
    ndx = np.float64(grid_n) * np.float64(pixscale)
    return (nf * ndx) / np.float64(C_LIGHT)


def cell_index(u_m, v_m, s, grid_n: int, flagged=None):
    """Signed cell indices and the keep mask for baselines at one scale s.

    i_u = rint(u * s), i_v = rint(v * s), each a single correctly rounded
    double product followed by round-half-to-even. A baseline is kept iff it
    is not flagged and |i_u| < N/2 and |i_v| < N/2.
    Returns (i_u, i_v, keep) as (int64, int64, bool) arrays.
    """
    u = np.asarray(u_m, dtype=np.float64)
    v = np.asarray(v_m, dtype=np.float64)
    s = np.float64(s)
    iu = np.rint(u * s)
    iv = np.rint(v * s)
    half = grid_n // 2
    keep = (np.abs(iu) < half) & (np.abs(iv) < half)
    if flagged is not None:
        keep &= ~np.asarray(flagged, dtype=bool)
    iu = np.where(keep, iu, 0).astype(np.int64)
    iv = np.where(keep, iv, 0).astype(np.int64)
    return iu, iv, keep


# --------------------------------------------------------------------------
# Visibility load (Sec. 4.2 (ii) gains; reduced-precision storage)
# --------------------------------------------------------------------------
def apply_gains(vis, gains=None, ant1=None, ant2=None):
    """V' = g[a1] * conj(g[a2]) * V in complex128 (gains optional)."""
    v = np.asarray(vis).astype(np.complex128)
    if gains is None:
        return v
    g = np.asarray(gains).astype(np.complex128)
    return g[np.asarray(ant1)] * np.conj(g[np.asarray(ant2)]) * v


def dequantize(q_re, q_im, sigma):
    """Stored half-precision pair times the per-channel scale, in FP64.

    ``q_re``/``q_im`` are float16 arrays or bfloat16 bit patterns given as
    uint16 (then decoded by placing them in the top half of a float32).
    """
    def to64(q):
        q = np.asarray(q)
        if q.dtype == np.uint16:  # bfloat16 bit pattern
            return (q.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
        return q.astype(np.float64)
    return (to64(q_re) + 1j * to64(q_im)) * np.float64(sigma)


# --------------------------------------------------------------------------
# Gridding and weighting (Sec. 5.2.1 steps 2-3; Sec. 4.4.2)
# --------------------------------------------------------------------------
def grid(vis_prime, iu, iv, keep, grid_n: int):
    """Accumulate V' at (i_v mod N, i_u mod N) and conj(V') at the mirror cell.

    Returns (S, n): complex128 grid sums and int64 per-cell counts, both
    [N][N] with row = v cell, column = u cell, DC at [0][0].
    """
    n_ = grid_n
    S = np.zeros((n_, n_), dtype=np.complex128)
    cnt = np.zeros((n_, n_), dtype=np.int64)
    k = np.flatnonzero(np.asarray(keep))
    vp = np.asarray(vis_prime, dtype=np.complex128)[k]
    r = np.mod(iv[k], n_)
    c = np.mod(iu[k], n_)
    rb = np.mod(-iv[k], n_)
    cb = np.mod(-iu[k], n_)
    np.add.at(S, (r, c), vp)
    np.add.at(cnt, (r, c), 1)
    np.add.at(S, (rb, cb), np.conj(vp))
    np.add.at(cnt, (rb, cb), 1)
    return S, cnt


def weight(S, cnt, weighting: int):
    """Weighted grid G and weight sum W (Sec. 4.4.2).

    Natural: G = S, W = sum of counts. Uniform: G = S / n on occupied cells,
    W = number of occupied cells.
    """
    if weighting == NATURAL:
        return S.copy(), float(cnt.sum())
    if weighting == UNIFORM:
        occ = cnt > 0
        G = np.zeros_like(S)
        G[occ] = S[occ] / cnt[occ]
        return G, float(occ.sum())
    raise ValueError("unknown weighting")


# --------------------------------------------------------------------------
# Discrete Fourier transforms (Sec. 4.3 Eq. 6; Sec. 5.2.2)
# --------------------------------------------------------------------------
def _smallest_factor(n: int) -> int:
    for p in (2, 3, 5, 7):
        if n % p == 0:
            return p
    f = 11
    while f * f <= n:
        if n % f == 0:
            return f
        f += 2
    return n


def _root(e, n, sign):
    """exp(sign * 2 pi i * e / n) with e an exact integer already reduced mod n."""
    return np.exp(sign * 2j * np.pi * (np.asarray(e, dtype=np.float64) / n))


def fft_last_axis(x, sign: int):
    """Unnormalised DFT along the last axis: X[k] = sum_n x[n] exp(sign 2 pi i n k / N).

    Recursive mixed-radix decimation in time (Cooley-Tukey): split x into p
    interleaved subsequences x[r::p] (p the smallest prime factor), transform
    each, and combine X[k + m s] = sum_r w^(r (k + m s)) Y_r[k] with m = N/p.
    A prime length is summed directly. Exponents are reduced mod N as exact
    integers before the exponential.
    """
    x = np.asarray(x, dtype=np.complex128)
    n = x.shape[-1]
    if n == 1:
        return x.copy()
    p = _smallest_factor(n)
    if p == n:
        q = np.arange(n)
        mat = _root(np.outer(q, q) % n, n, sign)  # [k][n]
        return x @ mat.T
    m = n // p
    subs = [fft_last_axis(x[..., r::p], sign) for r in range(p)]
    k = np.arange(m)
    out = np.empty(x.shape, dtype=np.complex128)
    for s_ in range(p):
        acc = np.zeros(x.shape[:-1] + (m,), dtype=np.complex128)
        for r in range(p):
            acc += _root((r * (k + m * s_)) % n, n, sign) * subs[r]
        out[..., m * s_:m * (s_ + 1)] = acc
    return out


def fft2(G, sign: int):
    """Unnormalised 2D DFT with exp(sign 2 pi i (k_v q_v + k_u q_u) / N)."""
    a = fft_last_axis(G, sign)            # along u (last axis)
    a = fft_last_axis(np.swapaxes(a, -1, -2), sign)   # along v
    return np.swapaxes(a, -1, -2).copy()


def dft_matrix(n: int, sign: int):
    q = np.arange(n)
    return _root(np.outer(q, q) % n, n, sign)


def dft2_matrix(G, sign: int):
    """The same 2D DFT as a separable matrix product F G F^T (second form)."""
    ny, nx = G.shape[-2], G.shape[-1]
    Fy = dft_matrix(ny, sign)
    Fx = dft_matrix(nx, sign)
    return Fy @ np.asarray(G, dtype=np.complex128) @ Fx.T


# --------------------------------------------------------------------------
# Image formation (Sec. 5.2.2: real part and FFT shift)
# --------------------------------------------------------------------------
def shift_real_cut(R, W, out_n: int, norm: int):
    """Real part, fftshift (phase centre to [N/2][N/2]), 1/W, central cutout."""
    n_ = R.shape[-1]
    img = np.real(np.roll(R, (n_ // 2, n_ // 2), axis=(-2, -1)))
    if norm == NORM_WEIGHTS:
        img = img / W if W > 0 else np.zeros_like(img)
    a = n_ // 2 - out_n // 2
    return img[..., a:a + out_n, a:a + out_n].copy()


def image_one(vis, u_m, v_m, freq_hz, grid_n, pixscale, out_n, weighting,
              norm, flagged=None, gains=None, ant1=None, ant2=None,
              fft="recursive"):
    """Dirty image of one (timestep, channel): the whole path for one image.

    Returns a dict with the float64 image [M][M], the grid sums S, counts n,
    weight sum W, kept mask and signed cell indices.
    """
    s = uv_scale(freq_hz, grid_n, pixscale)
    iu, iv, keep = cell_index(u_m, v_m, s, grid_n, flagged)
    vp = apply_gains(vis, gains, ant1, ant2)
    S, cnt = grid(vp, iu, iv, keep, grid_n)
    G, W = weight(S, cnt, weighting)
    R = fft2(G, +1) if fft == "recursive" else dft2_matrix(G, +1)
    img = shift_real_cut(R, W, out_n, norm)
    return dict(image=img, S=S, counts=cnt, W=W, keep=keep, iu=iu, iv=iv, s=s)


def image_batch(vis, uvw_m, freq_hz, grid_n, pixscale, out_n, weighting,
                norm, flags=None, gains=None, ant1=None, ant2=None,
                images=None):
    """Dirty images for a cube vis[T][C][B] (optionally a subset of images).

    ``images`` is an iterable of flat image indices i = t * C + c; default
    all. Returns float64 images [len][M][M] and W [len].
    """
    T, C, B = vis.shape
    idx = range(T * C) if images is None else list(images)
    out, ws = [], []
    for i in idx:
        t, c = divmod(int(i), C)
        r = image_one(vis[t, c], uvw_m[t, :, 0], uvw_m[t, :, 1], freq_hz[c],
                      grid_n, pixscale, out_n, weighting, norm,
                      None if flags is None else flags[t], gains, ant1, ant2)
        out.append(r["image"])
        ws.append(r["W"])
    return np.stack(out), np.asarray(ws)


# --------------------------------------------------------------------------
# Brute-force direct sum (a check of grid + FFT that uses neither)
# --------------------------------------------------------------------------
def direct_image(vis_prime, iu, iv, keep, grid_n, out_n, weighting, norm):
    """Image pixel by pixel as a direct sum over kept baselines.

    I[p_m][p_l] = sum_b w_b * 2 Re(V'_b exp(+2 pi i (i_u q_u + i_v q_v) / N))
    with q = p - N/2 and w_b = 1 (natural) or 1/n[k_b] (uniform), divided by
    W for norm=1. Identical to the gridded FFT image up to rounding.
    """
    n_ = grid_n
    k = np.flatnonzero(keep)
    vp = np.asarray(vis_prime, dtype=np.complex128)[k]
    bu, bv = iu[k], iv[k]
    # cell counts of the full (Hermitian) grid, by brute force
    cells = {}
    for a, b in zip(bu, bv):
        for key in ((b % n_, a % n_), ((-b) % n_, (-a) % n_)):
            cells[key] = cells.get(key, 0) + 1
    if weighting == NATURAL:
        wb = np.ones(len(k))
        W = float(2 * len(k))
    else:
        wb = np.array([1.0 / cells[(b % n_, a % n_)] for a, b in zip(bu, bv)])
        W = float(len(cells))
    a0 = n_ // 2 - out_n // 2
    img = np.zeros((out_n, out_n))
    for pm in range(out_n):
        qv = pm + a0 - n_ // 2
        for pl in range(out_n):
            qu = pl + a0 - n_ // 2
            e = np.mod(bu * qu + bv * qv, n_)
            img[pm, pl] = np.sum(wb * 2.0 * np.real(vp * _root(e, n_, +1)))
    if norm == NORM_WEIGHTS:
        img = img / W if W > 0 else np.zeros_like(img)
    return img


# --------------------------------------------------------------------------
# Adjoint (differentiation form): gradients of a real loss of the images
# --------------------------------------------------------------------------
def adjoint_one(image_grad, vis, u_m, v_m, freq_hz, grid_n, pixscale,
                weighting, norm, flagged=None, gains=None, ant1=None,
                ant2=None):
    """Gradient of sum(image * image_grad) w.r.t. V (and the gains).

    Complex gradients use the convention grad z = dL/dx + i dL/dy. Steps:
    zero-pad the M x M gradient into the N x N image, times 1/W (norm=1),
    undo the shift, forward DFT (exp(-2 pi i ...)), times the cell weight
    (1 or 1/n), gather gamma'_b = Ghat[k_b] + conj(Ghat[-k_b]) for kept b;
    grad V_b = conj(g1) g2 gamma'_b; grad g1 += gamma'_b g2 conj(V_b);
    grad g2 += conj(gamma'_b) g1 V_b. W and the counts depend only on the
    geometry and flags, never on V, so the map V -> image is linear.
    Returns (vis_grad [B] complex128, gain_grad [A] complex128 or None).
    """
    n_ = grid_n
    m_ = image_grad.shape[-1]
    s = uv_scale(freq_hz, grid_n, pixscale)
    iu, iv, keep = cell_index(u_m, v_m, s, grid_n, flagged)
    vp = apply_gains(vis, gains, ant1, ant2)
    S, cnt = grid(vp, iu, iv, keep, grid_n)
    _, W = weight(S, cnt, weighting)
    P = np.zeros((n_, n_))
    a = n_ // 2 - m_ // 2
    P[a:a + m_, a:a + m_] = image_grad
    if norm == NORM_WEIGHTS:
        P = P / W if W > 0 else np.zeros_like(P)
    P = np.roll(P, (-(n_ // 2), -(n_ // 2)), axis=(0, 1))
    Gh = fft2(P.astype(np.complex128), -1)
    if weighting == UNIFORM:
        Gh = np.where(cnt > 0, Gh / np.maximum(cnt, 1), 0)
    gp = np.zeros(len(keep), dtype=np.complex128)
    k = np.flatnonzero(keep)
    gp[k] = (Gh[np.mod(iv[k], n_), np.mod(iu[k], n_)]
             + np.conj(Gh[np.mod(-iv[k], n_), np.mod(-iu[k], n_)]))
    if gains is None:
        return gp, None
    g = np.asarray(gains).astype(np.complex128)
    g1 = g[np.asarray(ant1)]
    g2 = g[np.asarray(ant2)]
    v = np.asarray(vis).astype(np.complex128)
    vgrad = np.conj(g1) * g2 * gp
    ggrad = np.zeros(len(g), dtype=np.complex128)
    np.add.at(ggrad, np.asarray(ant1), gp * g2 * np.conj(v))
    np.add.at(ggrad, np.asarray(ant2), np.conj(gp) * g1 * v)
    return vgrad, ggrad


def adjoint_batch(image_grad, vis, uvw_m, freq_hz, grid_n, pixscale,
                  weighting, norm, flags=None, gains=None, ant1=None,
                  ant2=None):
    """Adjoint over a cube: image_grad [T*C][M][M] -> vis_grad [T][C][B], gain_grad [A]."""
    T, C, B = vis.shape
    vg = np.zeros((T, C, B), dtype=np.complex128)
    gg = None if gains is None else np.zeros(len(gains), dtype=np.complex128)
    for t in range(T):
        for c in range(C):
            v_, g_ = adjoint_one(image_grad[t * C + c], vis[t, c],
                                 uvw_m[t, :, 0], uvw_m[t, :, 1], freq_hz[c],
                                 grid_n, pixscale, weighting, norm,
                                 None if flags is None else flags[t],
                                 gains, ant1, ant2)
            vg[t, c] = v_
            if gg is not None:
                gg += g_
    return vg, gg


def fft_flops_estimate(n_px: int) -> float:
    """N^2 log2(N^2): the operation-count model of a 2D FFT (Sec. 4.4.3 table)."""
    return float(n_px) ** 2 * math.log2(float(n_px) ** 2)
