"""FP64 oracle of gridding with an anti-aliasing convolution kernel.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: the slow, obviously
correct reference that the HIP path is checked against. Only the test suite,
the package smoke check and the benchmark's CPU-baseline leg may import it.

Sec. 4.4.1 notes that with a limited field of view, sources outside it are
aliased into the image unless the gridded visibilities are convolved with a
gridding kernel, at N_kern times the gridding cost (the cost table of
Sec. 4.4.3), and the comparison of EDA2 all-sky images with MIRIAD and CASA
(Sec. 5) attributes 10-20% differences to the kernel those packages apply. The paper
names neither the kernel nor its correction; the readings used here are:

* Kernel: separable Kaiser-Bessel of support W cells and shape beta,
  C(d) = I0(beta sqrt(1 - (2 d / W)^2)) / I0(beta) for |d| <= W/2, else 0,
  where d is the distance in cells from the visibility's exact position to a
  cell centre. Default beta for a grid twice the size of the kept image
  (alpha = 2): beta = pi sqrt((W / alpha)^2 (alpha - 1/2)^2 - 0.8)
  (Beatty, Nishimura and Pauly 2005, IEEE TMI 24, 799).
* A visibility at the fractional cell position x = (u s_c, v s_c) adds
  C(i - x_u) C(j - x_v) V' to every cell (j, i) with |i - x_u| <= W/2 and
  |j - x_v| <= W/2, and the same weight times conj(V') to the mirror cell
  (-j, -i) (its conjugate sits at -x).
* A baseline is kept iff it is unflagged, finite and all its footprint cells
  satisfy |i| < N/2 and |j| < N/2 (so the grid stays exactly Hermitian).
* Natural weighting: G = S, W = the sum of every weight added (direct and
  mirror). ``norm=1`` divides by W.
* Uniform weighting (Sec. 4.4.2, every occupied uv cell counting equally),
  read for a gridding kernel as a weight per visibility: baseline b gets
  omega_b = 1 / n[k_b], n the number of kept entries (direct and mirror)
  whose nearest cell is b's nearest cell k_b = (rint(x_v), rint(x_u)); it is
  then gridded with the kernel as above with omega_b V' (and W sums
  omega_b times every kernel weight added). With a box kernel of width 1 this
  is exactly the nearest-cell uniform weighting (cell value = sum / count,
  W = number of occupied cells).
* Correction: the image pixel at offset (q_m, q_l) from the centre is divided
  by c(q_l / N) c(q_m / N), c the Fourier transform of the continuous kernel
  normalised to c(0) = 1. For the Kaiser-Bessel kernel it has the closed form
  c(xi) = [sinh(z) / z] / [sinh(beta) / beta], z = sqrt(beta^2 - (pi W xi)^2)
  (sin(|z|) / |z| once pi W |xi| > beta), Jackson et al. 1991, IEEE TMI 10, 473.
* Adjoint (differentiation through kernel gridding): the map V' -> image is
  linear (weights, W and the correction depend only on geometry and flags),
  so its adjoint divides the image gradient by the same correction, pads it,
  scales by 1/W, undoes the shift, applies the forward transform Gh, and
  degrids: gamma'_b = sum over b's footprint cells of w Gh[cell] plus the
  conjugate of the same sum over its mirror cells; the gains then follow as
  for nearest-cell gridding.
"""
from __future__ import annotations

import math

import numpy as np

from .blink_oracle import (NORM_WEIGHTS, apply_gains, fft2, uv_scale)

ALPHA = 2.0


def kb_default_beta(support: int) -> float:
    """beta = pi sqrt((W / alpha)^2 (alpha - 1/2)^2 - 0.8) with alpha = 2."""
    q = (support / ALPHA) ** 2 * (ALPHA - 0.5) ** 2 - 0.8
    if q <= 0:
        raise ValueError("support too small for the default shape")
    return math.pi * math.sqrt(q)


def kb(d, support: int, beta: float):
    """Kaiser-Bessel weight at distance d (cells); zero outside |d| <= W/2."""
    d = np.asarray(d, dtype=np.float64)
    t = 1.0 - (2.0 * d / support) ** 2
    inside = np.abs(d) <= support / 2.0
    arg = beta * np.sqrt(np.where(inside, np.maximum(t, 0.0), 0.0))
    return np.where(inside, np.i0(arg) / np.i0(beta), 0.0)


def kb_taper(xi, support: int, beta: float):
    """Fourier transform of the continuous kernel at xi cycles per cell, c(0) = 1."""
    xi = np.asarray(xi, dtype=np.float64)
    a = math.pi * support * xi
    z2 = beta * beta - a * a

    def sinhc(z):
        return np.where(z == 0, 1.0, np.sinh(z) / np.where(z == 0, 1.0, z))

    def sinc_(z):
        return np.where(z == 0, 1.0, np.sin(z) / np.where(z == 0, 1.0, z))

    zp = np.sqrt(np.maximum(z2, 0.0))
    zn = np.sqrt(np.maximum(-z2, 0.0))
    f = np.where(z2 >= 0, sinhc(zp), sinc_(zn))
    return f / float(sinhc(np.float64(beta)))


def footprint(x: float, support: int):
    """Integer cells i with |i - x| <= W/2."""
    h = support / 2.0
    return np.arange(math.ceil(x - h), math.floor(x + h) + 1, dtype=np.int64)


def conv_keep(xu, xv, support: int, grid_n: int, flagged=None):
    """Kept iff unflagged, finite and the whole footprint lies in |i|, |j| < N/2."""
    xu = np.asarray(xu, dtype=np.float64)
    xv = np.asarray(xv, dtype=np.float64)
    h = support / 2.0
    half = grid_n // 2
    fin = np.isfinite(xu) & np.isfinite(xv)
    xu0 = np.where(fin, xu, 0.0)
    xv0 = np.where(fin, xv, 0.0)
    keep = fin & (np.ceil(xu0 - h) > -half) & (np.floor(xu0 + h) < half) \
        & (np.ceil(xv0 - h) > -half) & (np.floor(xv0 + h) < half)
    if flagged is not None:
        keep &= ~np.asarray(flagged, dtype=bool)
    return keep


def uniform_weights(xu, xv, keep, grid_n: int):
    """omega_b = 1 / n[k_b] for kept b (0 otherwise): n counts the kept entries,
    each baseline once at its nearest cell and once (its conjugate) at the
    mirror cell."""
    n_ = grid_n
    k = np.flatnonzero(np.asarray(keep))
    iu = np.rint(np.asarray(xu, dtype=np.float64)[k]).astype(np.int64)
    iv = np.rint(np.asarray(xv, dtype=np.float64)[k]).astype(np.int64)
    n = np.zeros((n_, n_), dtype=np.int64)
    np.add.at(n, (np.mod(iv, n_), np.mod(iu, n_)), 1)
    np.add.at(n, (np.mod(-iv, n_), np.mod(-iu, n_)), 1)
    om = np.zeros(len(keep))
    om[k] = 1.0 / n[np.mod(iv, n_), np.mod(iu, n_)]
    return om


def grid_conv(vis_prime, xu, xv, keep, grid_n: int, support: int, beta: float, omega=None):
    """Convolutional gridding: returns (S, counts, W).

    S[j mod N][i mod N] collects w V' over each kept baseline's footprint and
    w conj(V') at the mirror cells; counts holds the number of contributions
    per cell and W the sum of all weights added. ``omega`` (uniform
    weighting) multiplies each baseline's weights.
    """
    n_ = grid_n
    S = np.zeros((n_, n_), dtype=np.complex128)
    cnt = np.zeros((n_, n_), dtype=np.int64)
    wsum = 0.0
    vp = np.asarray(vis_prime, dtype=np.complex128)
    for b in np.flatnonzero(np.asarray(keep)):
        iu = footprint(xu[b], support)
        iv = footprint(xv[b], support)
        w = np.outer(kb(iv - xv[b], support, beta), kb(iu - xu[b], support, beta))   # [j][i]
        if omega is not None:
            w = w * omega[b]
        rows, cols = np.mod(iv, n_), np.mod(iu, n_)
        S[np.ix_(rows, cols)] += w * vp[b]
        cnt[np.ix_(rows, cols)] += 1
        S[np.ix_(np.mod(-iv, n_), np.mod(-iu, n_))] += w * np.conj(vp[b])
        cnt[np.ix_(np.mod(-iv, n_), np.mod(-iu, n_))] += 1
        wsum += 2.0 * float(w.sum())
    return S, cnt, wsum


def correct_taper(img, grid_n: int, support: int, beta: float):
    """Divide an M x M centred image by c(q_m / N) c(q_l / N)."""
    m = img.shape[-1]
    q = (np.arange(m) - m // 2) / grid_n
    c = kb_taper(q, support, beta)
    return img / np.outer(c, c)


def image_one_conv(vis, u_m, v_m, freq_hz, grid_n, pixscale, out_n, norm, support, beta=None,
                   flagged=None, gains=None, ant1=None, ant2=None, correct=True, weighting=0):
    """Dirty image of one (timestep, channel) with Kaiser-Bessel gridding
    (weighting 0 natural, 1 uniform)."""
    beta = kb_default_beta(support) if beta is None or beta < 0 else float(beta)
    s = uv_scale(freq_hz, grid_n, pixscale)
    xu = np.asarray(u_m, dtype=np.float64) * np.float64(s)
    xv = np.asarray(v_m, dtype=np.float64) * np.float64(s)
    keep = conv_keep(xu, xv, support, grid_n, flagged)
    vp = apply_gains(vis, gains, ant1, ant2)
    om = uniform_weights(xu, xv, keep, grid_n) if weighting == 1 else None
    S, cnt, W = grid_conv(vp, xu, xv, keep, grid_n, support, beta, om)
    R = fft2(S, +1)
    n_ = grid_n
    img = np.real(np.roll(R, (n_ // 2, n_ // 2), axis=(-2, -1)))
    if norm == NORM_WEIGHTS:
        img = img / W if W > 0 else np.zeros_like(img)
    a = n_ // 2 - out_n // 2
    img = img[a:a + out_n, a:a + out_n]
    if correct:
        img = correct_taper(img, grid_n, support, beta)
    return dict(image=img, S=S, counts=cnt, W=W, keep=keep, xu=xu, xv=xv, beta=beta)


def image_batch_conv(vis, uvw_m, freq_hz, grid_n, pixscale, out_n, norm, support, beta=None,
                     flags=None, gains=None, ant1=None, ant2=None, images=None, weighting=0):
    """Images [len][M][M] and W [len] for flat indices t * C + c (default all)."""
    T, C, B = vis.shape
    idx = range(T * C) if images is None else list(images)
    out, ws = [], []
    for i in idx:
        t, c = divmod(int(i), C)
        r = image_one_conv(vis[t, c], uvw_m[t, :, 0], uvw_m[t, :, 1], freq_hz[c], grid_n, pixscale,
                           out_n, norm, support, beta, None if flags is None else flags[t],
                           gains, ant1, ant2, weighting=weighting)
        out.append(r["image"])
        ws.append(r["W"])
    return np.stack(out), np.asarray(ws)


def direct_fractional_image(vis_prime, xu, xv, keep, grid_n: int, out_n: int):
    """Ungridded dirty image at the pixel centres, normalised per kept entry.

    I[p_m][p_l] = sum_b 2 Re(V'_b exp(+2 pi i (x_u q_l + x_v q_m) / N)) / (2 n_kept)
    with q = p - M/2: the exact transform of the visibilities at their true
    positions, which kernel gridding plus correction approximates.
    """
    q = np.arange(out_n) - out_n // 2
    k = np.flatnonzero(np.asarray(keep))
    vp = np.asarray(vis_prime, dtype=np.complex128)[k]
    eu = np.exp(2j * np.pi * np.outer(xu[k], q) / grid_n)      # [b][l]
    ev = np.exp(2j * np.pi * np.outer(xv[k], q) / grid_n)      # [b][m]
    img = 2.0 * np.real(np.einsum("b,bm,bl->ml", vp, ev, eu))
    return img / (2.0 * len(k)) if len(k) else img


def adjoint_one_conv(image_grad, vis, u_m, v_m, freq_hz, grid_n, pixscale, norm, support, beta=None,
                     flagged=None, gains=None, ant1=None, ant2=None, weighting=0, correct=True):
    """Gradient of sum(image * image_grad) through image_one_conv w.r.t. V (and
    the gains), convention grad z = dL/dx + i dL/dy: (vis_grad [B], gain_grad
    [A] or None)."""
    beta = kb_default_beta(support) if beta is None or beta < 0 else float(beta)
    n_ = grid_n
    m_ = image_grad.shape[-1]
    s = uv_scale(freq_hz, grid_n, pixscale)
    xu = np.asarray(u_m, dtype=np.float64) * np.float64(s)
    xv = np.asarray(v_m, dtype=np.float64) * np.float64(s)
    keep = conv_keep(xu, xv, support, grid_n, flagged)
    vp = apply_gains(vis, gains, ant1, ant2)
    om = uniform_weights(xu, xv, keep, grid_n) if weighting == 1 else None
    _, _, W = grid_conv(vp, xu, xv, keep, grid_n, support, beta, om)
    g = np.asarray(image_grad, dtype=np.float64)
    if correct:
        g = correct_taper(g, grid_n, support, beta)          # a diagonal scaling is its own adjoint
    P = np.zeros((n_, n_))
    a = n_ // 2 - m_ // 2
    P[a:a + m_, a:a + m_] = g
    if norm == NORM_WEIGHTS:
        P = P / W if W > 0 else np.zeros_like(P)
    P = np.roll(P, (-(n_ // 2), -(n_ // 2)), axis=(0, 1))
    Gh = fft2(P.astype(np.complex128), -1)
    gp = np.zeros(len(keep), dtype=np.complex128)
    for b in np.flatnonzero(np.asarray(keep)):
        iu = footprint(xu[b], support)
        iv = footprint(xv[b], support)
        w = np.outer(kb(iv - xv[b], support, beta), kb(iu - xu[b], support, beta))   # [j][i]
        if om is not None:
            w = w * om[b]
        direct = np.sum(w * Gh[np.ix_(np.mod(iv, n_), np.mod(iu, n_))])
        mirror = np.sum(w * Gh[np.ix_(np.mod(-iv, n_), np.mod(-iu, n_))])
        gp[b] = direct + np.conj(mirror)
    if gains is None:
        return gp, None
    gg_ = np.asarray(gains).astype(np.complex128)
    g1 = gg_[np.asarray(ant1)]
    g2 = gg_[np.asarray(ant2)]
    v = np.asarray(vis).astype(np.complex128)
    vgrad = np.conj(g1) * g2 * gp
    ggrad = np.zeros(len(gg_), dtype=np.complex128)
    np.add.at(ggrad, np.asarray(ant1), gp * g2 * np.conj(v))
    np.add.at(ggrad, np.asarray(ant2), np.conj(gp) * g1 * v)
    return vgrad, ggrad


def adjoint_batch_conv(image_grad, vis, uvw_m, freq_hz, grid_n, pixscale, norm, support, beta=None,
                       flags=None, gains=None, ant1=None, ant2=None, weighting=0):
    """Adjoint over a cube: image_grad [T*C][M][M] -> (vis_grad [T][C][B], gain_grad [A] or None)."""
    T, C, B = vis.shape
    vg = np.zeros((T, C, B), dtype=np.complex128)
    gg = None if gains is None else np.zeros(len(gains), dtype=np.complex128)
    for t in range(T):
        for c in range(C):
            v_, g_ = adjoint_one_conv(image_grad[t * C + c], vis[t, c], uvw_m[t, :, 0], uvw_m[t, :, 1],
                                      freq_hz[c], grid_n, pixscale, norm, support, beta,
                                      None if flags is None else flags[t], gains, ant1, ant2,
                                      weighting=weighting)
            vg[t, c] = v_
            if gg is not None:
                gg += g_
    return vg, gg
