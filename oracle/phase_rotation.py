"""FP64 oracle of the geometric phase rotation applied at visibility load.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: only the test suite,
the package smoke check and the benchmark's CPU-baseline leg may import it.

Sec. 4.2 (iii): correlation yields visibilities phase-centred at zenith;
for an instrument with a smaller field of view a geometric phase factor
rotates them to the pointing centre before imaging. Readings used here:

* the new phase centre is given by its direction cosines (l0, m0) relative
  to zenith, n0 = sqrt(1 - l0^2 - m0^2);
* a source in direction (l, m, n) contributes exp(-2 pi i (u l + v m +
  w (n - 1)) / lambda) to a zenith-centred visibility (the sign of Eq. 5,
  with the w term kept), so the rotation multiplies every visibility by
  exp(+2 pi i (u l0 + v m0 + w (n0 - 1)) nu / c), which turns a source at
  the new centre into a constant;
* (u, v, w) are not re-projected: the image stays on the zenith tangent
  plane, shifted so that the new centre is at its middle;
* the factor multiplies V' after the gains (both are per-visibility
  scalars, so their order does not matter).

Re-projection (an option; Sec. 4.2 (iii) only names the rotation): with it
the image lies on the tangent plane at the new centre instead of the zenith
one. Reading used: the new frame's axes are the zenith frame's axes (east,
north, up) carried by the smallest rotation that takes zenith to s0 (about
the axis z x s0), so e_w' = s0 and the frame reduces to the zenith frame at
zenith; each baseline is gridded at u' = b . e_u', v' = b . e_v' (metres).
The phase factor is unchanged: b . (s0 - z) is the same path difference in
any frame, and after it a source in direction s carries
exp(-2 pi i (u' l' + v' m' + w' (n' - 1)) / lambda) with (l', m', n') its
direction cosines in the new frame, so its image sits at (l', m').

Sec. 4.2 (i), the cable correction, reads as follows here: antenna a's
signal path is longer by an electrical length l_a (metres of free-space
propagation), which delays its voltage by l_a / c and multiplies its
component at frequency nu by exp(-2 pi i nu l_a / c); the visibility of
baseline (ant1, ant2) = x_ant1 conj(x_ant2) then carries
exp(-2 pi i nu (l_ant1 - l_ant2) / c), and the correction multiplies it by
exp(+2 pi i nu (l_ant1 - l_ant2) / c). It is the same factor as the
geometric rotation with the path difference l_ant1 - l_ant2, so the two add
into one delay per baseline.
"""
from __future__ import annotations

import numpy as np

from .blink_oracle import C_LIGHT, image_one


def reprojection_matrix(l0: float, m0: float):
    """3 x 3 matrix whose columns are the new frame's axes e_u', e_v', e_w' = s0
    in zenith-frame components (the smallest rotation taking z to s0, applied
    to the zenith axes); uvw' = uvw @ R."""
    from scipy.spatial.transform import Rotation

    s0 = np.array([l0, m0, np.sqrt(1.0 - l0 * l0 - m0 * m0)])
    axis = np.cross([0.0, 0.0, 1.0], s0)
    sin = np.linalg.norm(axis)
    if sin == 0.0:
        return np.eye(3)
    angle = np.arctan2(sin, s0[2])
    return Rotation.from_rotvec(axis / sin * angle).as_matrix()


def plane_uvw(uvw_m, l0: float, m0: float, reproject: bool):
    """Baseline coordinates the imager grids: uvw itself, or re-projected."""
    uvw = np.asarray(uvw_m, dtype=np.float64)
    return uvw @ reprojection_matrix(l0, m0) if reproject else uvw


def geometric_delay(uvw_m, l0: float, m0: float):
    """u l0 + v m0 + w (n0 - 1) in metres for uvw [..., 3]."""
    uvw = np.asarray(uvw_m, dtype=np.float64)
    n0 = np.sqrt(1.0 - l0 * l0 - m0 * m0)
    return uvw[..., 0] * l0 + uvw[..., 1] * m0 + uvw[..., 2] * (n0 - 1.0)


def cable_delay(cable_m, ant1, ant2):
    """l_ant1 - l_ant2 in metres per baseline."""
    cab = np.asarray(cable_m, dtype=np.float64)
    return cab[np.asarray(ant1)] - cab[np.asarray(ant2)]


def rotate(vis, uvw_m, freq_hz: float, l0: float, m0: float, cable_m=None, ant1=None, ant2=None):
    """V exp(+2 pi i d nu / c) for one channel (vis and uvw over the same baselines),
    d the geometric delay plus, with cable lengths, l_ant1 - l_ant2."""
    d = geometric_delay(uvw_m, l0, m0)
    if cable_m is not None:
        d = d + cable_delay(cable_m, ant1, ant2)
    return np.asarray(vis, dtype=np.complex128) * np.exp(2j * np.pi * d * (np.float64(freq_hz) / C_LIGHT))


def image_batch_rotated(vis, uvw_m, freq_hz, grid_n, pixscale, out_n, weighting, norm, l0, m0,
                        flags=None, gains=None, ant1=None, ant2=None, images=None, cable_m=None,
                        reproject=False):
    """Images [len][M][M] and W [len] with the phase centre rotated to (l0, m0)
    and, with cable lengths, the cable correction applied; with ``reproject``
    on the tangent plane at (l0, m0)."""
    T, C, B = vis.shape
    idx = range(T * C) if images is None else list(images)
    out, ws = [], []
    for i in idx:
        t, c = divmod(int(i), C)
        v = rotate(vis[t, c], uvw_m[t], freq_hz[c], l0, m0, cable_m, ant1, ant2)
        uv = plane_uvw(uvw_m[t], l0, m0, reproject)
        r = image_one(v, uv[:, 0], uv[:, 1], freq_hz[c], grid_n, pixscale, out_n, weighting,
                      norm, None if flags is None else flags[t], gains, ant1, ant2)
        out.append(r["image"])
        ws.append(r["W"])
    return np.stack(out), np.asarray(ws)


def adjoint_batch_rotated(image_grad, vis, uvw_m, freq_hz, grid_n, pixscale, weighting, norm, l0, m0,
                          flags=None, gains=None, ant1=None, ant2=None, cable_m=None, reproject=False):
    """Gradients (vis_grad [T][C][B], gain_grad [A] or None) of sum(images *
    image_grad) through the rotated imaging of image_batch_rotated.

    Per image the imager sees U = p V with p = exp(+2 pi i d nu / c) (|p| = 1,
    fixed by the geometry), then applies the gains as for any input. So the
    gain gradient is the plain adjoint's with U in place of V, and the chain
    rule through U = p V (convention grad z = dL/dx + i dL/dy) multiplies the
    gradient with respect to U by conj(p).
    """
    from .blink_oracle import adjoint_one

    T, C, B = vis.shape
    vg = np.zeros((T, C, B), dtype=np.complex128)
    gg = None if gains is None else np.zeros(len(gains), dtype=np.complex128)
    for t in range(T):
        for c in range(C):
            d = geometric_delay(uvw_m[t], l0, m0)
            if cable_m is not None:
                d = d + cable_delay(cable_m, ant1, ant2)
            p = np.exp(2j * np.pi * d * (np.float64(freq_hz[c]) / C_LIGHT))
            u = np.asarray(vis[t, c], dtype=np.complex128) * p
            uv = plane_uvw(uvw_m[t], l0, m0, reproject)
            gu, g_ = adjoint_one(image_grad[t * C + c], u, uv[:, 0], uv[:, 1], freq_hz[c],
                                 grid_n, pixscale, weighting, norm, None if flags is None else flags[t],
                                 gains, ant1, ant2)
            vg[t, c] = np.conj(p) * gu
            if gg is not None:
                gg += g_
    return vg, gg
