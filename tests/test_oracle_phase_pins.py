"""Pins of the phase-rotation oracle.

* rotating to zenith (0, 0) changes nothing;
* a source exactly at the new centre, with the w term, becomes a constant
  visibility, so its image peaks at the centre with its flux;
* for a coplanar array (w = 0) a source at (l1, m1) moves to the pixel of
  (l1 - l0, m1 - m0) (point-source placement of the imaging oracle);
* the delay is the dot product of the baseline with s0 - z (a brute-force
  check of the n0 - 1 term);
* cable correction: equal lengths change nothing; visibilities correlated
  from cable-delayed voltages of a zenith source become constant and image
  at the centre with its flux; lengths that mimic a plane wave from (l0, m0)
  give exactly the geometric rotation to (l0, m0) on a coplanar array.
* re-projection: the frame is a proper rotation that takes zenith to s0 and
  leaves the axis z x s0 fixed (which fixes it uniquely), is the identity at
  zenith, preserves baseline lengths and gives w' = b . s0; a source placed at
  tangent-plane offsets (l', m') from a centre far from zenith images at that
  pixel with its flux, where the zenith-plane image would put it elsewhere;
  the re-projected imaging keeps its exact adjoint.
"""
import numpy as np

import oracle
from oracle import phase_rotation as pr


def _array(seed, nb=300, w_scale=0.0):
    rng = np.random.default_rng(seed)
    uvw = np.zeros((nb, 3))
    uvw[:, 0] = rng.uniform(-12, 12, nb)
    uvw[:, 1] = rng.uniform(-12, 12, nb)
    uvw[:, 2] = rng.uniform(-1, 1, nb) * w_scale
    return uvw


def test_zenith_is_identity():
    uvw = _array(1, w_scale=5.0)
    v = np.exp(1j * np.linspace(0, 3, len(uvw)))
    assert np.array_equal(pr.rotate(v, uvw, 1.5e8, 0.0, 0.0), v.astype(np.complex128))


def test_source_at_new_centre_becomes_constant():
    uvw = _array(2, w_scale=8.0)
    l0, m0 = 0.21, -0.13
    n0 = np.sqrt(1 - l0 ** 2 - m0 ** 2)
    freq = 1.7e8
    lam = oracle.C_LIGHT / freq
    v = 3.0 * np.exp(-2j * np.pi * (uvw[:, 0] * l0 + uvw[:, 1] * m0 + uvw[:, 2] * (n0 - 1)) / lam)
    r = pr.rotate(v, uvw, freq, l0, m0)
    assert np.allclose(r, 3.0, rtol=0, atol=1e-9)
    n = 64
    img = oracle.image_one(r, uvw[:, 0], uvw[:, 1], freq, n, lam / (3 * 24.0) / lam, n, oracle.NATURAL,
                           oracle.NORM_WEIGHTS)["image"]
    assert np.unravel_index(np.argmax(img), img.shape) == (n // 2, n // 2)
    assert abs(img[n // 2, n // 2] - 3.0) <= 1e-9


def test_coplanar_shift_moves_source_by_the_rotation():
    uvw = _array(3)
    freq = oracle.C_LIGHT                      # lambda = 1 m: u in wavelengths = metres
    n, pix = 64, 1.0 / (3 * 24.0)
    l1, m1 = 12 * pix, -5 * pix                # source 12 pixels right, 5 down of zenith
    l0, m0 = 4 * pix, 3 * pix                  # new centre
    v = np.exp(-2j * np.pi * (uvw[:, 0] * l1 + uvw[:, 1] * m1))
    r = pr.rotate(v, uvw, freq, l0, m0)
    img = oracle.image_one(r, uvw[:, 0], uvw[:, 1], freq, n, pix, n, oracle.NATURAL,
                           oracle.NORM_WEIGHTS)["image"]
    assert np.unravel_index(np.argmax(img), img.shape) == (n // 2 - 8, n // 2 + 8)


def test_delay_is_baseline_dot_direction_change():
    uvw = _array(4, w_scale=3.0)
    l0, m0 = -0.3, 0.4
    s0 = np.array([l0, m0, np.sqrt(1 - l0 ** 2 - m0 ** 2)])
    z = np.array([0.0, 0.0, 1.0])
    for b in range(0, len(uvw), 37):
        ref = sum(uvw[b, k] * (s0[k] - z[k]) for k in range(3))
        assert abs(pr.geometric_delay(uvw[b], l0, m0) - ref) <= 1e-12


# ------------------------------------------------------------ cable correction
def _antennas(seed, na=24, span=15.0):
    rng = np.random.default_rng(seed)
    xy = rng.uniform(-span, span, size=(na, 2))
    a1, a2 = np.triu_indices(na, k=1)
    uvw = np.zeros((len(a1), 3))
    uvw[:, :2] = xy[a2] - xy[a1]                   # baseline (ant1, ant2): position of ant2 - ant1
    return xy, a1.astype(np.int32), a2.astype(np.int32), uvw


def test_equal_cable_lengths_change_nothing():
    xy, a1, a2, uvw = _antennas(5)
    v = np.exp(1j * np.linspace(0, 2, len(a1)))
    cab = np.full(len(xy), 123.25)
    assert np.array_equal(pr.rotate(v, uvw, 1.6e8, 0.0, 0.0, cab, a1, a2), v.astype(np.complex128))


def test_cable_delayed_voltages_are_corrected():
    # a zenith plane wave seen through cables of different electrical length:
    # antenna a's voltage is the common signal delayed by l_a / c. The
    # correlated products x_i conj(x_j) differ from baseline to baseline until
    # corrected; corrected, all equal |s|^2 and the image of the zenith source
    # peaks at the centre with its flux.
    xy, a1, a2, uvw = _antennas(6)
    rng = np.random.default_rng(7)
    cab = rng.uniform(0.0, 300.0, len(xy))
    freq = 1.55e8
    s = 2.0 * np.exp(0.4j)
    x = s * np.exp(-2j * np.pi * freq * cab / oracle.C_LIGHT)
    vis = x[a1] * np.conj(x[a2])
    assert np.ptp(np.angle(vis)) > 1.0
    r = pr.rotate(vis, uvw, freq, 0.0, 0.0, cab, a1, a2)
    assert np.allclose(r, abs(s) ** 2, rtol=0, atol=1e-9)
    n = 64
    img = pr.image_batch_rotated(vis[None, None], uvw[None], np.array([freq]), n, 1.0 / (3 * 60.0), n, 0, 1,
                                 0.0, 0.0, ant1=a1, ant2=a2, cable_m=cab)[0][0]
    assert np.unravel_index(np.argmax(img), img.shape) == (n // 2, n // 2)
    assert abs(img[n // 2, n // 2] - abs(s) ** 2) <= 1e-9


def test_cable_lengths_of_a_tilted_plane_equal_the_geometric_rotation():
    # electrical lengths l_a = -(x_a l0 + y_a m0) delay each antenna as a plane
    # wave from (l0, m0) would; on a coplanar array the cable correction then
    # equals the geometric rotation to (l0, m0), term by term
    xy, a1, a2, uvw = _antennas(8)
    l0, m0 = 0.17, -0.09
    cab = -(xy[:, 0] * l0 + xy[:, 1] * m0)
    v = np.exp(1j * np.linspace(0, 5, len(a1)))
    freq = 1.9e8
    by_cable = pr.rotate(v, uvw, freq, 0.0, 0.0, cab, a1, a2)
    by_geometry = pr.rotate(v, uvw, freq, l0, m0)
    assert np.allclose(by_cable, by_geometry, rtol=0, atol=1e-12)


def _rot_case(seed=31, n=16, nb=36, n_ant=9):
    rng = np.random.default_rng(seed)
    uvw = np.zeros((1, nb, 3))
    uvw[0, :, 0] = rng.uniform(-6, 6, nb)
    uvw[0, :, 1] = rng.uniform(-6, 6, nb)
    uvw[0, :, 2] = rng.uniform(-2, 2, nb)
    a1 = rng.integers(0, n_ant, nb)
    a2 = (a1 + 1 + rng.integers(0, n_ant - 1, nb)) % n_ant
    vis = (rng.normal(size=(1, 1, nb)) + 1j * rng.normal(size=(1, 1, nb)))
    g = 1 + 0.05 * rng.normal(size=n_ant) + 0.05j * rng.normal(size=n_ant)
    cab = rng.uniform(0, 40, n_ant)
    return uvw, vis, a1, a2, g, cab, np.array([oracle.C_LIGHT]), 1.0 / n


def test_rotated_adjoint_dot_product():
    # gains off: the rotated image is linear in V, so <I(V), Ibar> = sum Re(conj(grad) V)
    uvw, vis, a1, a2, g, cab, freq, dx = _rot_case()
    rng = np.random.default_rng(4)
    ibar = rng.normal(size=(1, 12, 12))
    img, _ = pr.image_batch_rotated(vis, uvw, freq, 16, dx, 12, 0, 1, 0.2, -0.1, cable_m=cab, ant1=a1,
                                    ant2=a2)
    vg, _ = pr.adjoint_batch_rotated(ibar, vis, uvw, freq, 16, dx, 0, 1, 0.2, -0.1, cable_m=cab,
                                     ant1=a1, ant2=a2)
    lhs = np.sum(img * ibar)
    rhs = np.sum(vg.real * vis.real + vg.imag * vis.imag)
    assert np.isclose(lhs, rhs, rtol=1e-12, atol=1e-12)


def test_rotated_adjoint_finite_differences():
    # FP64 central differences of ||I - T||^2 through rotation, cable lengths and gains
    uvw, vis, a1, a2, g, cab, freq, dx = _rot_case(seed=32)
    rng = np.random.default_rng(6)
    target = rng.normal(size=(1, 14, 14))
    kw = dict(cable_m=cab, ant1=a1, ant2=a2)

    def loss(vv, gg):
        img, _ = pr.image_batch_rotated(vv, uvw, freq, 16, dx, 14, 1, 1, 0.15, 0.1, gains=gg, **kw)
        return float(np.sum((img - target) ** 2))

    img, _ = pr.image_batch_rotated(vis, uvw, freq, 16, dx, 14, 1, 1, 0.15, 0.1, gains=g, **kw)
    vg, gg = pr.adjoint_batch_rotated(2 * (img - target), vis, uvw, freq, 16, dx, 1, 1, 0.15, 0.1,
                                      gains=g, **kw)

    def fd(f, x, idx, part):
        h = 1e-6 * max(1.0, abs(x[idx]))
        xp = x.copy(); xp[idx] += h if part == 0 else 1j * h
        xm = x.copy(); xm[idx] -= h if part == 0 else 1j * h
        return (f(xp) - f(xm)) / (2 * h)

    for k in range(len(g)):
        for part in (0, 1):
            num = fd(lambda q: loss(vis, q), g, k, part)
            ana = (gg[k].real, gg[k].imag)[part]
            assert abs(num - ana) <= 1e-6 * max(1.0, abs(ana))
    for b in range(0, vis.shape[2], 2):
        for part in (0, 1):
            num = fd(lambda q: loss(q, g), vis, (0, 0, b), part)
            ana = (vg[0, 0, b].real, vg[0, 0, b].imag)[part]
            assert abs(num - ana) <= 1e-6 * max(1.0, abs(ana))


# ------------------------------------------------------------ re-projection
def test_reprojection_frame_is_the_smallest_rotation_to_the_centre():
    for l0, m0 in [(0.3, -0.2), (-0.55, 0.41), (0.0, 0.7), (1e-3, 0.0)]:
        R = pr.reprojection_matrix(l0, m0)
        s0 = np.array([l0, m0, np.sqrt(1 - l0 ** 2 - m0 ** 2)])
        assert np.allclose(R.T @ R, np.eye(3), atol=1e-14)
        assert abs(np.linalg.det(R) - 1.0) <= 1e-14
        assert np.allclose(R @ np.array([0.0, 0.0, 1.0]), s0, atol=1e-14)
        k = np.cross([0.0, 0.0, 1.0], s0)
        k /= np.linalg.norm(k)
        assert np.allclose(R @ k, k, atol=1e-14)
    assert np.array_equal(pr.reprojection_matrix(0.0, 0.0), np.eye(3))
    uvw = _array(9, w_scale=4.0)
    up = pr.plane_uvw(uvw, 0.3, -0.2, True)
    assert np.allclose(np.linalg.norm(up, axis=1), np.linalg.norm(uvw, axis=1), rtol=1e-14)
    s0 = np.array([0.3, -0.2, np.sqrt(1 - 0.13)])
    assert np.allclose(up[:, 2], uvw @ s0, atol=1e-12)
    assert np.array_equal(pr.plane_uvw(uvw, 0.3, -0.2, False), uvw)


def test_reprojected_source_images_at_its_tangent_plane_offset():
    # baselines in the plane perpendicular to s0 (w' = 0, but w != 0 in the
    # zenith frame), so the image on the new tangent plane has no w term: a
    # source at an exact pixel of that plane peaks there (nearest-cell
    # gridding lowers an off-centre peak, so only its place is checked)
    freq = oracle.C_LIGHT                      # lambda = 1 m
    n, pix = 64, 1.0 / (3 * 24.0)
    l0, m0 = 0.45, 0.3                         # centre well away from zenith (n0 = 0.84)
    R = pr.reprojection_matrix(l0, m0)
    rng = np.random.default_rng(10)
    xy = rng.uniform(-12, 12, size=(400, 2))
    uvw = xy[:, :1] * R[:, 0] + xy[:, 1:] * R[:, 1]
    assert np.ptp(uvw[:, 2]) > 5.0
    lp, mp = 18 * pix, -12 * pix               # 18 pixels right, 12 down on the new tangent plane
    s = R @ np.array([lp, mp, np.sqrt(1 - lp ** 2 - mp ** 2)])
    v = 2.5 * np.exp(-2j * np.pi * (uvw @ (s - np.array([0.0, 0.0, 1.0]))))
    kw = dict(vis=v[None, None], uvw_m=uvw[None], freq_hz=np.array([freq]), grid_n=n, pixscale=pix,
              out_n=n, weighting=0, norm=1, l0=l0, m0=m0)
    img = pr.image_batch_rotated(reproject=True, **kw)[0][0]
    assert np.unravel_index(np.argmax(img), img.shape) == (n // 2 - 12, n // 2 + 18)
    flat = pr.image_batch_rotated(reproject=False, **kw)[0][0]
    assert np.unravel_index(np.argmax(flat), flat.shape) != (n // 2 - 12, n // 2 + 18)


def test_reprojection_at_zenith_changes_nothing():
    uvw, vis, a1, a2, g, cab, freq, dx = _rot_case(seed=33)
    a = pr.image_batch_rotated(vis, uvw, freq, 16, dx, 12, 1, 1, 0.0, 0.0, gains=g, ant1=a1, ant2=a2,
                               cable_m=cab, reproject=True)
    b = pr.image_batch_rotated(vis, uvw, freq, 16, dx, 12, 1, 1, 0.0, 0.0, gains=g, ant1=a1, ant2=a2,
                               cable_m=cab)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_reprojected_adjoint_dot_product():
    uvw, vis, a1, a2, g, cab, freq, dx = _rot_case(seed=34)
    rng = np.random.default_rng(5)
    ibar = rng.normal(size=(1, 12, 12))
    kw = dict(cable_m=cab, ant1=a1, ant2=a2, reproject=True)
    img, _ = pr.image_batch_rotated(vis, uvw, freq, 16, dx, 12, 0, 1, 0.35, -0.25, **kw)
    vg, _ = pr.adjoint_batch_rotated(ibar, vis, uvw, freq, 16, dx, 0, 1, 0.35, -0.25, **kw)
    lhs = np.sum(img * ibar)
    rhs = np.sum(vg.real * vis.real + vg.imag * vis.imag)
    assert np.isclose(lhs, rhs, rtol=1e-12, atol=1e-12)
