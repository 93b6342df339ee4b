"""Pins of the X-engine oracle.

* a hand-worked 3-antenna, 2-sample case (tests/golden/correlator_hand.json);
* the full matrix is Hermitian with real, non-negative autocorrelations equal
  to the summed power; the pair index enumerates numpy's upper triangle;
* a brute-force loop over samples on a tiny input;
* a plane wave from direction (l, m) seen by every antenna, correlated and
  imaged with the (separately pinned) imaging oracle, peaks at (l, m): the
  correlator's conjugation and the imager's sign convention agree.
"""
import json
import os

import numpy as np

import oracle
from oracle import correlator as xc

HERE = os.path.dirname(os.path.abspath(__file__))


def test_hand_worked():
    g = json.load(open(os.path.join(HERE, "golden", "correlator_hand.json")))
    volt = np.array(g["volt"], dtype=np.int8)[None]            # [T=1][C=1][A=3][S=2][2]
    vis, autos = xc.correlate(volt)
    exp = np.array([complex(a, b) for a, b in g["vis"]])
    assert np.array_equal(vis[0, 0], exp)
    assert np.array_equal(autos[0, 0], np.array(g["autos"], dtype=np.float64))


def test_hermitian_autos_and_pair_order():
    rng = np.random.default_rng(4)
    volt = rng.integers(-128, 128, size=(2, 3, 7, 48, 2)).astype(np.int8)
    x = volt[..., 0].astype(np.float64) + 1j * volt[..., 1]
    V = xc.correlation_matrix(x)
    assert np.array_equal(V, np.conj(np.swapaxes(V, -1, -2)))
    vis, autos = xc.correlate(volt)
    assert np.array_equal(autos, (np.abs(x) ** 2).sum(axis=-1))
    assert np.all(autos >= 0)
    i, j = np.triu_indices(7, k=1)
    assert np.array_equal(xc.pair_index(i, j, 7), np.arange(len(i)))


def test_brute_force_loop():
    rng = np.random.default_rng(9)
    volt = rng.integers(-128, 128, size=(1, 1, 4, 5, 2)).astype(np.int8)
    vis, _ = xc.correlate(volt)
    b = 0
    for i in range(4):
        for j in range(i + 1, 4):
            re = im = 0
            for s in range(5):
                ar, ai = int(volt[0, 0, i, s, 0]), int(volt[0, 0, i, s, 1])
                br, bi = int(volt[0, 0, j, s, 0]), int(volt[0, 0, j, s, 1])
                re += ar * br + ai * bi          # x_i conj(x_j)
                im += ai * br - ar * bi
            assert vis[0, 0, b] == complex(re, im)
            b += 1


def test_plane_wave_images_at_its_direction():
    rng = np.random.default_rng(12)
    A, S, n = 24, 400, 64
    xy = rng.uniform(-10, 10, size=(A, 2))            # metres; one channel at lambda = 1 m
    freq = oracle.C_LIGHT
    pix = 1.0 / (3 * 40.0)                             # dx = 1 / (3 u_max), u_max ~ 40 wavelengths
    ql, qm = 9, -6                                     # source offset in pixels from the centre
    l, m = ql * pix, qm * pix
    sig = rng.normal(size=S) + 1j * rng.normal(size=S)
    x = sig[None, :] * np.exp(2j * np.pi * (xy[:, 0] * l + xy[:, 1] * m))[:, None]
    volt = np.stack([np.round(20 * x.real), np.round(20 * x.imag)], axis=-1).astype(np.int8)[None, None]
    vis, _ = xc.correlate(volt)
    a1, a2 = np.triu_indices(A, k=1)
    d = xy[a2] - xy[a1]                                # the imaging inputs' baseline vector
    img = oracle.image_one(vis[0, 0], d[:, 0], d[:, 1], freq, n, pix, n, oracle.NATURAL,
                           oracle.NORM_WEIGHTS)["image"]
    assert np.unravel_index(np.argmax(img), img.shape) == (n // 2 + qm, n // 2 + ql)
