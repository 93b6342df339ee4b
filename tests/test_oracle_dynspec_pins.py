"""Pins of the dynamic-spectra oracle against a hand-worked cube and closed forms.

* a 4 x 2 x (1 x 2) cube worked by hand (tests/golden/dynamic_spectra_hand.json);
* window 1 is the first difference (numpy.diff) with a zero first sample;
* a cube constant in time gives zero differences;
* a linear ramp a + b t gives b (k + 1) / 2 for a window of k preceding images;
* a model reference equal to the first image gives a zero first sample.
"""
import json
import os

import numpy as np

from oracle import dynamic_spectra as ds

HERE = os.path.dirname(os.path.abspath(__file__))


def test_hand_worked_cube():
    g = json.load(open(os.path.join(HERE, "golden", "dynamic_spectra_hand.json")))
    I = np.array(g["images"], dtype=np.float64)[:, :, None, :]      # [T][C][1][2]
    assert np.array_equal(ds.dynamic_spectra(I, ds.REF_NONE), np.array(g["none"]))
    assert np.array_equal(ds.dynamic_spectra(I, ds.REF_MEAN, 1), np.array(g["mean1"]))
    assert np.array_equal(ds.dynamic_spectra(I, ds.REF_MEAN, 2), np.array(g["mean2"]))
    R = np.array(g["model"]["ref"], dtype=np.float64)[:, None, :]
    assert np.array_equal(ds.dynamic_spectra(I, ds.REF_MODEL, ref_image=R), np.array(g["model"]["spectra"]))


def test_window_one_is_first_difference():
    rng = np.random.default_rng(1)
    I = rng.normal(size=(7, 3, 4, 4))
    S = ds.dynamic_spectra(I, ds.REF_MEAN, 1)            # [p][c][t]
    d = np.diff(I.reshape(7, 3, 16), axis=0)              # [t-1][c][p]
    assert np.allclose(S[:, :, 1:], np.transpose(d, (2, 1, 0)), rtol=0, atol=1e-15)
    assert np.all(S[:, :, 0] == 0)


def test_constant_cube_and_ramp():
    T, C, P = 12, 2, 5
    const = np.broadcast_to(np.arange(C * P, dtype=np.float64).reshape(1, C, P), (T, C, P))
    assert np.all(ds.dynamic_spectra(const, ds.REF_MEAN, 4) == 0)
    a, b = 3.0, 0.5
    ramp = np.broadcast_to((a + b * np.arange(T))[:, None, None], (T, C, P))
    K = 4
    S = ds.dynamic_spectra(ramp, ds.REF_MEAN, K)
    for t in range(1, T):
        k = min(K, t)
        assert np.allclose(S[:, :, t], b * (k + 1) / 2, rtol=0, atol=1e-13)


def test_model_equal_to_first_image():
    rng = np.random.default_rng(2)
    I = rng.normal(size=(5, 2, 3, 3))
    S = ds.dynamic_spectra(I, ds.REF_MODEL, ref_image=I[0])
    assert np.all(S[:, :, 0] == 0)
    assert np.allclose(S[:, :, 4], (I[4] - I[0]).reshape(2, 9).T)
