"""FP64 oracle of dynamic spectra with reference-image subtraction.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: only the test suite,
the package smoke check and the benchmark's CPU-baseline leg may import it.

Sec. 2 describes the pipeline around the imager: once the cube of images over
timesteps and channels exists, the time series of every pixel (a direction
on the sky) across channels - its dynamic spectrum - is formed and searched
for transients, and the artefacts of the dirty images are removed by
subtracting a reference image of the same field. Sec. 4.3 lists the reference
choices: the preceding dirty image, an average of the preceding images of the
same observation, or a model image. Readings used here:

* input cube I[t][c][p] (p = m M + l, the flattened M x M image), output
  S[p][c][t] (for each pixel, channel-major time series);
* reference NONE: S = I, transposed;
* reference MEAN with window K >= 1: S[p][c][t] = I[t][c][p] minus the mean of
  the k = min(K, t) preceding images I[t-k .. t-1][c][p]; at t = 0 there is
  no preceding image and S is 0. K = 1 is the preceding-image reference;
* reference MODEL: S[p][c][t] = I[t][c][p] - R[c][p], R given per channel.
"""
from __future__ import annotations

import numpy as np

REF_NONE = 0
REF_MEAN = 1
REF_MODEL = 2


def difference_cube(images, ref_mode: int, ref_len: int = 1, ref_image=None):
    """I[t][c][p] minus the reference, in float64 (same layout)."""
    I = np.asarray(images, dtype=np.float64)
    T = I.shape[0]
    if ref_mode == REF_NONE:
        return I.copy()
    if ref_mode == REF_MODEL:
        return I - np.asarray(ref_image, dtype=np.float64)[None]
    if ref_mode == REF_MEAN:
        if ref_len < 1:
            raise ValueError("window must be >= 1")
        D = np.zeros_like(I)
        for t in range(1, T):
            k = min(ref_len, t)
            ref = I[t - k:t].sum(axis=0) / k
            D[t] = I[t] - ref
        return D
    raise ValueError("unknown reference mode")


def dynamic_spectra(images, ref_mode: int, ref_len: int = 1, ref_image=None):
    """S[p][c][t] from I[t][c][m][l] (or I[t][c][p]) with the chosen reference."""
    I = np.asarray(images)
    T, C = I.shape[0], I.shape[1]
    D = difference_cube(I.reshape(T, C, -1), ref_mode, ref_len,
                        None if ref_image is None else np.asarray(ref_image).reshape(C, -1))
    return np.ascontiguousarray(np.transpose(D, (2, 1, 0)))
