"""FP64 / integer oracle of the correlator X-engine.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: only the test suite,
the package smoke check and the benchmark's CPU-baseline leg may import it.

Sec. 4.1 (FX correlation): the channelised complex voltages of antennas i and
j in the same channel are multiplied, V_ij = Vhat_i Vhat_j, for the
N(N+1)/2 pairs including the autocorrelations, and accumulated over the n_t
samples of an integration. Readings used here:

* the product carries the conjugate of the second antenna,
  V_ij = sum_s x_i(s) conj(x_j(s)) (the equation as printed drops it; with
  it, V_ji = conj(V_ij) and the autocorrelations are real);
* the accumulation is the plain sum over the integration's samples (an
  average is the same up to the factor 1/n_t, which normalised images do
  not see), so integer voltages give exact integer visibilities;
* input x[t][c][a][s] complex (8-bit integer real and imaginary parts),
  output vis[t][c][b] for the pairs i < j in row-major upper-triangle order
  (the baseline order of the imaging inputs) and autos[t][c][a] = V_aa.
"""
from __future__ import annotations

import numpy as np


def pair_index(i, j, n_ant: int):
    """Baseline index of the pair i < j in row-major upper-triangle order."""
    i = np.asarray(i)
    j = np.asarray(j)
    return i * n_ant - i * (i + 1) // 2 + (j - i - 1)


def correlation_matrix(x):
    """Full matrix V[..., i, j] = sum_s x[..., i, s] conj(x[..., j, s]) (complex128)."""
    x = np.asarray(x, dtype=np.complex128)
    return x @ np.conj(np.swapaxes(x, -1, -2))


def correlate(volt):
    """(vis [T][C][B] complex128, autos [T][C][A] float64) from int8 volt [T][C][A][S][2]."""
    v = np.asarray(volt)
    x = v[..., 0].astype(np.float64) + 1j * v[..., 1].astype(np.float64)   # exact for 8-bit parts
    V = correlation_matrix(x)
    A = x.shape[-2]
    i, j = np.triu_indices(A, k=1)
    return V[..., i, j], np.real(np.diagonal(V, axis1=-2, axis2=-1)).copy()
