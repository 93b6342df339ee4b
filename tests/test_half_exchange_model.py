"""Host model of the half-length LDS exchange of the column and row kernels.

The kernels run every Stockham stage-to-stage exchange of a length-N transform
through a padded buffer of N/2 points in two rounds: a stage writes the
outputs of its butterflies j < N/(2R) (exactly the outputs below N/2), the
next stage reads its inputs x[j + r N/R'] with r < R'/2 (exactly the inputs
below N/2), then the upper halves follow at padded index - pad(N/2). This
test replays that index arithmetic in numpy for every power-of-two plan the
kernels use (radix 16, then 8, 4, 2 as the length allows), checks that every
access stays inside the buffer, that no round overwrites a value before the
next stage has read it, and that the result equals numpy's transform. It
models the indexing only; the GPU parity tests check the kernels themselves.
"""
import numpy as np
import pytest


def pick_radix(rem):
    for r in (16, 8, 4, 2):
        if rem % r == 0:
            return r
    raise ValueError(rem)


def pad(i):
    return i + (i >> 4)


def padded_len(n):
    return n + (n >> 4) + 4


def plan(n):
    out, cur = [], 1
    while cur < n:
        r = pick_radix(n // cur)
        out.append((r, cur))
        cur *= r
    return out


def dft(v, sign):
    r = len(v)
    k = np.arange(r)
    return np.exp(sign * 2j * np.pi * np.outer(k, k) / r) @ v


def stage_compute(n, r, ns, sign, v):
    """v[j][r]: twiddle by w_{NS R}^(sign (j mod NS) r) and the length-R DFT."""
    nb = n // r
    out = np.empty_like(v)
    for j in range(nb):
        k = j % ns
        x = v[j] * np.exp(sign * 2j * np.pi * k * np.arange(r) / (ns * r))
        out[j] = dft(x, sign)
    return out


def read_index(n, r, j, rr, hf):
    """Padded read index of input x[j + rr N/R] in round hf, in both forms the
    kernels use: per-lane base plus a compile-time offset when N/R is a
    multiple of 16, the direct formula otherwise."""
    nb = n // r
    direct = pad(j + rr * nb) - hf * pad(n // 2)
    if nb % 16 == 0:
        assert pad(j) + (rr * (nb + nb // 16) - hf * pad(n // 2)) == direct
    return direct


def write_index(n, r, ns, j, rr, hf):
    """Padded write index of output rr of butterfly j in round hf (both forms)."""
    base = (j // ns) * ns * r + j % ns
    direct = pad(base + rr * ns) - hf * pad(n // 2)
    if ns % 16 == 0 or (ns == 1 and 16 % r == 0):
        step = 1 if ns == 1 else ns + ns // 16
        assert pad(base) - hf * pad(n // 2) + rr * step == direct
    return direct


def half_exchange(n, sign, x):
    h, length = n // 2, padded_len(n // 2)
    stages = plan(n)
    buf = np.full(length, np.nan + 0j)
    # first stage inputs come from the gridded column, also in two rounds
    r0, _ = stages[0]
    nb0 = n // r0
    v = np.empty((nb0, r0), dtype=complex)
    for hf in (0, 1):
        buf[:] = np.nan
        for row in range(hf * h, (hf + 1) * h):
            buf[pad(row - hf * h)] = x[row]
        for j in range(nb0):
            for r in range(hf * r0 // 2, (hf + 1) * r0 // 2):
                idx = read_index(n, r0, j, r, hf)
                assert 0 <= idx < length and not np.isnan(buf[idx])
                v[j][r] = buf[idx]
    for s, (r, ns) in enumerate(stages):
        v = stage_compute(n, r, ns, sign, v)
        if s == len(stages) - 1:
            y = np.empty(n, dtype=complex)
            for j in range(n // r):
                for rr in range(r):
                    y[j + rr * ns] = v[j][rr]          # last stage: q = j + r NS
            return y
        r2, _ = stages[s + 1]
        nb, nb2 = n // r, n // r2
        v2 = np.empty((nb2, r2), dtype=complex)
        for hf in (0, 1):
            buf[:] = np.nan                             # whatever the buffer held is dead
            written = set()
            for j in range(nb):
                if (j < nb // 2) != (hf == 0):
                    continue
                base = (j // ns) * ns * r + j % ns
                for rr in range(r):
                    e = base + rr * ns
                    assert (e < h) == (hf == 0)         # the round holds its half only
                    idx = write_index(n, r, ns, j, rr, hf)
                    assert 0 <= idx < length and idx not in written
                    written.add(idx)
                    buf[idx] = v[j][rr]
            assert len(written) == h
            for j in range(nb2):
                for rr in range(hf * r2 // 2, (hf + 1) * r2 // 2):
                    idx = read_index(n, r2, j, rr, hf)
                    assert 0 <= idx < length and not np.isnan(buf[idx])
                    v2[j][rr] = buf[idx]
        v = v2


@pytest.mark.parametrize("n", [32, 64, 128, 256, 512, 1024, 2048])
def test_half_exchange_matches_numpy(n):
    rng = np.random.default_rng(n)
    x = rng.normal(size=n) + 1j * rng.normal(size=n)
    y = half_exchange(n, +1, x)
    ref = np.fft.ifft(x) * n                            # sum_k x_k exp(+2 pi i k q / N)
    assert np.allclose(y, ref, rtol=0, atol=1e-9 * np.abs(ref).max())


def test_rounds_split_at_half_for_every_stage():
    # the property the two rounds rest on, for every stage but the last
    for n in (32, 64, 128, 256, 512, 1024, 2048):
        for r, ns in plan(n)[:-1]:
            assert (n // 2) % (ns * r) == 0
            nb = n // r
            for j in range(nb):
                base = (j // ns) * ns * r + j % ns
                lows = [base + rr * ns < n // 2 for rr in range(r)]
                assert all(lows) if j < nb // 2 else not any(lows)


# ---------------------------------------------------------------- zero band
def zero_band(n, bound):
    """The rule the kernels use: the widest of 6, 4 middle inputs of a radix-16
    first stage that every nonzero row (min(i, n - i) < bound) avoids."""
    if pick_radix(n) != 16:
        return 0
    for zb in (6, 4):
        if bound <= n // 2 - zb * (n // 32):
            return zb
    return 0


@pytest.mark.parametrize("n", [32, 64, 128, 256, 512, 1024, 2048])
def test_zero_band_inputs_are_empty_rows(n):
    """A radix-16 first stage reads x[j + r n/16] for butterfly j < n/16; the
    band r in [8 - zb/2, 8 + zb/2) covers rows [n/2 - zb n/32, n/2 + zb n/32).
    For every bound, those rows hold no row with min(i, n - i) < bound, so
    skipping those inputs leaves every butterfly's result unchanged; the
    transform with the band zeroed equals the full one."""
    rng = np.random.default_rng(n)
    nb = n // 16
    for bound in range(0, n // 2 + 2):
        zb = zero_band(n, bound)
        if zb == 0:
            continue
        rows = [j + r * nb for j in range(nb) for r in range(8 - zb // 2, 8 + zb // 2)]
        assert min(rows) == n // 2 - zb * n // 32 and max(rows) == n // 2 + zb * n // 32 - 1
        assert all(min(i, n - i) >= bound for i in rows)
    # a column whose rows reach exactly the bound: the band's inputs are zero
    for bound, zb in ((n // 2 - 6 * n // 32, 6), (n // 2 - 4 * n // 32, 4)):
        assert zero_band(n, bound) == zb and zero_band(n, bound + 1) < zb
        x = np.zeros(n, complex)
        i = np.arange(n)
        live = np.minimum(i, n - i) < bound
        x[live] = rng.normal(size=live.sum()) + 1j * rng.normal(size=live.sum())
        band = np.zeros(n, bool)
        band[n // 2 - zb * n // 32: n // 2 + zb * n // 32] = True
        assert not np.any(live & band)
