"""The float-reciprocal division the LDS tail kernels use to split a flat
index into (z, y, x): q = trunc(float(e) * float(1/m)) followed by one
correction step.  Emulated here in IEEE float32 (the device arithmetic),
with the reciprocal exact or one ulp off (a hardware reciprocal), against
exact integer division over every divisor the kernels meet and the edge
dividends of the stated range e < 2^22."""
import numpy as np
import pytest


def _small_div(e, m, rcp):
    q = (e.astype(np.float32) * np.float32(rcp)).astype(np.int64)  # truncation toward zero
    r = e - q * m
    return q + (r >= m).astype(np.int64) - (r < 0).astype(np.int64)


def _dividends(m, rng):
    top = 1 << 22
    e = [np.arange(0, 2048), top - 1 - np.arange(0, 2048)]
    # multiples of m and their neighbours, where truncation is most fragile
    k = rng.integers(0, top // m + 1, size=1500)
    e += [k * m - 1, k * m, k * m + 1, rng.integers(0, top, size=1500)]
    e = np.concatenate(e)
    return e[(e >= 0) & (e < top)].astype(np.int64)


@pytest.mark.parametrize("ulps", [0, 1, -1])
def test_small_div_matches_integer_division(ulps):
    rng = np.random.default_rng(5)
    divisors = sorted(set(list(range(1, 130)) + [2 ** k for k in range(8, 22)] +
                          [2 ** k + 1 for k in range(8, 21)] + [3 * 2 ** k for k in range(8, 20)] +
                          list(rng.integers(130, 1 << 21, size=60))))
    for m in divisors:
        rcp = np.float32(1.0) / np.float32(m)
        for _ in range(abs(ulps)):
            rcp = np.nextafter(rcp, np.float32(np.inf if ulps > 0 else 0.0), dtype=np.float32)
        e = _dividends(m, rng)
        q = _small_div(e, m, rcp)
        assert np.array_equal(q, e // m), m
