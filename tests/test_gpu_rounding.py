"""Storage rounding of the reduced forms, bit for bit: pm_write of float64
planes followed by pm_read gives float32 round-to-nearest-even (FP32) and
bfloat16 round-to-nearest-even of that float32 value (BF16), computed here
independently from the bit patterns with numpy.  Inputs: random float32 bit
patterns over the whole finite range (subnormals included), exact halfway
cases with even and odd kept bits, doubles that are not float32 values,
the largest finite values (which round to infinity in bfloat16), signed
zeros and infinities; a NaN must stay a NaN."""
import numpy as np
import pytest

import paper_2004_02833_amd as pm

from gpu_util import say

pytestmark = pytest.mark.gpu

SHAPE = (16, 64, 64)


def bf16_rne(f32):
    """float32 array -> float64 values of its bfloat16 round-to-nearest-even."""
    b = np.asarray(f32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) & 0xFFFF
    return (r.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def inputs():
    rng = np.random.default_rng(7)
    n = int(np.prod(SHAPE))
    bits = rng.integers(0, 2 ** 32, size=n, dtype=np.uint64).astype(np.uint32)
    finite = (bits & 0x7F800000) != 0x7F800000
    bits = np.where(finite, bits, bits & 0xBFFFFFFF)            # exponent 0xff -> 0x7f
    v = bits.view(np.float32).astype(np.float64)
    k = 0
    # halfway cases: low 16 bits exactly 0x8000, kept lowest bit 0 and 1
    for hi in (0x3F80, 0x3F81, 0x4049, 0x404A, 0x0001, 0x0002, 0x7F7E, 0x7F7F, 0xBF80, 0xBF81):
        for lo in (0x8000, 0x7FFF, 0x8001):
            v[k] = np.array([(hi << 16) | lo], dtype=np.uint32).view(np.float32)[0]
            k += 1
    # doubles that are not float32 values (rounded twice: to float32, then bfloat16)
    d = rng.normal(size=2000) * np.exp(rng.uniform(-80, 80, 2000))
    v[k:k + d.size] = d
    k += d.size
    specials = [0.0, -0.0, np.inf, -np.inf, 3.4028234663852886e38, -3.4028234663852886e38,
                1.401298464324817e-45, -1.401298464324817e-45, 1.1754943508222875e-38]
    v[k:k + len(specials)] = specials
    k += len(specials)
    v[k] = np.nan
    return v.reshape(SHAPE), k


@pytest.mark.parametrize("prec", [1, 2])
def test_write_read_rounds_to_nearest_even(prec):
    v, inan = inputs()
    flat = v.reshape(-1)
    nz, ny, nx = SHAPE
    pm.pm_set_precision(prec)
    pm.pm_init(0, nx, ny, nz, 0.1, 0.05, np.zeros(SHAPE), np.zeros(SHAPE))
    try:
        pm.pm_write(0, v)
        got = pm.pm_read(0).reshape(-1)
    finally:
        pm.pm_finalize()
    f32 = flat.astype(np.float32)
    want = f32.astype(np.float64) if prec == 1 else bf16_rne(f32)
    ok = np.ones(flat.size, dtype=bool)
    ok[inan] = False
    bad = np.flatnonzero((got[ok].view(np.uint64) != want[ok].view(np.uint64)))
    say("prec %d: %d values, %d differ" % (prec, ok.sum(), bad.size))
    assert bad.size == 0, (flat[ok][bad[:5]], got[ok][bad[:5]], want[ok][bad[:5]])
    assert np.isnan(got[inan])
