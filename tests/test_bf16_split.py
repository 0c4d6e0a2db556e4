"""Host check of the exact three-term BF16 split used by the precision form's
matrix-core products: for FP32 x, hi = x with the low 16 bits cleared,
mid = (x - hi) cleared the same way, lo = x - hi - mid.  The two differences
are exact in FP32, lo fits in BF16, and hi + mid + lo = x exactly, so each
product a * x with a BF16-valued a is the exact sum of three products of BF16
values (each exact in FP32).  This holds while lo is a normal number, i.e. for
|x| >= 2^-110; below that (far under any data scale of the method) the
lowest bits are dropped, an error under 2^-126 in absolute terms."""
import numpy as np

MASK = np.uint32(0xFFFF0000)


def split(x):
    x = np.asarray(x, dtype=np.float32)
    hi = (x.view(np.uint32) & MASK).view(np.float32)
    r = (x - hi).astype(np.float32)
    mid = (r.view(np.uint32) & MASK).view(np.float32)
    lo = (r - mid).astype(np.float32)
    return hi, mid, lo


def test_split_is_exact_and_bf16():
    rng = np.random.default_rng(0)
    x = (rng.standard_normal(200000) * 2.0 ** rng.integers(-60, 60, size=200000)).astype(np.float32)
    x = np.concatenate([x, np.float32([0.0, -0.0, 1.0, -1.0, 1.0 + 2.0 ** -23, 3.4e38, 2.0 ** -110])])
    hi, mid, lo = split(x)
    for t in (hi, mid, lo):
        assert np.all((t.view(np.uint32) & np.uint32(0xFFFF)) == 0)     # BF16-representable
    s = hi.astype(np.float64) + mid.astype(np.float64) + lo.astype(np.float64)
    assert np.array_equal(s, x.astype(np.float64))


def test_split_products_exact():
    rng = np.random.default_rng(1)
    a = ((rng.standard_normal(50000).astype(np.float32).view(np.uint32) & MASK).view(np.float32))
    x = rng.standard_normal(50000).astype(np.float32)
    for t in split(x):
        p32 = (a * t).astype(np.float32)
        assert np.array_equal(p32.astype(np.float64), a.astype(np.float64) * t.astype(np.float64))


def test_split_below_normal_range_error_tiny():
    x = np.float32([1.2e-38, -3e-36, 2.0 ** -120])
    hi, mid, lo = split(x)
    lo_b = (lo.view(np.uint32) & MASK).view(np.float32)
    err = np.abs(hi.astype(np.float64) + mid + lo_b - x.astype(np.float64))
    assert np.all(err < 2.0 ** -126)
