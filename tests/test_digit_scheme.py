"""The fixed-point digit scheme of the reduced forms' occupied block, checked
on the CPU in numpy: each operand v in [-1/2, 1/2] written as six balanced
base-128 digits (the two FP64 roundings through the 1.5 2^52 shifter, then
three 7-bit fields of each 21-bit integer), and the sum of the digit products
of order <= 7.  These are the error statements the kernel's design rests on
(digit ranges, the 2^-43 representation bound, the bound on the products left
out, no sign bias); the GPU tests check the kernel itself against the FP64
block and exact sums."""
import numpy as np

SHIFT = 6755399441055744.0       # 1.5 * 2^52


def _low32(x):
    b = np.asarray(x, dtype=np.float64).view(np.uint64) & np.uint64(0xFFFFFFFF)
    return b.astype(np.uint32).view(np.int32).astype(np.int64)


def _sext7(x):
    x = x & 127
    return np.where(x >= 64, x - 128, x)


def digits(v):
    """[6][n] digits a_i with v = sum_i a_i 2^(-7 i) + e."""
    h = np.asarray(v, np.float64) * 2.0**21
    th = h + SHIFT
    hr = th - SHIFT
    tl = (h - hr) * 2.0**21 + SHIFT        # the product is exact: no rounding before the shift
    out = []
    for X in (_low32(th), _low32(tl)):
        u = X + 8256
        x = u ^ 0x2040
        out += [u >> 14, _sext7(x >> 7), _sext7(x)]
    return np.stack(out)


def kept_product(da, db):
    """sum of a_i b_j 2^(-7(i+j)) over i + j <= 7 (1-based digits)."""
    s = 0.0
    for o in range(6):
        for i in range(o + 1):
            s = s + da[i] * db[o - i] * 2.0 ** (-7 * (o + 2))
    return s


def _samples(seed, n):
    rng = np.random.default_rng(seed)
    edge = [0.0, 0.5, -0.5, 0.5 * (1 + 2e-16), -0.5 * (1 + 4e-16), 2.0**-43, -2.0**-44, 2.0**-21, 0.4999999999999]
    return np.concatenate([rng.uniform(-0.5, 0.5, n), rng.normal(0, 1e-3, n // 2), rng.normal(0, 1e-9, 1000), edge])


def test_digit_ranges_and_representation_error():
    v = _samples(1, 100000)
    d = digits(v)
    assert d[[0, 3]].min() >= -64 and d[[0, 3]].max() <= 64           # top digits of H and L
    assert d[[1, 2, 4, 5]].min() >= -64 and d[[1, 2, 4, 5]].max() <= 63
    rec = (d * 2.0 ** (-7 * np.arange(1, 7))[:, None]).sum(0)
    assert np.abs(rec - v).max() <= 2.0**-43
    assert abs((rec - v).mean()) < 1e-15                               # round to nearest: no bias


def test_left_out_products_bound():
    """The products of order >= 8 that the block leaves out are at most
    2.87e-13 (the figure the full-size test uses) for operands in
    [-1/2, 1/2]; with the representation errors the kept sum is within
    2^-43 (|a| + |b|) + 2.87e-13 of a b."""
    left_out = sum(64 * 64 * 2.0 ** (-7 * (i + j)) for i in range(1, 7) for j in range(1, 7) if i + j >= 8)
    assert left_out < 2.87e-13
    a, b = _samples(2, 100000), _samples(3, 100000)[::-1]
    err = np.abs(kept_product(digits(a), digits(b)) - a * b)
    assert np.all(err <= 2.0**-43 * (np.abs(a) + np.abs(b)) + 2.87e-13)


def test_sum_of_products_has_no_coherent_error():
    """Over many products the kept sums' errors cancel: their mean is far
    below the per-product bound (a coherent error would add up in the grid
    sums of K and then in E0)."""
    rng = np.random.default_rng(4)
    a = rng.uniform(-0.5, 0.5, 200000)
    b = rng.uniform(0.0, 0.5, 200000)          # one-signed, like a diagonal pair density
    e = kept_product(digits(a), digits(b)) - a * b
    assert abs(e.mean()) < 1e-15 and np.abs(e).max() < 3e-13


def test_int32_accumulators_hold_a_segment():
    """At most six digit pairs per order, each at most 64 x 64 in magnitude:
    a segment of 65 536 points cannot overflow the int32 accumulators."""
    assert 6 * 64 * 64 * 65536 < 2**31
