"""The error bound of the three-term BF16 product (precision IFGF_FP32_BF16X3),
checked on the CPU with a bit-exact emulation of round-to-nearest-even BF16:
x = bf16(x) + bf16(x - bf16(x)) represents an FP32 x to about 2^-18, and
a b ~ a_lo b_hi + a_hi b_lo + a_hi b_hi (low-by-low dropped) to about 2^-16
relative, against 2^-24 for an FP32 product.  The GPU kernels are checked
against the oracle in the GPU parity tests; this pins the arithmetic claim."""
import numpy as np


def bf16_rne(x):
    """Round float32 values to the nearest bfloat16 (ties to even), as float32."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def split(x):
    hi = bf16_rne(x)
    lo = bf16_rne((x - hi).astype(np.float32))
    return hi, lo


def test_bf16_rounding_is_nearest_even():
    # 1 + 2^-8 lies halfway between 1 and 1 + 2^-7: ties to the even (1).
    assert bf16_rne(np.float32(1 + 2 ** -8)) == np.float32(1.0)
    # 1 + 3 * 2^-8 is halfway between 1 + 2^-7 and 1 + 2^-6: ties to 1 + 2^-6.
    assert bf16_rne(np.float32(1 + 3 * 2 ** -8)) == np.float32(1 + 2 ** -6)
    assert bf16_rne(np.float32(1 + 2 ** -7)) == np.float32(1 + 2 ** -7)
    assert bf16_rne(np.float32(-2.5)) == np.float32(-2.5)


def test_split_represents_fp32_to_2pow_minus_17():
    rng = np.random.default_rng(7)
    x = (rng.uniform(-1, 1, 200000) * 10.0 ** rng.uniform(-3, 3, 200000)).astype(np.float32)
    hi, lo = split(x)
    rel = np.abs((hi.astype(np.float64) + lo) - x) / np.abs(x.astype(np.float64))
    assert rel.max() <= 2.0 ** -17


def test_three_term_product_error_about_2pow_minus_16():
    rng = np.random.default_rng(8)
    a = rng.uniform(-3, 3, 200000).astype(np.float32)   # Lagrange weights
    b = rng.uniform(-50, 50, 200000).astype(np.float32)  # cone values
    ah, al = split(a)
    bh, bl = split(b)
    f64 = np.float64
    approx = f64(al) * bh + f64(ah) * bl + f64(ah) * bh
    exact = f64(a) * f64(b)
    rel = np.abs(approx - exact) / np.abs(exact)
    assert rel.max() <= 2.0 ** -15
    assert np.median(rel) <= 2.0 ** -17
    # Two terms (low-by-high dropped as well) would not reach it.
    two = f64(ah) * bh + f64(ah) * bl
    assert (np.abs(two - exact) / np.abs(exact)).max() > 2.0 ** -12


def test_dot_product_of_75_terms_stays_near_fp32():
    """A 75-term interpolation sum with Lagrange-sized weights: the split
    product's error relative to sum |a_q b_q| stays below 2^-15."""
    rng = np.random.default_rng(9)
    for _ in range(200):
        a = rng.uniform(-2, 2, 75).astype(np.float32)
        b = (rng.uniform(-1, 1, 75) * 20).astype(np.float32)
        ah, al = split(a)
        bh, bl = split(b)
        f64 = np.float64
        s3 = np.sum(f64(al) * bh + f64(ah) * bl + f64(ah) * bh)
        s = np.sum(f64(a) * f64(b))
        scale = np.sum(np.abs(f64(a) * f64(b)))
        assert abs(s3 - s) / scale <= 2.0 ** -15
