"""The arithmetic the network forward relies on (no GPU): an FP32 value truncated to its BF16
head leaves a remainder of at most 16 significant bits, whose own BF16 head leaves at most
8, which BF16 holds; so x = hi + mid + lo exactly with three BF16 terms while the remainders
are normal numbers (|x| >= 2^-110), and below that the third term, packed as its BF16 head,
drops less than 2^-133.  The product of a BF16 weight with each term is exact in FP32 (8 x 8
significant bits)."""
import numpy as np


def bf16_head(x):
    """Round toward zero to BF16 (keep the top 16 bits of the FP32 encoding)."""
    return (x.view(np.uint32) & np.uint32(0xFFFF0000)).view(np.float32)


def is_bf16(x):
    return np.all((x.view(np.uint32) & np.uint32(0xFFFF)) == 0)


def split3(x):
    hi = bf16_head(x)
    r1 = (x - hi).astype(np.float32)
    mid = bf16_head(r1)
    lo = (r1 - mid).astype(np.float32)
    return hi, mid, lo


def test_three_term_split_is_exact():
    rng = np.random.default_rng(0)
    x = np.concatenate([
        rng.standard_normal(200000).astype(np.float32) * np.float32(3.0),
        (rng.standard_normal(20000) * 1e-30).astype(np.float32),
        (rng.standard_normal(20000) * 1e-36).astype(np.float32),
        (rng.standard_normal(20000) * 1e30).astype(np.float32),
        np.array([0.0, -0.0, 1.0, -1.0, np.float32(1) + np.float32(2.0 ** -23), 3.4e38, 1.2e-38], dtype=np.float32),
    ])
    hi, mid, lo = split3(x)
    assert is_bf16(hi) and is_bf16(mid)
    # the sum of the three terms, taken in double (exact for these magnitudes), is x
    assert np.array_equal(hi.astype(np.float64) + mid.astype(np.float64) + lo.astype(np.float64), x.astype(np.float64))
    # the third term is a BF16 value where the remainders are normal numbers
    normal = np.abs(x) >= np.float32(2.0 ** -110)
    assert is_bf16(lo[normal])
    # below, packing it as its BF16 head (as the kernel does) drops less than 2^-133
    packed = hi.astype(np.float64) + mid.astype(np.float64) + bf16_head(lo).astype(np.float64)
    assert np.all(np.abs(packed - x.astype(np.float64))[~normal] < 2.0 ** -133)
    assert (~normal).sum() > 1000


def test_bf16_products_are_exact_in_fp32():
    rng = np.random.default_rng(1)
    w = bf16_head(rng.standard_normal(100000).astype(np.float32))
    x = rng.standard_normal(100000).astype(np.float32) * np.float32(10.0)
    for t in split3(x):
        p32 = (w * t).astype(np.float32)
        assert np.array_equal(p32.astype(np.float64), w.astype(np.float64) * t.astype(np.float64))
    # and the three products sum to the exact product w x (in double)
    hi, mid, lo = split3(x)
    exact = w.astype(np.float64) * x.astype(np.float64)
    parts = sum((w * t).astype(np.float64) for t in (hi, mid, lo))
    assert np.array_equal(parts, exact)
