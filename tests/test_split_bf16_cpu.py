"""The three-term BF16 split behind the mixed-precision projector, emulated on the CPU (no GPU
arithmetic): v = h + m + l with h = bf16(v), m = bf16(v - h), l = bf16(v - h - m), and a real
product kept as the six largest term products.  Pins the accuracy claim the kernels rely on: the
dropped products and the last term's rounding stay below 2^-24 relative."""
import numpy as np


def _bf16(x):
    """Round FP64 values to BF16 (through FP32, nearest-even on the 16 dropped bits)."""
    f = np.asarray(x, np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def _split3(v):
    h = _bf16(v)
    m = _bf16(v - h)
    lo = _bf16(v - h - m)
    return h, m, lo


def test_split_terms_and_products():
    rng = np.random.default_rng(0)
    a = rng.standard_normal(200000) * 10.0 ** rng.uniform(-6, 3, 200000)
    b = rng.standard_normal(200000) * 10.0 ** rng.uniform(-6, 3, 200000)
    ah, am, al = _split3(a)
    bh, bm, bl = _split3(b)
    # every term is a BF16 value (8 significant bits)
    for t in (ah, am, al, bh, bm, bl):
        assert np.array_equal(_bf16(t), t)
    # the split represents each value to 2^-25 relative (two rounding steps below the 16th bit)
    assert np.max(np.abs(a - (ah + am + al)) / np.abs(a)) <= 2.0 ** -25
    # six products: hh, hm, mh, hl, mm, lh
    p6 = ah * bh + ah * bm + am * bh + ah * bl + am * bm + al * bh
    rel = np.abs(p6 - a * b) / np.abs(a * b)
    assert rel.max() <= 2.0 ** -24, rel.max()
    # three products (hh, hm, mh) would not do: they stop near 2^-16
    p3 = ah * bh + ah * bm + am * bh
    assert np.max(np.abs(p3 - a * b) / np.abs(a * b)) > 2.0 ** -20
