"""Error bounds of the low-precision chi0 operators, derived on the CPU.

The GPU test of the operators (test_gpu_mixed.py) bounds one chi0
application's normwise relative error by 3e-6 (FP32 transforms) and 3e-5
(split BF16 x 3 dense transforms, FP32 occupied ones).  Where these come from:

* FP32: each product's operands and the accumulation are rounded to
  u = 2^-24; normwise that is a few u sqrt(K) at these depths (K <= 5200),
  ~3e-7 per transform, and the operator chains four transforms.
* split BF16 x 3: x = hi + lo with hi = bf16(x), lo = bf16(x - hi), so
  |x - hi - lo| <= 2^-16 |x|; the product keeps hi.hi + hi.lo + lo.hi and
  drops lo.lo (also ~2^-16 relative); accumulation is FP32.  Normwise the
  neglected terms come to ~4e-6 per transform (emulated below), and the
  BF16 x 3 operator has two of them plus two FP32 transforms.

The bounds leave a factor of a few over these, and must still fail a split
product that lost one of its cross terms (hi.lo or lo.hi dropped: ~2^-9
per element), which the emulation shows to be ~60x above the bound.
"""
import numpy as np
import pytest

BOUND_FP32, BOUND_BF16X3 = 3e-6, 3e-5


def _bf16(x):
    """Round float32 to bfloat16 (nearest, ties to even), returned as float32."""
    u = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def _products(K, seed=0):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((128, K))
    B = rng.standard_normal((K, 128))
    C = A @ B
    A32, B32 = A.astype(np.float32), B.astype(np.float32)
    ah, bh = _bf16(A32), _bf16(B32)
    al, bl = _bf16(A32 - ah), _bf16(B32 - bh)
    f = lambda x: x.astype(np.float64)   # noqa: E731  exact products; FP32 accumulation is ~1e-7
    rel = lambda X: np.linalg.norm(X - C) / np.linalg.norm(C)   # noqa: E731
    return {"fp32": rel((A32 @ B32).astype(np.float64)),
            "bf16x3": rel(f(ah) @ f(bh) + f(ah) @ f(bl) + f(al) @ f(bh)),
            "bf16x3_no_hi_lo": rel(f(ah) @ f(bh) + f(al) @ f(bh)),
            "bf16x3_no_lo_hi": rel(f(ah) @ f(bh) + f(ah) @ f(bl))}


@pytest.mark.parametrize("K", [576, 1824, 5248])
def test_bounds_cover_the_arithmetic_and_catch_a_lost_cross_term(K):
    e = _products(K)
    # four chained transforms (two for BF16 x 3 plus two FP32) stay inside the bounds
    assert 4 * e["fp32"] < BOUND_FP32
    assert 2 * e["bf16x3"] + 2 * e["fp32"] < BOUND_BF16X3
    # a split product missing hi.lo or lo.hi fails the bound by far
    assert min(e["bf16x3_no_hi_lo"], e["bf16x3_no_lo_hi"]) > 30 * BOUND_BF16X3
    # and BF16 x 3 is really coarser than FP32 (the GPU test's lower bound)
    assert e["bf16x3"] > 3 * e["fp32"]
