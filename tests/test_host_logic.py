"""Host-side arithmetic facts the kernels rely on (CPU)."""
import numpy as np


def _bf16(x: np.ndarray) -> np.ndarray:
    """fp32 -> bf16 (round to nearest even) -> fp32."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32)


def test_three_bf16_terms_carry_an_fp32_weight_exactly():
    """w = hi + mid + lo with hi = bf16(w), mid = bf16(w - hi), lo = bf16(w - hi - mid): every
    fp32 value of the weights' range is the exact sum of its three terms, and each product of a
    bf16 frame value with a term is exact in fp32, so the three-term GEMM computes the fp32
    GEMM's products exactly."""
    rng = np.random.default_rng(5)
    w = np.concatenate([rng.normal(0, s, 200_000) for s in (1e-3, 1e-2, 0.1, 1.0, 10.0)]).astype(np.float32)
    w = (w * 4.0).astype(np.float32)                      # the folded scale of bf16 frames
    hi = _bf16(w)
    r1 = (w - hi).astype(np.float32)
    assert np.array_equal(r1.astype(np.float64), w.astype(np.float64) - hi.astype(np.float64))
    mid = _bf16(r1)
    r2 = (r1 - mid).astype(np.float32)
    assert np.array_equal(r2.astype(np.float64), r1.astype(np.float64) - mid.astype(np.float64))
    lo = _bf16(r2)
    assert np.array_equal(lo, r2)                          # the remainder is itself a bf16 value
    total = hi.astype(np.float64) + mid.astype(np.float64) + lo.astype(np.float64)
    assert np.array_equal(total, w.astype(np.float64))
    x = _bf16(rng.uniform(0, 1, w.size).astype(np.float32))
    for t in (hi, mid, lo):
        p32 = (x * t).astype(np.float32).astype(np.float64)
        assert np.array_equal(p32, x.astype(np.float64) * t.astype(np.float64))
