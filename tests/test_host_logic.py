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


def test_three_leading_products_bound():
    """The three-product tier keeps hi x hi + hi x mid + mid x hi of operands split as above
    (weights and fp32 activations alike) and drops the rest.  Since |w - hi| <= 2^-8 |w| and
    |w - hi - mid| <= 2^-16 |w| (bf16 keeps 8 significant bits), each dropped product is at most
    about 2^-16 |w x|: the kept sum is within 3 x 2^-16 (1 + 2^-7) |w x| of the exact product,
    and on typical operands far closer."""
    rng = np.random.default_rng(11)
    n = 400_000
    w = (rng.normal(0, 1, n) * 10.0 ** rng.uniform(-3, 1, n)).astype(np.float32)
    x = np.abs(rng.normal(0, 1, n) * 10.0 ** rng.uniform(-2, 2, n)).astype(np.float32)   # ReLU outputs

    def split(v):
        hi = _bf16(v)
        mid = _bf16((v - hi).astype(np.float32))
        return hi.astype(np.float64), mid.astype(np.float64)

    wh, wm = split(w)
    xh, xm = split(x)
    kept = wh * xh + wh * xm + wm * xh
    exact = w.astype(np.float64) * x.astype(np.float64)
    rel = np.abs(kept - exact) / np.abs(exact)
    assert rel.max() <= 3 * 2.0 ** -16 * (1 + 2.0 ** -7)
    assert np.median(rel) < 2.0 ** -18
    # and the residues are as stated
    assert np.all(np.abs(w - wh) <= 2.0 ** -8 * np.abs(w))
    assert np.all(np.abs(w - wh - wm) <= 2.0 ** -16 * np.abs(w))
