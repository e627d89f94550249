"""Routing, multi-split, forwarding and result materialisation on given predicate outcomes
(hydro_compaction_debug): the query path of sections 3.2-3.3 with the inference tiers replaced
by a lookup of each tuple's outcome in a bitmap.  Ids are compared with the oracle's
``result_ids`` and, for the written order, the per-predicate counts with its
``short_circuit_eval``; the random masks, the all-pass / none-pass cases, ragged sizes,
n = 0 and K = 1..8 follow the compaction edge cases of the test plan, and the 2^26-tuple
case is the size at which the kernels are measured."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2403_14902_amd import hydro
from oracle import hydro_oracle as ho
from tests.gpu_util import log

pytestmark = pytest.mark.gpu


def _bits(P: np.ndarray) -> np.ndarray:
    """Truth table [n][K] -> [K][ceil(n/32)] uint32 words, bit t % 32 of word t / 32."""
    n, k = P.shape
    words = (n + 31) // 32
    pad = np.zeros((k, words * 32), dtype=np.uint8)
    pad[:, :n] = P.T
    b = np.packbits(pad.reshape(k, words, 4, 8)[:, :, :, ::-1], axis=-1, bitorder="big")
    return b.reshape(k, words, 4).view("<u4").reshape(k, words)


def test_bit_packing_matches_definition():
    rng = np.random.default_rng(1)
    P = rng.random((100, 3)) < 0.5
    w = _bits(P)
    for j in range(3):
        for t in range(100):
            assert bool((int(w[j, t // 32]) >> (t % 32)) & 1) == P[t, j]


def _run(P, route="fixed", wave=1 << 20):
    n, k = P.shape
    bits = torch.from_numpy(_bits(P).astype(np.int32).reshape(-1).copy()).cuda() if n else torch.zeros(1, dtype=torch.int32).cuda()
    out = torch.full((max(1, n),), -1, dtype=torch.int64, device="cuda")
    cnt, stats, ms = hydro.compaction_debug(k, n, bits, out, route=route, wave=wave)
    return out[:cnt].cpu().numpy(), stats, ms


def _check_counts(P, ids, stats):
    """Every tuple outside the result failed exactly one predicate; passes never exceed
    evaluations; each result tuple passed all K."""
    n, k = P.shape
    ev = np.array([s["evaluated"] for s in stats])
    ps = np.array([s["passed"] for s in stats])
    assert np.all(ps <= ev)
    assert int((ev - ps).sum()) == n - ids.size
    assert np.all(ps >= ids.size)


@pytest.mark.parametrize("k", [1, 2, 3, 5, 8])
@pytest.mark.parametrize("n", [0, 1, 63, 64, 65, 1000, 100_003])
def test_fixed_order_counts_and_ids(k, n):
    rng = np.random.default_rng(1000 * k + n)
    sel = rng.uniform(0.3, 0.95, k)
    P = rng.random((n, k)) < sel
    ids, stats, _ = _run(P, "fixed", wave=4096)
    assert np.array_equal(ids, ho.result_ids(P))
    _, ev, ps = ho.short_circuit_eval(P, list(range(k)))
    assert [s["evaluated"] for s in stats] == list(ev)
    assert [s["passed"] for s in stats] == list(ps)


@pytest.mark.parametrize("route", ["selectivity", "score", "cost"])
def test_adaptive_routes_ids(route):
    rng = np.random.default_rng(7)
    n, k = 300_001, 4
    P = rng.random((n, k)) < np.array([0.9, 0.2, 0.6, 0.75])
    ids, stats, _ = _run(P, route, wave=8192)
    assert np.array_equal(ids, ho.result_ids(P))
    _check_counts(P, ids, stats)
    if route != "cost":
        # after the first round the most selective predicate (index 1) goes first
        assert stats[1]["evaluated"] > 0.95 * n


@pytest.mark.parametrize("fill", [True, False])
def test_all_pass_and_none_pass(fill):
    n, k = 70_000, 3
    P = np.full((n, k), fill)
    ids, stats, _ = _run(P, "score", wave=16_384)
    assert np.array_equal(ids, ho.result_ids(P))
    _check_counts(P, ids, stats)
    if fill:
        assert all(s["evaluated"] == n for s in stats)
    else:
        assert sum(s["evaluated"] for s in stats) == n


def test_pushes_of_2_24_at_2_26_tuples():
    """2^26 tuples (four pushes of 2^24, the entry format's local index range): ids against the
    numpy conjunction, counts against the written-order evaluation."""
    n, k = 1 << 26, 4
    rng = np.random.default_rng(26)
    P = rng.random((n, k), dtype=np.float32) < np.array([0.5, 0.7, 0.8, 0.9], dtype=np.float32)
    log(f"[gpu] compaction n=2^26 k={k}")
    ids, stats, ms = _run(P, "fixed", wave=1 << 22)
    assert np.array_equal(ids, ho.result_ids(P))
    _, ev, ps = ho.short_circuit_eval(P, list(range(k)))
    assert [s["evaluated"] for s in stats] == list(ev)
    assert [s["passed"] for s in stats] == list(ps)
    log(f"  |R|={ids.size} ms route={ms[0]:.3f} decide={ms[1]:.3f} results={ms[2]:.3f} total={ms[3]:.3f}")


def test_rejects_bad_arguments():
    bits = torch.zeros(4, dtype=torch.int32, device="cuda")
    out = torch.zeros(64, dtype=torch.int64, device="cuda")
    with pytest.raises(hydro.HydroError):
        hydro.compaction_debug(9, 64, bits.repeat(9), out)
    with pytest.raises(hydro.HydroError):
        hydro.compaction_debug(2, 64, bits, out, wave=32)
