"""The three-product re-score tier (policy rescore3) of a BF16 first pass on the uint8 128x128x3
workload: the tier's logits against the oracle's FP64 logits, queries through the chain BF16 ->
three-product -> FP32 -> FP64 with ids equal to the oracle's, routes replayed, and the rules."""
import numpy as np
import pytest

import hydro_synth as hs
from oracle import hydro_oracle as ho
from tests.gpu_util import case, check_stats, log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2403_14902_amd import hydro  # noqa: E402


@pytest.fixture(scope="module")
def c5():
    return case(5, 1024)


@pytest.fixture(scope="module")
def c5z():
    return case(5, 64, logits=True)


def _cal(cfg):
    return torch.from_numpy(hs.make_frames(cfg, 0, 256, data_seed=cfg.data_seed + 101)).cuda()


def test_rescore3_tier_logits(c5z):
    """Tier 3 of a rescore3 session is the three-product arithmetic: within 1e-4 of the FP64
    logits (three products of at most about 2^-16 of |w x| dropped), not the FP32 tier's values, and
    between the FP32 and BF16 tiers' errors."""
    s = hydro.Session(c5z.specs(), hydro.make_policy("score", precision="bf16", rescore3=1), 128, 256)
    s.calibrate(_cal(c5z.cfg), "u8", safety=2.0)
    t0, t16, t32 = s.bands()
    log(f"[gpu] rescore3 bands tau={np.round(t0, 4).tolist()} tau16={t16.tolist()} tau32={t32.tolist()}")
    dev = c5z.device_frames()
    for k in range(c5z.cfg.k):
        z0, z3, z1 = (s.logits(k, t, dev, "u8") for t in (0, 3, 1))
        e0, e3, e1 = (float(np.abs(z - c5z.Z[k]).max()) for z in (z0, z3, z1))
        log(f"  predicate {k}: max |z - z64| bf16 {e0:.3e}, three-product {e3:.3e}, fp32 {e1:.3e}")
        assert e3 <= 1e-4                                   # measured 9.0e-6
        assert not np.array_equal(z3, z1)
        assert e1 <= e3 <= e0
        assert t32[k] <= t16[k] <= t0[k]
    s.close()


@pytest.mark.parametrize("route,graph", [("score", 0), ("fixed", 0), ("learned", 0), ("score", 1)])
def test_rescore3_query(c5, route, graph):
    """Ids equal to the oracle through the four-tier chain; the middle tier sees every first-pass
    deferral and passes a subset on."""
    pol = hydro.make_policy(route, precision="bf16", rescore3=1, wave=256, log_routes=1 - graph, use_graph=graph)
    s = hydro.Session(c5.specs(), pol, 128, c5.n)
    s.calibrate(_cal(c5.cfg), "u8", safety=3.0)
    dev = c5.device_frames()
    for rep in range(1 + graph):                 # a graph is captured, then replayed
        s.reset()
        s.push(dev, "u8", c5.pt.thresholds, c5.seg_len)
        ids, stats = s.finish()
        log(f"[gpu] rescore3 {route} graph={graph} rep {rep}: |R|={ids.size} "
            f"evaluated={[st['evaluated'] for st in stats]} rescored={[st['rescored'] for st in stats]} "
            f"rescored16={[st['rescored16'] for st in stats]} escalated={[st['escalated'] for st in stats]}")
        assert np.array_equal(ids, c5.expect)
        check_stats(stats, c5.n, ids.size)
        for st in stats:
            assert st["rescored16"] <= st["rescored"] <= st["evaluated"]
            assert st["escalated"] <= st["rescored16"]
        assert sum(st["rescored"] for st in stats) > 0
    if not graph:
        ok, rev, rps, out, msg = ho.replay_route(c5.P, hydro.decode_routes(s.routes(0, c5.n)))
        assert ok, msg
        assert [st["evaluated"] for st in stats] == list(rev)
        if route == "fixed":
            _, ev, ps = ho.short_circuit_eval(c5.P, [0, 1, 2, 3])
            assert [st["evaluated"] for st in stats] == list(ev)
            assert [st["passed"] for st in stats] == list(ps)
    s.close()


def test_rescore3_automatic_band(c5):
    """Without calibration the middle band is measured on the first push, floor 3e-4."""
    s = hydro.Session(c5.specs(), hydro.make_policy("score", precision="bf16", rescore3=1, wave=256), 128, c5.n)
    s.push(c5.device_frames(), "u8", c5.pt.thresholds, c5.seg_len)
    ids, stats = s.finish()
    _, t16, _ = s.bands()
    log(f"[gpu] rescore3 automatic tau16={t16.tolist()}")
    assert np.array_equal(ids, c5.expect)
    assert np.all(t16 >= np.float32(3e-4)) and np.all(t16 < 0.015)
    s.close()


def test_rescore3_rules(c5):
    for prec in ("fp32", "fp8"):
        with pytest.raises(hydro.HydroError) as e:
            hydro.Session(c5.specs(), hydro.make_policy("score", precision=prec, rescore3=1), 128, 16)
        assert e.value.code == hydro.EUNSUPPORTED
    c = case(1, 2048)
    with pytest.raises(hydro.HydroError) as e:
        hydro.Session(c.specs(), hydro.make_policy("score", precision="bf16", rescore3=1), 32, 16)
    assert e.value.code == hydro.EUNSUPPORTED
    with pytest.raises(hydro.HydroError) as e:
        hydro.Session(c5.specs(), hydro.make_policy("score", precision="bf16", rescore3=2), 128, 16)
    assert e.value.code == hydro.EINVAL



def test_rescore3_noalloc_capacity(c5):
    """The 4-layer CNNs' buffers (weight images of every tier, fp32 activations) exceed the
    allocation-free entry point's fixed array: with the middle tier as without it,
    hydro_query_noalloc returns ECAPACITY naming the size, and hydro_query answers."""
    n = 96
    dev = c5.device_frames()[:n]
    exp = ho.result_ids(c5.P[:n])
    for mid in (0, 1):
        pol = hydro.make_policy("score", precision="bf16", rescore3=mid, wave=64, tau=0.02, tau16=3e-4, tau32=1e-5)
        ids, stats = hydro.query(dev, "u8", c5.specs(), c5.pt.thresholds, c5.seg_len, pol)
        assert np.array_equal(ids, exp)
        check_stats(stats, n, ids.size)
        with pytest.raises(hydro.HydroError) as e:
            hydro.query_noalloc(dev, "u8", c5.specs(), c5.pt.thresholds, c5.seg_len, pol, out_cap=n)
        assert e.value.code == hydro.ECAPACITY and "bytes" in str(e.value)
