"""GPU parity of the generic layer-wise CNN path on the uint8 128x128x3 workload (four CNN
predicates conv 32-64-128-256 + FC), including host-memory pushes through the staging ring."""
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


def test_c5_logits_each_tier(c5z):
    s = hydro.Session(c5z.specs(), hydro.make_policy("score", precision="bf16"), 128, c5z.n)
    dev = c5z.device_frames()
    for k in range(c5z.cfg.k):
        for tier, tol in ((0, 0.1), (1, 1e-4), (2, 1e-9)):
            err = np.abs(s.logits(k, tier, dev, "u8") - c5z.Z[k]).max()
            log(f"[gpu] c5 predicate {k} tier {tier}: max |z - z64| = {err:.3e}")
            assert err <= tol
    s.close()


@pytest.mark.parametrize("route,prec", [("score", "bf16"), ("fixed", "bf16"), ("score", "fp32")])
def test_c5_query_device_frames(c5, route, prec):
    cfg = c5.cfg
    cal = torch.from_numpy(hs.make_frames(cfg, 0, 256, data_seed=cfg.data_seed + 101)).cuda()
    s = hydro.Session(c5.specs(), hydro.make_policy(route, precision=prec, wave=256, log_routes=1), 128, c5.n)
    tau, tau32 = s.calibrate(cal, "u8", safety=3.0)
    log(f"[gpu] c5 tau={np.round(tau, 5).tolist()} tau32={tau32.tolist()}")
    s.push(c5.device_frames(), "u8", c5.pt.thresholds, c5.seg_len)
    ids, stats = s.finish()
    log(f"  |R|={ids.size} evaluated={[st['evaluated'] for st in stats]} rescored={[st['rescored'] for st in stats]}")
    assert np.array_equal(ids, c5.expect)
    check_stats(stats, c5.n, ids.size)
    ok, rev, rps, out, msg = ho.replay_route(c5.P, hydro.decode_routes(s.routes(0, c5.n)))
    assert ok, msg
    if route == "fixed":
        _, ev, ps = ho.short_circuit_eval(c5.P, [0, 1, 2, 3])
        assert [st["evaluated"] for st in stats] == list(ev)
        assert [st["passed"] for st in stats] == list(ps)
    s.close()


def test_c5_ungrouped_launches(c5z, c5):
    """One launch per predicate (the plain form): every predicate runs its own weights."""
    pol = hydro.make_policy("score", precision="fp32", grouped=0, wave=256)
    s = hydro.Session(c5z.specs(), pol, 128, 1024)
    dev = c5z.device_frames()
    for k in range(c5z.cfg.k):
        for tier in (0, 2):
            err = np.abs(s.logits(k, tier, dev, "u8") - c5z.Z[k]).max()
            log(f"[gpu] c5 ungrouped predicate {k} tier {tier}: max |z - z64| = {err:.3e}")
            assert err <= (1e-5 if tier == 0 else 1e-12)
    s.push(c5.device_frames(), "u8", c5.pt.thresholds, c5.seg_len)
    ids, stats = s.finish()
    assert np.array_equal(ids, c5.expect)
    check_stats(stats, c5.n, ids.size)
    s.close()


def test_c5_pinned_host_pushes(c5):
    """Frames pushed from pinned host memory in blocks, as the streaming form does."""
    pin = torch.from_numpy(c5.frames).pin_memory()
    s = hydro.Session(c5.specs(), hydro.make_policy("score", precision="bf16", wave=128), 128, 256)
    for lo in range(0, c5.n, 256):
        s.push(pin[lo:lo + 256], "u8", c5.pt.thresholds, c5.seg_len, id_base=lo)
    ids, stats = s.finish()
    assert np.array_equal(ids, c5.expect)
    check_stats(stats, c5.n, ids.size)
    s.close()


def test_c5_fp64_fallback_path(c5, monkeypatch):
    monkeypatch.setenv("HYDRO_ESC_CAP", "2")
    c = case(5, 256)
    s = hydro.Session(c.specs(), hydro.make_policy("score", precision="fp32", tau32=0.2, wave=128), 128, c.n)
    s.push(c.device_frames(), "u8", c.pt.thresholds, c.seg_len)
    ids, stats = s.finish()
    log(f"[gpu] c5 fp64-heavy escalated={[st['escalated'] for st in stats]}")
    assert sum(st["escalated"] for st in stats) > 20
    assert np.array_equal(ids, c.expect)
    s.close()
