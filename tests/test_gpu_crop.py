"""Variable-size inputs (section 5.3: a classifier on Crop(frame, bbox)) and the data-aware
scheduling of their work, through the C ABI: a CNN predicate on each tuple's crop beside a
whole-frame CNN predicate; ids against the oracle's ``crop_logits`` decisions for both
schedules (queue order, largest estimated work first) and several policies, routes replayed,
written orders counted exactly, and the argument rules."""
import numpy as np
import pytest

import hydro_synth as hs
from oracle import hydro_oracle as ho
from tests.gpu_util import case, check_stats, log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2403_14902_amd import hydro  # noqa: E402


def make_crops(n, side, seed):
    """Crops with log-uniform sides from 2 to the frame side (many small, a few large), at
    uniform positions inside the frame."""
    rng = np.random.default_rng(seed)
    h = np.minimum(side, np.round(np.exp(rng.uniform(np.log(2), np.log(side), n)))).astype(np.int32)
    w = np.minimum(side, np.round(np.exp(rng.uniform(np.log(2), np.log(side), n)))).astype(np.int32)
    y0 = (rng.random(n) * (side - h + 1)).astype(np.int32)
    x0 = (rng.random(n) * (side - w + 1)).astype(np.int32)
    return np.stack([y0, x0, h, w], axis=1).astype(np.int32)


@pytest.fixture(scope="module")
def cropcase():
    c = case(2, 4096)
    crops = make_crops(c.n, c.cfg.hw, 9)
    crop_model = c.weights[0]
    z = ho.crop_logits(crop_model, c.frames, c.cfg.dtype, crops)
    d = ho.predicate_margin(z, c.pt.class_masks[0])
    u = np.unique(d)
    m = np.searchsorted(u, np.median(d))
    theta = np.float32((u[m - 1] + u[m]) / 2.0)
    gap = float(np.abs(d - float(theta)).min())
    assert gap > 1e-9
    th = np.concatenate([np.full((c.pt.thresholds.shape[0], 1), theta, np.float32), c.pt.thresholds[:, [2]]],
                        axis=1).astype(np.float32)
    P = np.concatenate([(d > float(theta))[:, None], c.P[:, [2]]], axis=1)
    specs = [hydro.ModelSpec.from_weights(crop_model, c.pt.class_masks[0], on_crop=True, in_hw=c.cfg.hw),
             c.specs()[2]]
    log(f"[oracle] crop predicate: theta {float(theta):.6f}, pass rate {P[:, 0].mean():.3f}, min gap {gap:.3g}")
    return c, crops, specs, th, P


@pytest.mark.parametrize("balance", [0, 1])
@pytest.mark.parametrize("route", ["score", "cost"])
def test_crop_predicate_ids_and_routes(cropcase, balance, route):
    c, crops, specs, th, P = cropcase
    s = hydro.Session(specs, hydro.make_policy(route, wave=1024, log_routes=1, balance=balance), c.cfg.hw, c.n)
    s.push(c.device_frames(), c.cfg.dtype, th, c.seg_len, crops=crops)
    ids, stats = s.finish()
    assert np.array_equal(ids, ho.result_ids(P))
    check_stats(stats, c.n, ids.size)
    ok, rev, rps, out, msg = ho.replay_route(P, hydro.decode_routes(s.routes(0, c.n)))
    assert ok, msg
    assert [st["evaluated"] for st in stats] == list(rev)
    s.close()


@pytest.mark.parametrize("balance", [0, 1])
def test_crop_predicate_written_order_pushes(cropcase, balance):
    c, crops, specs, th, P = cropcase
    s = hydro.Session(specs, hydro.make_policy("fixed", order=[0, 1], wave=1024, balance=balance), c.cfg.hw, 1024)
    dev = c.device_frames()
    for lo in range(0, c.n, 1024):
        s.push(dev[lo:lo + 1024], c.cfg.dtype, th, c.seg_len, id_base=lo, crops=crops[lo:lo + 1024])
    ids, stats = s.finish()
    assert np.array_equal(ids, ho.result_ids(P))
    _, ev, ps = ho.short_circuit_eval(P, [0, 1])
    assert [st["evaluated"] for st in stats] == list(ev)
    assert [st["passed"] for st in stats] == list(ps)
    s.close()


def test_crop_rules(cropcase):
    c, crops, specs, th, P = cropcase
    s = hydro.Session(specs, hydro.make_policy("score"), c.cfg.hw, 64)
    dev = c.device_frames()[:64]
    with pytest.raises(hydro.HydroError):            # crops required
        s.push(dev, c.cfg.dtype, th, c.seg_len)
    bad = crops[:64].copy()
    bad[3] = [60, 0, 8, 8]                            # leaves the frame
    with pytest.raises(hydro.HydroError):
        s.push(dev, c.cfg.dtype, th, c.seg_len, crops=bad)
    with pytest.raises(hydro.HydroError):            # no whole-frame logits
        s.logits(0, 0, dev, c.cfg.dtype)
    s.close()
