"""GPU parity of the fused CNN path (64x64x3 frames, CNN predicates of widths (16m, 32m, 64m),
m = 1, 2, 4, drifting thresholds over 8 segments) against the FP64 oracle, through the C ABI."""
import itertools

import numpy as np
import pytest

import hydro_synth as hs
from oracle import hydro_oracle as ho
from tests.gpu_util import case, check_stats, log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2403_14902_amd import hydro  # noqa: E402


@pytest.fixture(scope="module")
def c2small():
    return case(2, 256, logits=True)


@pytest.fixture(scope="module")
def c2():
    # two drift segments (8192 tuples each)
    return case(2, 16384)


@pytest.mark.parametrize("tier", [0, 1])
def test_cnn_logits_batch_invariant_across_entry_ring_refills(tier):
    """One logits call over 70,000 frames (each workgroup then takes more than 128 frames, so the
    LDS ring holding its queue entries is refilled at least twice) equals four calls of 17,500
    frames bit for bit: a frame's logits do not depend on the batch it travels in."""
    cfg = hs.workload(2)
    n, blk = 70000, 17500
    frames = hs.make_frames_parallel(cfg, 0, n)
    pt = hs.load_predicates(cfg)
    specs = [hydro.ModelSpec.from_weights(hs.make_model(d), m) for d, m in zip(cfg.models, pt.class_masks)]
    s = hydro.Session(specs, hydro.make_policy("score", precision="bf16"), 64, n)
    dev = torch.from_numpy(frames).cuda()
    for k in (0, 2):          # the narrowest and the widest class
        log(f"[gpu] ring refills: tier {tier} predicate {k}, {n} frames")
        z_all = s.logits(k, tier, dev, cfg.dtype)
        z_blk = np.concatenate([s.logits(k, tier, dev[lo:lo + blk].contiguous(), cfg.dtype)
                                for lo in range(0, n, blk)])
        assert np.array_equal(z_all, z_blk)
    s.close()


# tolerances: a few times the largest errors measured on these frames (bf16 6.6e-3, fp32 4.5e-7,
# fp64 2.7e-15); the kernels are deterministic, so the errors do not vary between runs
@pytest.mark.parametrize("prec,tier,tol", [("bf16", 0, 0.03), ("bf16", 1, 5e-6), ("fp32", 0, 5e-6), ("bf16", 2, 1e-13)])
def test_cnn_logits_each_tier_vs_oracle(c2small, prec, tier, tol):
    c = c2small
    s = hydro.Session(c.specs(), hydro.make_policy("score", precision=prec), 64, c.n)
    dev = c.device_frames()
    for k in range(c.cfg.k):
        z = s.logits(k, tier, dev, c.cfg.dtype)
        err = np.abs(z - c.Z[k]).max()
        log(f"[gpu] cnn logits prec={prec} tier={tier} predicate {k}: max |z - z64| = {err:.3e}")
        assert err <= tol
    s.close()


def test_cnn_uint8_frames_logits_and_ids():
    """uint8 frames (value v/255) through the same CNN predicates."""
    cfg = hs.workload(2)
    fr = hs.make_frames(cfg, 0, 512)
    x = ho.frames_to_f64(fr, "bf16")
    u8 = np.rint(255.0 * x).astype(np.uint8)
    pt = hs.load_predicates(cfg)
    weights = [hs.make_model(d) for d in cfg.models]
    P, D, Z = ho.truth_table(u8, "u8", weights, pt.class_masks, pt.thresholds, cfg.n // cfg.n_seg,
                             return_logits=True)
    specs = [hydro.ModelSpec.from_weights(w, m) for w, m in zip(weights, pt.class_masks)]
    dev = torch.from_numpy(u8).cuda()
    s = hydro.Session(specs, hydro.make_policy("score", precision="bf16"), 64, 512)
    for k in range(3):
        for tier, tol in ((0, 0.05), (1, 5e-6), (2, 1e-13)):      # measured 1.04e-2, 5.2e-7, 2.2e-15
            err = np.abs(s.logits(k, tier, dev, "u8") - Z[k]).max()
            log(f"[gpu] u8 logits tier {tier} predicate {k}: {err:.3e}")
            assert err <= tol
    s.push(dev, "u8", pt.thresholds, cfg.n // cfg.n_seg)
    ids, stats = s.finish()
    assert np.array_equal(ids, ho.result_ids(P))
    s.close()


@pytest.mark.parametrize("route,prec", [("score", "bf16"), ("score", "fp32"), ("selectivity", "bf16"),
                                        ("cost", "bf16")])
def test_cnn_adaptive_ids_stats_replay(c2, route, prec):
    log(f"[gpu] cnn route={route} prec={prec}")
    pol = hydro.make_policy(route, precision=prec, wave=4096, log_routes=1)
    s = hydro.Session(c2.specs(), pol, 64, c2.n)
    s.push(c2.device_frames(), c2.cfg.dtype, c2.pt.thresholds, c2.seg_len)
    ids, stats = s.finish()
    assert np.array_equal(ids, c2.expect)
    check_stats(stats, c2.n, ids.size)
    ok, rev, rps, out, msg = ho.replay_route(c2.P, hydro.decode_routes(s.routes(0, c2.n)))
    assert ok, msg
    assert [st["evaluated"] for st in stats] == list(rev)
    assert [st["passed"] for st in stats] == list(rps)
    log(f"  |R|={ids.size} rescored={[st['rescored'] for st in stats]} escalated={[st['escalated'] for st in stats]}")
    s.close()


@pytest.mark.parametrize("order", [(0, 1, 2), (2, 1, 0), (1, 2, 0)])
def test_cnn_fixed_orders_exact_counts(c2, order):
    pol = hydro.make_policy("fixed", order=order, precision="bf16", wave=8192)
    s = hydro.Session(c2.specs(), pol, 64, c2.n)
    s.push(c2.device_frames(), c2.cfg.dtype, c2.pt.thresholds, c2.seg_len)
    ids, stats = s.finish()
    assert np.array_equal(ids, c2.expect)
    _, ev, ps = ho.short_circuit_eval(c2.P, order)
    assert [st["evaluated"] for st in stats] == list(ev)
    assert [st["passed"] for st in stats] == list(ps)
    s.close()


def test_cnn_static_cost_routes_are_reproducible(c2):
    pol = hydro.make_policy("score", precision="bf16", wave=2048, cost_source="static", log_routes=1)
    runs = []
    for _ in range(2):
        s = hydro.Session(c2.specs(), pol, 64, c2.n)
        s.push(c2.device_frames(), c2.cfg.dtype, c2.pt.thresholds, c2.seg_len)
        ids, stats = s.finish()
        assert np.array_equal(ids, c2.expect)
        runs.append(([st["evaluated"] for st in stats], s.routes(0, c2.n)))
        s.close()
    assert runs[0][0] == runs[1][0]
    assert np.array_equal(runs[0][1], runs[1][1])


@pytest.mark.parametrize("esc_cap", [None, "3"])
def test_cnn_fp64_tier_heavy(monkeypatch, esc_cap):
    """A huge FP32 band sends most decisions to the FP64 tier (layer-parallel path, and with a
    tiny cap the one-entry-per-block path too); ids must still equal the oracle's."""
    if esc_cap:
        monkeypatch.setenv("HYDRO_ESC_CAP", esc_cap)
    c = case(2, 1024)
    pol = hydro.make_policy("score", precision="fp32", tau32=0.5, wave=512)
    s = hydro.Session(c.specs(), pol, 64, c.n)
    s.push(c.device_frames(), c.cfg.dtype, c.pt.thresholds, c.seg_len)
    ids, stats = s.finish()
    esc = [st["escalated"] for st in stats]
    log(f"[gpu] fp64-heavy cap={esc_cap}: escalated={esc}")
    assert sum(esc) > 100
    assert np.array_equal(ids, c.expect)
    check_stats(stats, c.n, ids.size)
    s.close()


@pytest.mark.parametrize("prec", ["bf16", "fp32"])
def test_learned_router_ids_stats_replay(c2, prec):
    """Learned content-based routing (online-trained router MLP, control arm on score routing):
    routes differ, the answer set may not."""
    pol = hydro.make_policy("learned", precision=prec, wave=1024, log_routes=1, explore=0.1, seed=4242)
    s = hydro.Session(c2.specs(), pol, 64, c2.n)
    s.push(c2.device_frames(), c2.cfg.dtype, c2.pt.thresholds, c2.seg_len)
    ids, stats = s.finish()
    info = s.info()
    log(f"[gpu] learned prec={prec}: train_steps={info['train_steps']} active={info['learned_active']} "
        f"learned_routed={info['learned_routed']} stats_routed={info['stats_routed']} "
        f"evaluated={[st['evaluated'] for st in stats]}")
    assert np.array_equal(ids, c2.expect)
    check_stats(stats, c2.n, ids.size)
    ok, rev, rps, out, msg = ho.replay_route(c2.P, hydro.decode_routes(s.routes(0, c2.n)))
    assert ok, msg
    assert [st["evaluated"] for st in stats] == list(rev)
    assert info["train_steps"] > 0
    assert info["learned_routed"] + info["stats_routed"] == c2.n
    s.close()


@pytest.mark.parametrize("route", ["score", "learned"])
def test_graph_replays_match_eager(c2, route):
    """A push captured in a HIP graph and replayed several times, with eager work and
    synchronisation in between, gives the eager result every time."""
    eager = hydro.Session(c2.specs(), hydro.make_policy(route, precision="bf16", wave=2048), 64, c2.n)
    eager.push(c2.device_frames(), c2.cfg.dtype, c2.pt.thresholds, c2.seg_len)
    ids_e, st_e = eager.finish()
    eager.close()
    assert np.array_equal(ids_e, c2.expect)
    dev = c2.device_frames()
    s = hydro.Session(c2.specs(), hydro.make_policy(route, precision="bf16", wave=2048, use_graph=1), 64, c2.n)
    for rep in range(4):
        s.reset()
        s.push(dev, c2.cfg.dtype, c2.pt.thresholds, c2.seg_len)
        ids, stats = s.finish()
        torch.cuda.synchronize()
        _ = torch.ones(1024, device="cuda").sum().item()      # eager work between replays
        assert np.array_equal(ids, c2.expect), f"replay {rep}"
        check_stats(stats, c2.n, ids.size)
    s.close()


def test_cnn_calibrated_bands(c2):
    cfg = hs.workload(2)
    cal = torch.from_numpy(hs.make_frames(cfg, 0, 2048, data_seed=cfg.data_seed + 101)).cuda()
    s = hydro.Session(c2.specs(), hydro.make_policy("score", precision="bf16", wave=4096), 64, c2.n)
    tau, tau32 = s.calibrate(cal, "bf16", safety=2.0)
    log(f"[gpu] cnn calibrated tau={np.round(tau, 5).tolist()} tau32={tau32.tolist()}")
    assert np.all(tau > 0) and np.all(tau < 0.05) and np.all(tau32 < 1e-4)
    s.push(c2.device_frames(), c2.cfg.dtype, c2.pt.thresholds, c2.seg_len)
    ids, stats = s.finish()
    assert np.array_equal(ids, c2.expect)
    s.close()
