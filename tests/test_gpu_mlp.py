"""GPU parity of the MLP path (small MLP workload: 2,048 frames 32x32x3 fp32, two MLP
3072-256-10 predicates) against the FP64 oracle, through the C ABI."""
import itertools

import numpy as np
import pytest

import hydro_synth as hs
from tests.gpu_util import case, check_stats, log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2403_14902_amd import hydro  # noqa: E402
from oracle import hydro_oracle as ho  # noqa: E402


@pytest.fixture(scope="module")
def c1():
    return case(1, 2048, logits=True)


def _session(c, policy, max_push=None):
    return hydro.Session(c.specs(), policy, c.cfg.hw, max_push or c.n)


# tolerances: a few times the largest errors measured on these frames (fp32 5.7e-6, bf16 3.7e-2 over
# 12,288-term dot products, fp64 1e-14); the kernels are deterministic
@pytest.mark.parametrize("prec,tier,tol", [("fp32", 0, 3e-5), ("bf16", 0, 0.08), ("bf16", 1, 3e-5), ("fp32", 2, 1e-12)])
def test_logits_each_tier_vs_oracle(c1, prec, tier, tol):
    log(f"[gpu] logits prec={prec} tier={tier}")
    s = _session(c1, hydro.make_policy("score", precision=prec))
    dev = c1.device_frames()
    for k in range(c1.cfg.k):
        z = s.logits(k, tier, dev, c1.cfg.dtype)
        err = np.abs(z - c1.Z[k]).max()
        log(f"  predicate {k}: max |z - z64| = {err:.3e}")
        assert err <= tol
    s.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("order", list(itertools.permutations(range(2))))
def test_fixed_order_ids_and_exact_counts(c1, prec, order):
    log(f"[gpu] fixed order {order} prec={prec}")
    pol = hydro.make_policy("fixed", order=order, precision=prec, wave=512, log_routes=1)
    s = _session(c1, pol)
    s.push(c1.device_frames(), c1.cfg.dtype, c1.pt.thresholds, c1.seg_len)
    ids, stats = s.finish()
    assert np.array_equal(ids, c1.expect)
    _, ev, ps = ho.short_circuit_eval(c1.P, order)
    assert [st["evaluated"] for st in stats] == list(ev)
    assert [st["passed"] for st in stats] == list(ps)
    routes = hydro.decode_routes(s.routes(0, c1.n))
    ok, rev, rps, out, msg = ho.replay_route(c1.P, routes)
    assert ok, msg
    assert np.array_equal(out, c1.expect)
    s.close()


@pytest.mark.parametrize("route", ["score", "selectivity", "cost"])
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_adaptive_policies_ids_stats_and_replay(c1, route, prec):
    log(f"[gpu] route={route} prec={prec}")
    pol = hydro.make_policy(route, precision=prec, wave=256, log_routes=1)
    s = _session(c1, pol)
    s.push(c1.device_frames(), c1.cfg.dtype, c1.pt.thresholds, c1.seg_len)
    ids, stats = s.finish()
    assert np.array_equal(ids, c1.expect)
    check_stats(stats, c1.n, ids.size)
    routes = hydro.decode_routes(s.routes(0, c1.n))
    ok, rev, rps, out, msg = ho.replay_route(c1.P, routes)
    assert ok, msg
    assert [st["evaluated"] for st in stats] == list(rev)
    assert [st["passed"] for st in stats] == list(rps)
    info = s.info()
    assert info["n_result"] == ids.size and info["rounds"] > 0
    s.close()


def test_one_shot_query_and_host_frames(c1):
    pol = hydro.make_policy("score", precision="bf16", wave=1000)
    ids, stats = hydro.query(c1.device_frames(), c1.cfg.dtype, c1.specs(), c1.pt.thresholds, c1.seg_len, pol)
    assert np.array_equal(ids, c1.expect)
    ids2, _ = hydro.query(c1.frames, c1.cfg.dtype, c1.specs(), c1.pt.thresholds, c1.seg_len, pol)
    assert np.array_equal(ids2, c1.expect)


@pytest.mark.parametrize("n", [0, 1, 63, 65, 1000])
def test_ragged_and_empty_pushes(c1, n):
    pol = hydro.make_policy("score", precision="bf16", wave=100)
    s = _session(c1, pol, max_push=2048)
    if n > 0:
        s.push(c1.device_frames()[:n].contiguous(), c1.cfg.dtype, c1.pt.thresholds, c1.seg_len)
    else:
        s.push(c1.device_frames()[:0], c1.cfg.dtype, c1.pt.thresholds, c1.seg_len)
    ids, stats = s.finish()
    assert np.array_equal(ids, c1.expect[c1.expect < n])
    s.close()


def test_several_pushes_one_query(c1):
    pol = hydro.make_policy("score", precision="bf16", wave=300)
    s = _session(c1, pol, max_push=700)
    dev = c1.device_frames()
    for lo in range(0, c1.n, 700):
        hi = min(c1.n, lo + 700)
        s.push(dev[lo:hi].contiguous(), c1.cfg.dtype, c1.pt.thresholds, c1.seg_len, id_base=lo)
    ids, stats = s.finish()
    assert np.array_equal(ids, c1.expect)
    check_stats(stats, c1.n, ids.size)
    # the session can run a second query after reset
    s.reset()
    s.push(dev[:700].contiguous(), c1.cfg.dtype, c1.pt.thresholds, c1.seg_len)
    ids, _ = s.finish()
    assert np.array_equal(ids, c1.expect[c1.expect < 700])
    s.close()


def test_threshold_extremes(c1):
    pol = hydro.make_policy("score", precision="bf16", wave=512)
    inf = np.full_like(c1.pt.thresholds, np.inf)
    ids, stats = hydro.query(c1.device_frames(), c1.cfg.dtype, c1.specs(), inf, c1.seg_len, pol)
    assert ids.size == 0
    ids, stats = hydro.query(c1.device_frames(), c1.cfg.dtype, c1.specs(), -inf, c1.seg_len, pol)
    assert np.array_equal(ids, np.arange(c1.n))


def test_capacity_error(c1):
    s = _session(c1, hydro.make_policy(), max_push=100)
    with pytest.raises(hydro.HydroError) as e:
        s.push(c1.device_frames()[:200].contiguous(), c1.cfg.dtype, c1.pt.thresholds, c1.seg_len)
    assert e.value.code == hydro.ECAPACITY
    s.close()


@pytest.mark.parametrize("esc_cap", [None, "5"])
def test_mlp_fp64_tier_heavy(c1, monkeypatch, esc_cap):
    if esc_cap:
        monkeypatch.setenv("HYDRO_ESC_CAP", esc_cap)
    pol = hydro.make_policy("score", precision="bf16", tau=1.0, tau32=0.5, wave=512)
    s = _session(c1, pol)
    s.push(c1.device_frames(), c1.cfg.dtype, c1.pt.thresholds, c1.seg_len)
    ids, stats = s.finish()
    esc = [st["escalated"] for st in stats]
    log(f"[gpu] mlp fp64-heavy cap={esc_cap}: escalated={esc}")
    assert sum(esc) > 100
    assert np.array_equal(ids, c1.expect)
    s.close()


def test_mlp_graph_replays(c1):
    s = _session(c1, hydro.make_policy("score", precision="bf16", wave=256, use_graph=1))
    dev = c1.device_frames()
    for rep in range(3):
        s.reset()
        s.push(dev, c1.cfg.dtype, c1.pt.thresholds, c1.seg_len)
        ids, stats = s.finish()
        _ = torch.ones(64, device="cuda").sum().item()
        assert np.array_equal(ids, c1.expect), f"replay {rep}"
    s.close()


@pytest.mark.parametrize("tile", ["0", "1", "2", "3"])
@pytest.mark.parametrize("prec", ["bf16", "fp32"])
def test_mlp_every_tile_shape(c1, monkeypatch, tile, prec):
    monkeypatch.setenv("HYDRO_MLP_TILE", tile)
    pol = hydro.make_policy("score", precision=prec, tau=0.1, wave=512)
    s = _session(c1, pol)
    z = s.logits(0, 0, c1.device_frames(), c1.cfg.dtype)
    assert np.abs(z - c1.Z[0]).max() <= (0.08 if prec == "bf16" else 2e-4)
    s.push(c1.device_frames(), c1.cfg.dtype, c1.pt.thresholds, c1.seg_len)
    ids, stats = s.finish()
    assert np.array_equal(ids, c1.expect)
    s.close()


def test_mlp_autotuned_session(c1, tmp_path, monkeypatch):
    monkeypatch.setenv("HYDRO_TUNE_CACHE", str(tmp_path / "tune.json"))
    for _ in range(2):      # second session reads the cache
        pol = hydro.make_policy("score", precision="bf16", tau=0.1, wave=512, autotune=1)
        s = _session(c1, pol)
        s.push(c1.device_frames(), c1.cfg.dtype, c1.pt.thresholds, c1.seg_len)
        ids, stats = s.finish()
        assert np.array_equal(ids, c1.expect)
        s.close()
    import json
    d = json.loads((tmp_path / "tune.json").read_text())
    assert any(k.startswith("gfx950/bf16/f32/D3072/h256") for k in d)


def test_calibration_in_blocks_of_max_push(c1):
    """Calibrating on more frames than a session's push capacity takes them in blocks: the bands
    equal those of a session that holds every frame in one block, and the query stays exact."""
    dev = c1.device_frames()
    pol = hydro.make_policy("score", precision="bf16")
    big = _session(c1, pol)
    t_big, t32_big = big.calibrate(dev[:1500], c1.cfg.dtype, 2.0)
    big.close()
    small = _session(c1, pol, max_push=512)
    t_small, t32_small = small.calibrate(dev[:1500], c1.cfg.dtype, 2.0)
    log(f"[gpu] blocked calibration tau={t_small.tolist()} tau32={t32_small.tolist()}")
    assert np.array_equal(t_big, t_small) and np.array_equal(t32_big, t32_small)
    for lo in range(0, c1.n, 512):
        small.push(dev[lo:lo + 512], c1.cfg.dtype, c1.pt.thresholds, c1.seg_len, id_base=lo)
    ids, stats = small.finish()
    assert np.array_equal(ids, c1.expect)
    check_stats(stats, c1.n, ids.size)
    small.close()


@pytest.mark.parametrize("prec", ["bf16", "fp32"])
def test_mlp_split_k_forced(c1, monkeypatch, prec):
    """Every GEMM launch split along K (the last part of each tile adds the parts in order): the
    ids stay exact and the logits match the unsplit ones to rounding."""
    pol = hydro.make_policy("score", precision=prec, wave=512)
    dev = c1.device_frames()
    monkeypatch.setenv("HYDRO_SPLITK_BELOW", "0")          # never split
    s0 = _session(c1, pol)
    z0 = s0.logits(0, 0, dev[:700], c1.cfg.dtype)
    s0.close()
    monkeypatch.setenv("HYDRO_SPLITK_BELOW", "1000000")
    s = _session(c1, pol)
    z1 = s.logits(0, 0, dev[:700], c1.cfg.dtype)
    log(f"[gpu] split-K {prec}: max logit change {np.abs(z1 - z0).max():.3g}")
    # only the fp32 summation order differs (3,072-term dot products)
    assert np.allclose(z1, z0, rtol=0, atol=1e-3 if prec == "bf16" else 2e-4)
    s.push(dev, c1.cfg.dtype, c1.pt.thresholds, c1.seg_len)
    ids, stats = s.finish()
    assert np.array_equal(ids, c1.expect)
    check_stats(stats, c1.n, ids.size)
    s.close()


@pytest.mark.parametrize("hidden", [128, 384])
def test_bf16_mlp_three_k_blocks(hidden):
    """Two bf16 MLPs on 8x8x3 bf16 frames (192 inputs: the direct-to-LDS GEMM's smallest k
    extent, three 64-element k-blocks, the whole ring filled by its prologue), grouped in one
    launch: ids and written-order counts against the oracle, bands measured by the session."""
    rng = np.random.default_rng(hidden)
    n = 3000
    frames = hs.f64_to_bf16_bits(rng.random((n, 8, 8, 3)))
    models = [hs.make_model(hs.ModelDesc(arch="mlp", seed=900 + hidden, d_in=192, hidden=hidden)),
              hs.make_model(hs.ModelDesc(arch="mlp", seed=901, d_in=192, hidden=128))]
    masks = [0b0000011111, 0b1111100000]
    D = np.stack([ho.predicate_margin(ho.model_logits(m, frames, "bf16"), k) for m, k in zip(models, masks)], axis=1)
    th = np.zeros((1, 2), dtype=np.float32)
    for j in range(2):                     # between two distinct margins near the median
        u = np.unique(D[:, j])
        m = np.searchsorted(u, np.median(D[:, j]))
        th[0, j] = np.float32((u[m - 1] + u[m]) / 2.0)
    theta = ho.tuple_thresholds(th, n, np.arange(n))
    assert np.abs(D - theta).min() > 1e-9
    P = ho.decide(D, theta)
    specs = [hydro.ModelSpec.from_weights(m, k) for m, k in zip(models, masks)]
    log(f"[gpu] bf16 MLP 192-{hidden}-10 and 192-128-10 on 8x8 frames: pass rates {P.mean(axis=0).round(3).tolist()}")
    s = hydro.Session(specs, hydro.make_policy("fixed", order=[0, 1], precision="bf16", wave=1024), 8, n)
    s.push(torch.from_numpy(frames).cuda(), "bf16", th, n)
    ids, stats = s.finish()
    assert np.array_equal(ids, ho.result_ids(P))
    _, ev, ps = ho.short_circuit_eval(P, [0, 1])
    assert [st["evaluated"] for st in stats] == list(ev)
    assert [st["passed"] for st in stats] == list(ps)
    s.close()
