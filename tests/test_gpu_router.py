"""GPU checks of the router against the oracle's policy definitions (section 4.1), of query
state rules, of the learned router's training arithmetic and of pushes that straddle threshold
segments, through the C ABI."""
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
def c2():
    return case(2, 16384)


def admission_schedule(n, k, policy):
    """Per round: (lo, hi, warmup) of the tuples the engine admits, as include/hydro.h states
    (a warmup round of warmup_batches routing batches per predicate, then waves)."""
    adm, pos = [], 0
    if policy.route != hydro.ROUTE_FIXED and policy.warmup_batches > 0 and n > 0:
        w0 = min(n, policy.warmup_batches * k * policy.routing_batch)
        adm.append((0, w0, True))
        pos = w0
    while pos < n:
        w = min(n - pos, policy.wave)
        adm.append((pos, pos + w, False))
        pos += w
    return adm


def reconstruct_routes(P, orders, adm, routing_batch):
    """Every tuple's visit sequence if, in round r, each live tuple goes to the first predicate of
    orders[r] it has not visited (warmup tuples: routing batch b starts at predicate b mod K)."""
    n, k = P.shape
    seq = [[] for _ in range(n)]
    live = []
    per_round = []
    for r in range(len(orders)):
        if r < len(adm):
            lo, hi, warm = adm[r]
            live += [(t, warm) for t in range(lo, hi)]
        ev = np.zeros(k, dtype=np.int64)
        ps = np.zeros(k, dtype=np.int64)
        nxt = []
        for t, warm in live:
            if warm and not seq[t]:
                j = (t // routing_batch) % k
            else:
                j = next(x for x in orders[r] if x not in seq[t])
            seq[t].append(j)
            ev[j] += 1
            if P[t, j]:
                ps[j] += 1
                if len(seq[t]) < k:
                    nxt.append((t, False))
        per_round.append((ev, ps))
        live = nxt
    assert not live
    return seq, per_round


@pytest.mark.parametrize("route,name", [("score", ho.POLICY_SCORE), ("selectivity", ho.POLICY_SEL),
                                        ("cost", ho.POLICY_COST)])
def test_device_ranking_equals_oracle_policy_order(c2, route, name):
    """With ewma_alpha = 1 and static (FLOP) costs, every round's ranking must be the oracle's
    policy_order of the previous round's smoothed selectivity, and every tuple's route must be the
    one those rankings imply on the FP64 truth table."""
    pol = hydro.make_policy(route, precision="bf16", wave=2048, ewma_alpha=1.0, cost_source="static",
                            log_routes=1)
    s = hydro.Session(c2.specs(), pol, 64, c2.n)
    s.push(c2.device_frames(), c2.cfg.dtype, c2.pt.thresholds, c2.seg_len)
    ids, stats = s.finish()
    assert np.array_equal(ids, c2.expect)
    info = s.info()
    recs = s.round_log(0, info["rounds"])
    k = c2.cfg.k
    sel = np.zeros(k)
    checked = 0
    for r, rec in enumerate(recs):
        e = np.array(rec["folded_evaluated"], dtype=np.float64)
        p = np.array(rec["folded_passed"], dtype=np.float64)
        sel = np.where(e > 0, (p + 1.0) / (e + 2.0), sel)
        assert np.array_equal(np.array(rec["selectivity"]), sel), f"round {r}: estimates"
        seen = np.array([(rec["seen_mask"] >> j) & 1 for j in range(k)], dtype=bool)
        assert np.array_equal(seen, sel > 0), f"round {r}: seen mask"
        # static costs are the model FLOPs, taken at a predicate's first fold (0 before it)
        assert np.allclose(np.array(rec["cost"])[seen], np.array(c2.flops)[seen], rtol=1e-6), f"round {r}: cost"
        assert not np.any(np.array(rec["cost"])[~seen]), f"round {r}: cost of an unseen predicate"
        if rec["seen_mask"] == (1 << k) - 1:
            want = ho.policy_order(name, np.array(rec["cost"]), sel)
            assert rec["order"] == want, f"round {r}: device {rec['order']} oracle {want}"
            checked += 1
    assert checked >= len(recs) - 2
    # routes implied by those rankings on the truth table, against the device's route log
    adm = admission_schedule(c2.n, k, pol)
    seq, per_round = reconstruct_routes(c2.P, [rec["order"] for rec in recs], adm, pol.routing_batch)
    got = hydro.decode_routes(s.routes(0, c2.n))
    bad = [t for t in range(c2.n) if got[t] != seq[t]]
    assert not bad, f"{len(bad)} routes differ, first tuple {bad[0]}: {got[bad[0]]} vs {seq[bad[0]]}"
    for r in range(1, len(recs)):
        assert recs[r]["folded_evaluated"] == list(per_round[r - 1][0]), f"round {r}: folded counts"
        assert recs[r]["folded_passed"] == list(per_round[r - 1][1])
    log(f"[gpu] {route}: {len(recs)} rounds, rankings {[rec['order'] for rec in recs]}")
    s.close()


def test_learned_router_short_later_pushes(c2):
    """Pushes shorter than the rounds the learned router needs before it routes: from the round of
    the query in which it can route, every round computes its tuples' keys, whichever push they
    belong to (no decision is taken on keys of an earlier round)."""
    pol = hydro.make_policy("learned", precision="bf16", wave=2048, log_routes=1, explore=0.1)
    s = hydro.Session(c2.specs(), pol, 64, 2048)
    dev = c2.device_frames()
    for lo in range(0, c2.n, 2048):
        s.push(dev[lo:lo + 2048], c2.cfg.dtype, c2.pt.thresholds, c2.seg_len, id_base=lo)
    ids, stats = s.finish()
    info = s.info()
    log(f"[gpu] learned, 8 pushes of 2048: steps={info['train_steps']} learned_routed={info['learned_routed']} "
        f"stale={info['learned_stale']} active={info['learned_active']}")
    assert np.array_equal(ids, c2.expect)
    check_stats(stats, c2.n, ids.size)
    assert info["learned_stale"] == 0
    assert info["learned_routed"] > 0
    assert info["learned_routed"] + info["stats_routed"] == c2.n
    s.close()


def test_learned_router_spans_drift_segments():
    """The 524,288-tuple drifting workload's predicates under the learned router, on a prefix that
    crosses a threshold-segment boundary (ids 61,440 .. 69,631)."""
    c = case(4, 8192, start=61440)
    pol = hydro.make_policy("learned", precision="bf16", wave=1024, log_routes=1, explore=0.1)
    s = hydro.Session(c.specs(), pol, 64, c.n)
    s.push(c.device_frames(), c.cfg.dtype, c.pt.thresholds, c.seg_len, id_base=c.start)
    ids, stats = s.finish()
    info = s.info()
    log(f"[gpu] c4 learned across segments: |R|={ids.size} learned_routed={info['learned_routed']}")
    assert np.array_equal(ids, c.expect)
    check_stats(stats, c.n, ids.size)
    ok, rev, rps, out, msg = ho.replay_route(c.P, hydro.decode_routes(s.routes(0, c.n)))
    assert ok, msg
    assert [st["evaluated"] for st in stats] == list(rev)
    assert info["learned_stale"] == 0
    s.close()


def test_pushes_straddle_threshold_segments():
    """Blocks of 5,000 tuples with id_base > 0 whose ranges cross segment boundaries (segments of
    8,192): each tuple's threshold row comes from its global id."""
    c = case(2, 12000, start=6000)
    s = hydro.Session(c.specs(), hydro.make_policy("score", precision="bf16", wave=1500), 64, 5000)
    dev = c.device_frames()
    for lo in range(0, c.n, 5000):
        s.push(dev[lo:lo + 5000], c.cfg.dtype, c.pt.thresholds, c.seg_len, id_base=c.start + lo)
    ids, stats = s.finish()
    assert np.array_equal(ids, c.expect)
    check_stats(stats, c.n, ids.size)
    s.close()


def test_query_state_rules(c2):
    """logits / calibrate between a push and finish are refused (they would discard the open
    query); after finish they run, and the next query is exact."""
    dev = c2.device_frames()
    s = hydro.Session(c2.specs(), hydro.make_policy("score", precision="bf16", wave=2048), 64, 8192)
    s.push(dev[:8192], c2.cfg.dtype, c2.pt.thresholds, c2.seg_len)
    with pytest.raises(hydro.HydroError) as e:
        s.calibrate(dev[:512], c2.cfg.dtype, 2.0)
    assert e.value.code == hydro.ESTATE
    with pytest.raises(hydro.HydroError) as e:
        s.logits(0, 0, dev[:64], c2.cfg.dtype)
    assert e.value.code == hydro.ESTATE
    with pytest.raises(hydro.HydroError) as e:
        s.set_order([0, 1, 2])
    assert e.value.code == hydro.ESTATE
    s.push(dev[8192:], c2.cfg.dtype, c2.pt.thresholds, c2.seg_len, id_base=8192)
    ids, stats = s.finish()
    assert np.array_equal(ids, c2.expect)
    s.calibrate(dev[:512], c2.cfg.dtype, 2.0)
    s.push(dev[:8192], c2.cfg.dtype, c2.pt.thresholds, c2.seg_len)
    ids, _ = s.finish()
    assert np.array_equal(ids, c2.expect[c2.expect < 8192])
    s.close()


def test_recalibration_reaches_captured_graphs(c2):
    """A push captured in a HIP graph, then new (wider) bands: the next graphed push re-scores
    exactly as an eager session with those bands (FIXED order: routes are deterministic)."""
    dev = c2.device_frames()
    cal = dev[:1024]
    pol_e = hydro.make_policy("fixed", order=[0, 1, 2], precision="bf16", wave=4096)
    eager = hydro.Session(c2.specs(), pol_e, 64, c2.n)
    eager.calibrate(cal, c2.cfg.dtype, 20.0)
    eager.push(dev, c2.cfg.dtype, c2.pt.thresholds, c2.seg_len)
    ids_e, st_e = eager.finish()
    eager.close()
    pol_g = hydro.make_policy("fixed", order=[0, 1, 2], precision="bf16", wave=4096, use_graph=1)
    g = hydro.Session(c2.specs(), pol_g, 64, c2.n)
    g.calibrate(cal, c2.cfg.dtype, 2.0)
    g.push(dev, c2.cfg.dtype, c2.pt.thresholds, c2.seg_len)
    ids_a, st_a = g.finish()
    g.calibrate(cal, c2.cfg.dtype, 20.0)
    for rep in range(2):
        g.reset()
        g.push(dev, c2.cfg.dtype, c2.pt.thresholds, c2.seg_len)
        ids_b, st_b = g.finish()
        assert np.array_equal(ids_b, c2.expect)
        assert [x["rescored"] for x in st_b] == [x["rescored"] for x in st_e], f"replay {rep}"
    log(f"[gpu] rescored narrow {[x['rescored'] for x in st_a]} wide {[x['rescored'] for x in st_b]}")
    assert sum(x["rescored"] for x in st_b) > sum(x["rescored"] for x in st_a)
    assert np.array_equal(ids_a, c2.expect) and np.array_equal(ids_e, c2.expect)
    g.close()


def test_every_fixed_order_on_six_mlps():
    """All 720 written orders of the six-MLP workload on a 256-tuple prefix: the same ids, and
    the exact short-circuit counts of each order (one session, the order changed between queries)."""
    c = case(3, 256)
    pol = hydro.make_policy("fixed", precision="bf16", wave=256, tau=0.2, tau32=1e-4)
    s = hydro.Session(c.specs(), pol, 64, c.n)
    dev = c.device_frames()
    for i, order in enumerate(itertools.permutations(range(6))):
        s.set_order(order)
        s.reset()
        s.push(dev, c.cfg.dtype, c.pt.thresholds, c.seg_len)
        ids, stats = s.finish()
        assert np.array_equal(ids, c.expect), f"order {order}"
        _, ev, ps = ho.short_circuit_eval(c.P, order)
        assert [st["evaluated"] for st in stats] == list(ev), f"order {order}"
        assert [st["passed"] for st in stats] == list(ps), f"order {order}"
    log(f"[gpu] 720 fixed orders: |R| = {c.expect.size}")
    s.close()


def test_allocation_failures_unwind(monkeypatch):
    """The n-th device allocation of a session fails (HYDRO_FAULT_ALLOC_AFTER = n): creation or the
    first push reports ENOMEM and releases what it took; the same process then runs a query."""
    c = case(1, 512)
    codes = []
    for n_ok in range(0, 40, 3):
        monkeypatch.setenv("HYDRO_FAULT_ALLOC_AFTER", str(n_ok))
        try:
            s = hydro.Session(c.specs(), hydro.make_policy("learned", precision="bf16", wave=256), 32, c.n)
        except hydro.HydroError as e:
            codes.append(e.code)
            continue
        try:
            s.push(c.device_frames(), c.cfg.dtype, c.pt.thresholds, c.seg_len)
            ids, _ = s.finish()
            assert np.array_equal(ids, c.expect)
            codes.append(0)
        except hydro.HydroError as e:
            codes.append(e.code)
        s.close()
    monkeypatch.delenv("HYDRO_FAULT_ALLOC_AFTER")
    log(f"[gpu] allocation-failure codes: {codes}")
    assert hydro.ENOMEM in codes
    assert set(codes) <= {0, hydro.ENOMEM}
    s = hydro.Session(c.specs(), hydro.make_policy("score", precision="bf16", wave=256), 32, c.n)
    s.push(c.device_frames(), c.cfg.dtype, c.pt.thresholds, c.seg_len)
    ids, _ = s.finish()
    assert np.array_equal(ids, c.expect)
    s.close()


# ---------------------------------------------------------------- learned router training step
def _bf16_bits_to_f64(b):
    return (b.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def adam_bce_reference(params, m, v, feats, pred, rej, steps_done, lr, k):
    """Two Adam steps of masked binary cross-entropy in fp64 (newest window first), written from the
    definitions: h = ReLU(F W1 + b1), o = h W2 + b2, loss = mean_b BCE(sigmoid(o[b, pred_b]), y_b)."""
    W1 = params[:192 * 64].reshape(192, 64).astype(np.float64)
    b1 = params[192 * 64:192 * 64 + 64].astype(np.float64)
    W2 = params[192 * 64 + 64:192 * 64 + 64 + 512].reshape(64, 8).astype(np.float64)
    b2 = params[-8:].astype(np.float64)
    P = [W1, b1, W2, b2]
    M = [x.astype(np.float64) for x in np.split(m, [192 * 64, 192 * 64 + 64, 192 * 64 + 64 + 512])]
    V = [x.astype(np.float64) for x in np.split(v, [192 * 64, 192 * 64 + 64, 192 * 64 + 64 + 512])]
    M[0] = M[0].reshape(192, 64); V[0] = V[0].reshape(192, 64)
    M[2] = M[2].reshape(64, 8); V[2] = V[2].reshape(64, 8)
    F = _bf16_bits_to_f64(feats)
    t = steps_done
    for lo in (64, 0):
        W1, b1, W2, b2 = P
        f = F[lo:lo + 64]
        kk = pred[lo:lo + 64]
        y = rej[lo:lo + 64].astype(np.float64)
        pre = f @ W1 + b1
        h = np.maximum(pre, 0.0)
        o = (h * W2[:, kk].T).sum(axis=1) + b2[kk]
        dO = (1.0 / (1.0 + np.exp(-o)) - y) / 64.0
        gW2 = np.zeros_like(W2)
        gb2 = np.zeros_like(b2)
        for b in range(64):
            gW2[:, kk[b]] += h[b] * dO[b]
            gb2[kk[b]] += dO[b]
        dH = np.where(pre > 0, dO[:, None] * W2[:, kk].T, 0.0)
        grads = [f.T @ dH, dH.sum(axis=0), gW2, gb2]
        t += 1
        c1, c2 = 1.0 / (1.0 - 0.9 ** t), 1.0 / (1.0 - 0.999 ** t)
        for i in range(4):
            M[i] = 0.9 * M[i] + 0.1 * grads[i]
            V[i] = 0.999 * V[i] + 0.001 * grads[i] ** 2
            P[i] = P[i] - lr * (M[i] * c1) / (np.sqrt(V[i] * c2) + 1e-8)
    flat = lambda L: np.concatenate([x.ravel() for x in L])
    return flat(P), flat(M), flat(V)


@pytest.mark.parametrize("steps_done", [0, 9])
def test_router_training_step_matches_fp64_adam(steps_done):
    rng = np.random.default_rng(5 + steps_done)
    k = 3
    n = hydro.ROUTER_NPARAM
    params = np.zeros(n, dtype=np.float32)
    params[:192 * 64] = rng.standard_normal(192 * 64) * np.sqrt(2 / 192)
    params[192 * 64:192 * 64 + 64] = rng.uniform(-0.1, 0.1, 64)
    params[192 * 64 + 64:192 * 64 + 64 + 512] = rng.standard_normal(512) * 0.2
    params[-8:] = rng.uniform(-0.1, 0.1, 8)
    m = (rng.standard_normal(n) * 1e-3).astype(np.float32) if steps_done else np.zeros(n, np.float32)
    v = (rng.random(n) * 1e-5).astype(np.float32) if steps_done else np.zeros(n, np.float32)
    feats = hs.f64_to_bf16_bits(rng.uniform(-2, 2, (128, 192)))
    pred = rng.integers(0, k, 128).astype(np.int32)
    rej = (rng.random(128) < 0.4).astype(np.uint8)
    lr = 3e-3
    gp, gm, gv = hydro.router_train_debug(k, feats, pred, rej, params, m, v, steps_done, lr)
    rp, rm, rv = adam_bce_reference(params, m, v, feats, pred, rej, steps_done, lr, k)
    # fp32 kernel arithmetic against fp64: the parameter change is at most lr per step and Adam's
    # normalised step amplifies gradient rounding only where v is tiny, so compare the updates
    err = np.abs((gp - params) - (rp - params))
    m_err = np.abs(gm - rm).max() / max(1e-12, np.abs(rm).max())
    log(f"[gpu] router training step (t0={steps_done}): |dparam err| max {err.max():.3e} p99.9 "
        f"{np.quantile(err, 0.999):.3e} (max |dparam| {np.abs(rp - params).max():.3e}), rel m err {m_err:.3e}")
    # a wrong sign or a dropped term moves most parameters by about lr; fp32 rounding does not
    assert np.quantile(err, 0.999) <= 1e-3 * lr
    assert err.max() <= 0.05 * lr
    assert m_err <= 1e-4
    # a planted sign error in the gradient would move the parameters the other way
    assert np.sign(gp - params)[np.abs(rp - params) > 0.5 * lr].tolist() == \
        np.sign(rp - params)[np.abs(rp - params) > 0.5 * lr].tolist()
