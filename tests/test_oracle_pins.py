"""Pins for the FP64 oracle: exact arithmetic, an independent library, closed
forms, decision special cases, order invariance, statistics invariants and the
paper's printed policy vectors.  CPU only."""
import itertools
import json
import os
from fractions import Fraction

import numpy as np
import pytest
import torch

import hydro_synth as hs
import oracle
from oracle import hydro_oracle as ho
from tests import bruteforce as bf

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- helpers
def tiny_mlp(seed, d, h):
    return hs.make_model(hs.ModelDesc(arch="mlp", seed=seed, d_in=d, hidden=h))


def tiny_cnn(seed, hw, widths):
    return hs.make_model(hs.ModelDesc(arch="cnn", seed=seed, in_hw=hw, widths=tuple(widths)))


def bf16_frames(rng, n, hw):
    return hs.f64_to_bf16_bits(rng.random((n, hw, hw, 3)))


def exact_frame(fr64):
    return [[[Fraction(float(fr64[y, x, c])) for c in range(3)] for x in range(fr64.shape[1])]
            for y in range(fr64.shape[0])]


# ---------------------------------------------------------------- O1-O4: exact brute force
def test_mlp_matches_exact_rationals():
    rng = np.random.default_rng(11)
    m = tiny_mlp(7, 48, 8)
    fr = bf16_frames(rng, 64, 4)
    z = ho.model_logits(m, fr, "bf16")
    x64 = ho.frames_to_f64(fr, "bf16")
    t = m.tensors
    for i in range(64):
        ze = bf.mlp_exact(exact_frame(x64[i]), t["W1"], t["b1"], t["W2"], t["b2"])
        for c in range(10):
            assert abs(float(Fraction(z[i, c]) - ze[c])) <= 1e-12 * (1 + abs(float(ze[c])))


def test_cnn_matches_exact_rationals():
    rng = np.random.default_rng(12)
    m = tiny_cnn(8, 8, [4, 8])
    fr = bf16_frames(rng, 64, 8)
    z = ho.model_logits(m, fr, "bf16")
    x64 = ho.frames_to_f64(fr, "bf16")
    t = m.tensors
    for i in range(64):
        ze = bf.cnn_exact(exact_frame(x64[i]), t["convs"], t["Wfc"], t["bfc"])
        for c in range(10):
            assert abs(float(Fraction(z[i, c]) - ze[c])) <= 1e-12 * (1 + abs(float(ze[c])))


def test_u8_frames_exact_rationals():
    """uint8 v means v/255: compare with the exact rational v/255."""
    rng = np.random.default_rng(13)
    m = tiny_cnn(9, 8, [4, 8])
    fr = rng.integers(0, 256, size=(16, 8, 8, 3), dtype=np.uint8)
    z = ho.model_logits(m, fr, "u8")
    t = m.tensors
    for i in range(16):
        fe = [[[Fraction(int(fr[i, y, x, c]), 255) for c in range(3)] for x in range(8)] for y in range(8)]
        ze = bf.cnn_exact(fe, t["convs"], t["Wfc"], t["bfc"])
        for c in range(10):
            assert abs(float(Fraction(z[i, c]) - ze[c])) <= 1e-12 * (1 + abs(float(ze[c])))


def test_decisions_match_exact_margins():
    """Margins and strict decisions agree with exact rationals (thresholds off-tie)."""
    rng = np.random.default_rng(14)
    m = tiny_cnn(10, 8, [4, 8])
    fr = bf16_frames(rng, 48, 8)
    z = ho.model_logits(m, fr, "bf16")
    x64 = ho.frames_to_f64(fr, "bf16")
    for mask in (0b1, 0b1000000001, 0b0011110000):
        d = ho.predicate_margin(z, mask)
        theta = float(np.float32(np.median(d)))
        got = ho.decide(d, theta)
        for i in range(48):
            ze = bf.cnn_exact(exact_frame(x64[i]), m.tensors["convs"], m.tensors["Wfc"], m.tensors["bfc"])
            de, kind = bf.margin_exact(ze, mask)
            assert kind == "finite"
            assert abs(float(de) - d[i]) <= 1e-12
            if abs(float(de - Fraction(theta))) > 1e-9:
                assert got[i] == (de > Fraction(theta))


# ---------------------------------------------------------------- O3/O4: independent library
def test_mlp_vs_torch_linear_on_small_workload():
    cfg = hs.workload(1)
    fr = hs.make_frames(cfg, 0, 512)
    for desc in cfg.models:
        m = hs.make_model(desc)
        z = ho.model_logits(m, fr, cfg.dtype)
        x = (torch.from_numpy(fr.astype(np.float64)).reshape(512, -1) - 0.5) * 4
        t = {k: torch.from_numpy(v.astype(np.float64)) for k, v in m.tensors.items()}
        h = torch.relu(torch.nn.functional.linear(x, t["W1"].T, t["b1"]))
        zt = torch.nn.functional.linear(h, t["W2"].T, t["b2"]).numpy()
        assert np.abs(z - zt).max() <= 1e-12 * max(1.0, np.abs(zt).max())


def _torch_cnn(m, x64):
    x = torch.from_numpy(x64).permute(0, 3, 1, 2)
    x = (x - 0.5) * 4
    for w, b in m.tensors["convs"]:
        x = torch.relu(torch.nn.functional.conv2d(x, torch.from_numpy(w.astype(np.float64)),
                                                  torch.from_numpy(b.astype(np.float64)),
                                                  stride=2, padding=1))
    g = x.mean(dim=(2, 3))
    return (g @ torch.from_numpy(m.tensors["Wfc"].astype(np.float64))
            + torch.from_numpy(m.tensors["bfc"].astype(np.float64))).numpy()


@pytest.mark.parametrize("wl,n", [(2, 64), (5, 8)])
def test_cnn_vs_torch_conv2d_on_workload_prefix(wl, n):
    cfg = hs.workload(wl)
    fr = hs.make_frames(cfg, 0, n)
    x64 = ho.frames_to_f64(fr, cfg.dtype)
    for desc in cfg.models[:2]:
        m = hs.make_model(desc)
        z = ho.model_logits(m, fr, cfg.dtype)
        zt = _torch_cnn(m, x64)
        assert np.abs(z - zt).max() <= 1e-12 * max(1.0, np.abs(zt).max())


# ---------------------------------------------------------------- closed forms
def test_zero_weights_give_bias():
    m = tiny_cnn(3, 8, [4, 8])
    for w, b in m.tensors["convs"]:
        w[...] = 0
    m.tensors["Wfc"][...] = 0
    fr = bf16_frames(np.random.default_rng(1), 5, 8)
    z = ho.model_logits(m, fr, "bf16")
    assert np.array_equal(z, np.tile(m.tensors["bfc"].astype(np.float64), (5, 1)))
    mm = tiny_mlp(4, 48, 8)
    mm.tensors["W1"][...] = 0
    mm.tensors["W2"][...] = 0
    z = ho.model_logits(mm, bf16_frames(np.random.default_rng(2), 3, 4), "bf16")
    assert np.array_equal(z, np.tile(mm.tensors["b2"].astype(np.float64), (3, 1)))


def test_delta_kernel_subsamples_even_pixels():
    """Centre tap 1 on one channel, zero bias: output = normalised input at (2i, 2j), clipped at 0."""
    rng = np.random.default_rng(3)
    a = rng.standard_normal((2, 8, 8, 3))
    w = np.zeros((3, 3, 3, 3))
    for c in range(3):
        w[c, c, 1, 1] = 1.0
    y = ho.conv3x3_s2_relu(a, w, np.zeros(3))
    assert np.array_equal(y, np.maximum(a[:, ::2, ::2, :], 0))


def test_corner_taps_read_the_zero_border():
    """Tap (0,0) reads input (2i-1, 2j-1): zero for i=0 or j=0, else the odd pixel."""
    a = np.arange(1, 2 * 6 * 6 + 1, dtype=np.float64).reshape(1, 6, 6, 2)
    w = np.zeros((2, 2, 3, 3))
    w[0, 0, 0, 0] = 1.0
    w[1, 1, 2, 2] = 1.0           # tap (2,2) reads (2i+1, 2j+1)
    y = ho.conv3x3_s2_relu(a, w, np.zeros(2))
    exp0 = np.zeros((3, 3))
    exp0[1:, 1:] = a[0, 1:4:2, 1:4:2, 0]
    assert np.array_equal(y[0, :, :, 0], exp0)
    assert np.array_equal(y[0, :, :, 1], a[0, 1::2, 1::2, 1])


def test_constant_image_constant_pool():
    """A frame of raw value 0.5 normalises to exactly zero (so does the padding):
    every conv output is ReLU(bias), the pool is ReLU(bias), z = ReLU(b) Wfc + bfc."""
    m = tiny_cnn(5, 8, [4])
    fr = np.full((1, 8, 8, 3), 0.5, dtype=np.float32)           # normalises to exactly 0
    z = ho.model_logits(m, fr, "f32")
    b0 = np.maximum(m.tensors["convs"][0][1].astype(np.float64), 0)
    exp = b0 @ m.tensors["Wfc"].astype(np.float64) + m.tensors["bfc"]
    assert np.allclose(z[0], exp, rtol=0, atol=1e-15)


def test_block_selector_mlp_gives_block_sums():
    """W1 selects pixel blocks, W2 = identity on the first 8 hidden units."""
    d, h = 48, 10
    m = tiny_mlp(6, d, h)
    W1 = np.zeros((d, h), dtype=np.float32)
    for j in range(h):
        W1[(j * 4):(j * 4 + 4), j] = 1.0 if j < 10 else 0.0
    m.tensors["W1"][...] = W1
    m.tensors["b1"][...] = 100.0                    # keeps ReLU inactive
    m.tensors["W2"][...] = np.eye(h, 10, dtype=np.float32)
    m.tensors["b2"][...] = -100.0
    fr = np.random.default_rng(4).random((3, 4, 4, 3)).astype(np.float32)
    z = ho.model_logits(m, fr, "f32")
    xn = (fr.astype(np.float64).reshape(3, -1) - 0.5) * 4
    exp = np.stack([xn[:, j * 4:j * 4 + 4].sum(axis=1) for j in range(10)], axis=1)
    assert np.allclose(z, exp, rtol=0, atol=1e-12)


# ---------------------------------------------------------------- O5 decision special cases
def test_decision_special_cases():
    z = np.random.default_rng(5).standard_normal((100, 10))
    d = ho.predicate_margin(z, 0b101)
    assert not ho.decide(d, np.inf).any()
    assert ho.decide(d, -np.inf).all()
    assert ho.decide(ho.predicate_margin(z, 0x3FF), 1e30).all()       # S = all classes
    assert not ho.decide(ho.predicate_margin(z, 0), -1e30).any()      # S = empty
    for mask in (0b1, 0b110, 0b1111100000):
        inside = np.array([(mask >> c) & 1 for c in range(10)], dtype=bool)
        assert np.array_equal(ho.decide(ho.predicate_margin(z, mask), 0.0), inside[np.argmax(z, axis=1)])


def test_tie_is_rejected():
    z = np.zeros((1, 10))
    z[0, 3] = z[0, 4] = 1.0
    assert not ho.decide(ho.predicate_margin(z, 1 << 3), 0.0)[0]


# ---------------------------------------------------------------- O6/O7 order invariance, stats
@pytest.fixture(scope="module")
def small_truth():
    cfg = hs.workload(1)
    fr = hs.make_frames(cfg)
    pt = hs.load_predicates(cfg)
    models = [hs.make_model(d) for d in cfg.models]
    P, D = ho.truth_table(fr, cfg.dtype, models, pt.class_masks, pt.thresholds, cfg.n // cfg.n_seg)
    return cfg, P, D, pt


def test_every_order_gives_the_same_result(small_truth):
    cfg, P, D, pt = small_truth
    R = ho.result_ids(P)
    for order in itertools.permutations(range(P.shape[1])):
        r, ev, ps = ho.short_circuit_eval(P, order)
        assert np.array_equal(r, R)


def test_every_order_random_truth_tables():
    rng = np.random.default_rng(6)
    for k in range(1, 7):
        P = rng.random((500, k)) < rng.uniform(0.2, 0.9, size=k)
        R = ho.result_ids(P)
        brute = np.array([t for t in range(500) if all(P[t, j] for j in range(k))], dtype=np.int64)
        assert np.array_equal(R, brute)
        for order in itertools.permutations(range(k)):
            r, ev, ps = ho.short_circuit_eval(P, order)
            assert np.array_equal(r, R)
            assert ho.stats_invariants(ev, ps, 500, R.size) == []
            assert ev[order[0]] == 500
            for a, b in zip(order[:-1], order[1:]):
                assert ev[b] == ps[a]


def test_small_workload_selectivities_near_targets(small_truth):
    cfg, P, D, pt = small_truth
    sel = P.mean(axis=0)
    assert np.all(np.abs(sel - np.array(cfg.targets[0])) < 0.06), sel


def test_small_workload_no_near_ties(small_truth):
    cfg, P, D, pt = small_truth
    assert ho.near_tie_gap(D, pt.thresholds, cfg.n // cfg.n_seg) > 1e-9


def test_replay_route_accepts_valid_and_flags_invalid():
    P = np.array([[1, 1, 0], [1, 1, 1], [0, 1, 1]], dtype=bool)
    ok, ev, ps, out, msg = ho.replay_route(P, [[0, 2], [2, 1, 0], [0]])
    assert ok and list(out) == [1]
    assert list(ev) == [3, 1, 2] and list(ps) == [2, 1, 1]
    assert not ho.replay_route(P, [[2, 0], [0, 1, 2], [0]])[0]          # continues after a fail
    assert not ho.replay_route(P, [[0, 1, 2], [0, 1], [0]])[0]          # stops after a pass
    assert not ho.replay_route(P, [[0, 0], [0, 1, 2], [0]])[0]          # revisits


def test_stats_invariants_catch_bad_counts():
    assert ho.stats_invariants([10, 6], [6, 3], 10, 3) == []
    assert ho.stats_invariants([10, 6], [6, 4], 10, 3) != []


# ---------------------------------------------------------------- paper policy vectors
@pytest.mark.parametrize("case", ["uc1_profile", "table1_case1", "table1_case2", "worked_example"])
def test_policy_first_choice_matches_paper(case):
    with open(os.path.join(GOLD, "paper_policy_vectors.json")) as f:
        v = json.load(f)[case]
    cost = v.get("cost_ms", v.get("cost"))
    sel = v["selectivity"]
    for pol, name in ((ho.POLICY_COST, "cost"), (ho.POLICY_SCORE, "score"), (ho.POLICY_SEL, "selectivity")):
        assert ho.policy_order(pol, cost, sel)[0] == v["first"][name], (case, name)
    if "score" in v:
        assert np.allclose(ho.policy_keys(ho.POLICY_SCORE, cost, sel), v["score"], rtol=1e-12)


def test_uc1_scores_match_printed_statistics():
    k = ho.policy_keys(ho.POLICY_SCORE, [35.11, 1.98], [0.254, 0.633])
    assert round(k[0], 2) == 47.06 and round(k[1], 2) == 5.40


def test_score_key_edge_cases():
    k = ho.policy_keys(ho.POLICY_SCORE, [1.0, 1.0, 5.0], [1.0, 0.0, 0.5])
    assert k[0] == np.inf and k[1] == 1.0 and k[2] == 10.0
    assert ho.policy_order(ho.POLICY_COST, [2.0, 2.0, 1.0], [0, 0, 0]) == [2, 0, 1]   # ties -> lower index
    assert np.allclose(ho.smoothed_selectivity([0, 5], [0, 8]), [0.5, 0.6])


# ---------------------------------------------------------------- planted mistakes are caught
def _mutant_results(monkeypatch, mutate):
    rng = np.random.default_rng(21)
    m = tiny_cnn(22, 8, [4, 8])
    fr = bf16_frames(rng, 4, 8)
    x64 = ho.frames_to_f64(fr, "bf16")
    exact = [bf.cnn_exact(exact_frame(x64[i]), m.tensors["convs"], m.tensors["Wfc"], m.tensors["bfc"])
             for i in range(4)]
    mutate(monkeypatch)
    z = ho.model_logits(m, fr, "bf16")
    return max(abs(float(Fraction(z[i, c]) - exact[i][c])) for i in range(4) for c in range(10))


@pytest.mark.parametrize("name", ["no_bias", "pad_offset", "kernel_transposed", "no_normalise", "sum_pool"])
def test_brute_force_catches_planted_oracle_mistakes(monkeypatch, name):
    orig_conv = ho.conv3x3_s2_relu

    def mutate(mp):
        if name == "no_bias":
            mp.setattr(ho, "conv3x3_s2_relu", lambda a, w, b: orig_conv(a, w, 0 * b))
        elif name == "pad_offset":
            def conv(a, w, b):
                a2 = np.zeros_like(a)
                a2[:, :-1, :-1] = a[:, 1:, 1:]
                return orig_conv(a2, w, b)
            mp.setattr(ho, "conv3x3_s2_relu", conv)
        elif name == "kernel_transposed":
            mp.setattr(ho, "conv3x3_s2_relu", lambda a, w, b: orig_conv(a, np.swapaxes(w, 2, 3), b))
        elif name == "no_normalise":
            mp.setattr(ho, "normalize", lambda x: x)
        elif name == "sum_pool":
            def cnn(t, xn):
                a = xn
                for w, b in t["convs"]:
                    a = ho.conv3x3_s2_relu(a, w, b)
                return a.sum(axis=(1, 2)) @ t["Wfc"] + t["bfc"]
            mp.setattr(ho, "cnn_logits", cnn)

    assert _mutant_results(monkeypatch, mutate) > 1e-6


# ---------------------------------------------------------------- input generator sanity
def test_bf16_rounding_is_nearest_even():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -9, 0.0], dtype=np.float64)
    bits = hs.f64_to_bf16_bits(vals)
    back = ho.frames_to_f64(bits, "bf16")
    assert list(back) == [1.0, 1.0, 1.0 + 2 ** -6, 1.0, 0.0]


def test_frame_chunks_regenerate_independently():
    cfg = hs.workload(2)
    a = hs.make_frames(cfg, 1000, 100)
    b = hs.make_frames(cfg, 0, 1100)[1000:]
    assert np.array_equal(a, b)


# ---------------------------------------------------------------- threshold rows, static orders, bound
def test_tuple_thresholds_hand_pin():
    """theta row of a tuple = its segment, min(id // seg_len, n_seg - 1), from the global id."""
    th = np.array([[1.0, 10.0], [2.0, 20.0], [3.0, 30.0]], dtype=np.float32)
    ids = np.array([0, 4, 5, 9, 10, 14, 15, 100])
    got = ho.tuple_thresholds(th, 5, ids)
    want = np.array([[1, 10], [1, 10], [2, 20], [2, 20], [3, 30], [3, 30], [3, 30], [3, 30]], dtype=np.float64)
    assert np.array_equal(got, want)
    # fp32 thresholds are used as stored (widened exactly)
    odd = np.array([[0.1]], dtype=np.float32)
    assert ho.tuple_thresholds(odd, 7, np.array([3]))[0, 0] == float(np.float32(0.1))


def test_truth_table_uses_global_ids_for_segments():
    """Zero weights make every margin the same constant d0 (= max over S of b - max outside S);
    thresholds just below / above d0 per segment fix which tuples pass, by hand, for a block that
    starts at id_base = 7 and crosses two segment boundaries (segments of 4 ids)."""
    m = tiny_mlp(3, 12, 128)
    t = m.tensors
    t["W1"][:] = 0
    t["W2"][:] = 0
    t["b2"][:] = np.arange(10, dtype=np.float32) * 0.25        # z = b2, class 9 largest
    mask = 1 << 9                                              # S = {9}: d0 = 2.25 - 2.0 = 0.25
    th = np.array([[0.3], [0.2], [0.3], [0.2]], dtype=np.float32)   # segment 1 and 3 pass
    frames = np.zeros((10, 2, 2, 3), dtype=np.float32)
    P, D = ho.truth_table(frames, "f32", [m], [mask], th, seg_len=4, id_base=7)
    assert np.allclose(D[:, 0], 0.25)
    # ids 7..16: segments 1,2,2,2,2,3,3,3,3,3 (id 16 is segment 4 -> clamped to the last row, 3)
    assert P[:, 0].tolist() == [True, False, False, False, False, True, True, True, True, True]
    assert ho.result_ids(P, id_base=7).tolist() == [7, 12, 13, 14, 15, 16]


HAND_P = np.array([[1, 1, 1], [1, 0, 1], [1, 0, 0], [1, 0, 1], [1, 1, 0], [1, 0, 0]], dtype=bool)
HAND_F = [1.0, 4.0, 2.0]


def test_best_static_order_hand_pin():
    # totals by hand: (0,1,2) 34, (0,2,1) 30, (1,0,2) 30, (1,2,0) 29, (2,0,1) 27, (2,1,0) 25
    order, total = ho.best_static_order(HAND_P, HAND_F)
    assert order == [2, 1, 0] and total == 25.0
    ev, _ = ho.fixed_order_counts(HAND_P, (0, 1, 2))
    assert list(ev) == [6, 6, 2] and float(np.dot(ev, HAND_F)) == 34.0


def test_clairvoyant_flops_hand_pin():
    # failing tuples pay their cheapest failing predicate (t1 4, t2 2, t3 4, t4 2, t5 2), the
    # passing tuple t0 pays all three (7)
    assert ho.clairvoyant_flops(HAND_P, HAND_F) == 21.0


def test_bounds_ordered_on_random_tables():
    """clairvoyant <= best static <= every static order, and all >= |R| * sum(F)."""
    rng = np.random.default_rng(3)
    for trial in range(30):
        k = int(rng.integers(2, 5))
        P = rng.random((int(rng.integers(1, 40)), k)) < rng.uniform(0.2, 0.9, k)
        f = rng.uniform(1, 10, k)
        best_o, best = ho.best_static_order(P, f)
        cl = ho.clairvoyant_flops(P, f)
        floor = P.all(axis=1).sum() * f.sum()
        assert floor - 1e-9 <= cl <= best + 1e-9
        for order in itertools.permutations(range(k)):
            ev, _ = ho.fixed_order_counts(P, order)
            assert best <= float(np.dot(ev, f)) + 1e-9


def test_reuse_aware_cost_closed_forms():
    """(1 - hit rate) * cost: a fully cached predicate costs nothing, an uncached one its full
    cost, and the estimate is linear in between (section 4.3)."""
    c = np.array([35.11, 1.98, 7.0])
    assert np.array_equal(ho.reuse_aware_cost([0.0, 0.0, 0.0], c), c)
    assert np.array_equal(ho.reuse_aware_cost([1.0, 1.0, 1.0], c), np.zeros(3))
    assert np.allclose(ho.reuse_aware_cost([0.25, 0.5, 0.75], c), [0.75 * 35.11, 0.5 * 1.98, 0.25 * 7.0], rtol=0, atol=1e-15)


def test_reuse_aware_order_prefers_cached_expensive_predicate():
    """The paper's UC2 situation: an expensive detector whose results are cached for the batch goes
    before a cheaper uncached one; without cache hits the cheaper one goes first."""
    cost, sel = [35.11, 1.98], [0.254, 0.633]
    assert ho.reuse_aware_order(ho.POLICY_COST, cost, sel, [0.0, 0.0]) == [1, 0]
    assert ho.reuse_aware_order(ho.POLICY_COST, cost, sel, [1.0, 0.0]) == [0, 1]
    assert ho.reuse_aware_order(ho.POLICY_SCORE, cost, sel, [0.0, 0.0]) == [1, 0]
    assert ho.reuse_aware_order(ho.POLICY_SCORE, cost, sel, [0.99, 0.0]) == [0, 1]
    # the selectivity policy ignores costs, hence the cache
    assert ho.reuse_aware_order(ho.POLICY_SEL, cost, sel, [0.0, 1.0]) == [0, 1]


def test_cached_decision_brute_force():
    """A cached outcome decides a new threshold exactly when every margin consistent with it gives
    the same decision there (brute force over a grid of margins)."""
    grid = np.linspace(-2.0, 2.0, 401)
    rng = np.random.default_rng(3)
    for _ in range(300):
        tc, t = (float(x) for x in rng.choice(grid[50:-50], 2))
        for passed in (True, False):
            consistent = grid[grid > tc] if passed else grid[grid <= tc]
            outs = set(bool(d > t) for d in consistent)
            decided, p = ho.cached_decision(tc, passed, t)
            assert decided == (len(outs) == 1), (tc, passed, t)
            if decided:
                assert {p} == outs


def test_color_fraction_hand_pin():
    """A 2x2 frame with one pixel inside the box on every channel, one outside on one channel,
    one exactly on the box's edges (inside: the bounds are inclusive), one far outside."""
    px = np.array([[[0.5, 0.5, 0.5], [0.5, 0.9, 0.5]],
                   [[0.25, 0.75, 0.25], [0.0, 0.0, 0.0]]], dtype=np.float32)[None]
    d = ho.color_fraction(px, "f32", [0.25, 0.25, 0.25], [0.75, 0.75, 0.75])
    assert d.tolist() == [0.5]
    # uint8 values are v / 255: 64 / 255 is just above 0.25, 63 / 255 just below
    u8 = np.array([[[[64, 64, 64], [63, 64, 64]]]], dtype=np.uint8)
    assert ho.color_fraction(u8, "u8", [0.25] * 3, [1.0] * 3).tolist() == [0.5]


def test_concurrent_makespan_paper_example():
    """Section 4.1's example: colour classifier (CPU, cost 1, selectivity 0.6) and breed classifier
    (GPU, cost 2, selectivity 0.1) running concurrently on 10 tuples: breed first takes 20 time
    units, colour first 14.  The pass patterns are the reading taken here of the figure (the one
    breed pass is not the last tuple; the six colour passes are tuples 2, 3, 5, 6, 8, 10)."""
    P = np.zeros((10, 2), dtype=bool)           # column 0: colour, column 1: breed
    P[[1, 2, 4, 5, 7, 9], 0] = True
    P[[1, 2, 4, 5, 7, 9][:1], 1] = True
    assert ho.concurrent_makespan([1, 0], P, [1.0, 2.0]) == 20.0
    assert ho.concurrent_makespan([0, 1], P, [1.0, 2.0]) == 14.0
    # the policies: selectivity and score put breed first, cost puts colour first
    cost, sel = [1.0, 2.0], [0.6, 0.1]
    assert ho.policy_first(ho.POLICY_SEL, cost, sel) == 1
    assert ho.policy_first(ho.POLICY_SCORE, cost, sel) == 1
    assert ho.policy_first(ho.POLICY_COST, cost, sel) == 0


def test_concurrent_makespan_brute_force_small():
    """Against an explicit event list on a tiny case with a tuple arriving while the second worker
    is busy (FIFO waits) and one arriving while it is idle."""
    P = np.array([[1, 1], [0, 1], [1, 1], [1, 0]], dtype=bool)
    # first stage (cost 3): ends 3, 6, 9, 12; passes tuples 0, 2, 3 -> arrive 3, 9, 12
    # second stage (cost 5): 3 -> 8, 9 -> 14, 14 -> 19
    assert ho.concurrent_makespan([0, 1], P, [3.0, 5.0]) == 19.0


def test_ab_sweep_cost_policy_never_worse():
    """The A/B sweep of section 4.1 on the concurrent model: A costs 10, B 20 (separate resources),
    selectivity of A from 0.1 to 0.9, of B 0.1, 0.5 and 0.9, 2,000 tuples with independent
    outcomes: the cost-driven first choice is never slower than the score- or selectivity-driven
    one (up to one tuple's pipeline fill), and the selectivity-driven one is the slowest on
    average."""
    rng = np.random.default_rng(17)
    cost = [10.0, 20.0]
    tot = {ho.POLICY_COST: 0.0, ho.POLICY_SCORE: 0.0, ho.POLICY_SEL: 0.0}
    for sb in (0.1, 0.5, 0.9):
        for sa in np.arange(0.1, 0.91, 0.1):
            P = np.stack([rng.random(2000) < sa, rng.random(2000) < sb], axis=1)
            sel = [P[:, 0].mean(), P[:, 1].mean()]
            ms = {}
            for pol in tot:
                first = ho.policy_first(pol, cost, sel)
                ms[pol] = ho.concurrent_makespan([first, 1 - first], P, cost)
                tot[pol] += ms[pol]
            assert ms[ho.POLICY_COST] <= min(ms[ho.POLICY_SCORE], ms[ho.POLICY_SEL]) + max(cost)
    assert tot[ho.POLICY_SEL] >= tot[ho.POLICY_SCORE] >= tot[ho.POLICY_COST]


def test_crop_logits_whole_frame_and_torch():
    """A crop covering the whole frame gives the frame's logits; a smaller crop equals torch
    float64 conv2d (stride 2, padding 1) on the cropped, normalised image."""
    torch = pytest.importorskip("torch")
    cfg = hs.workload(2)
    fr = hs.make_frames(cfg, 0, 3)
    m = hs.make_model(cfg.models[0])
    full = np.array([[0, 0, 64, 64]] * 3)
    assert np.allclose(ho.crop_logits(m, fr, "bf16", full), ho.model_logits(m, fr, "bf16"), rtol=0, atol=1e-12)
    crops = np.array([[5, 7, 19, 33], [0, 60, 64, 4], [30, 2, 1, 1]])
    z = ho.crop_logits(m, fr, "bf16", crops)
    for i, (y0, x0, h, w) in enumerate(crops):
        x = torch.from_numpy(ho.normalize(ho.frames_to_f64(fr[i:i + 1, y0:y0 + h, x0:x0 + w], "bf16"))).permute(0, 3, 1, 2)
        for wt, b in m.tensors["convs"]:
            x = torch.relu(torch.nn.functional.conv2d(x, torch.from_numpy(wt.astype(np.float64)),
                                                      torch.from_numpy(b.astype(np.float64)), stride=2, padding=1))
        g = x.mean(dim=(2, 3))
        zt = (g @ torch.from_numpy(m.tensors["Wfc"].astype(np.float64)) + torch.from_numpy(m.tensors["bfc"].astype(np.float64)))
        assert np.allclose(z[i], zt.numpy()[0], rtol=0, atol=1e-12)
