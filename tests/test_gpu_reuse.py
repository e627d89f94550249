"""Result reuse and reuse-aware routing (section 4.3, "Reuse-aware Routing"; the recurrent query of
UC2 that reuses the cached results of two earlier exploratory queries), through the C ABI.

Earlier queries on one session fill its device result cache; a later query takes the cached
decisions instead of evaluating them.  Checked against the oracle: the ids, the per-tuple visit
sequences (cached visits included: ``replay_route``), the exact split between evaluations and
cache hits for written orders, the threshold rule of cached decisions (``cached_decision``), and
that reuse-aware routing spends fewer UDF FLOPs than reuse-unaware cost routing on a workload
with a cached range."""
import numpy as np
import pytest

from oracle import hydro_oracle as ho
from tests.gpu_util import case, log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2403_14902_amd import hydro  # noqa: E402


N, A = 16384, 8192            # the query range and the cached prefix [0, A)


@pytest.fixture(scope="module")
def c2():
    return case(2, N)


def _query(s, c, lo, hi, thresholds=None):
    th = c.pt.thresholds if thresholds is None else thresholds
    dev = c.device_frames()
    s.reset()                 # a new query: statistics and results cleared, the cache kept
    s.push(dev[lo:hi].contiguous(), c.cfg.dtype, th, c.seg_len, id_base=lo)
    ids, stats = s.finish()
    return ids, stats


def _replay(s, c, lo, hi, P):
    routes = hydro.decode_routes(s.routes(lo, hi - lo))
    ok, ev, ps, out, msg = ho.replay_route(P[lo:hi], routes)
    assert ok, msg
    return ev, ps, routes


def _expensive_first(c):
    order = sorted(range(c.cfg.k), key=lambda j: -c.flops[j])
    return order


def test_written_order_reuses_every_cached_decision(c2):
    """Q1 evaluates the written order on [0, A); Q2 the same order on [0, N): every decision Q2
    needs on [0, A) is cached (exactly Q1's evaluations), and [A, N) is evaluated as usual."""
    c = c2
    order = _expensive_first(c)
    s = hydro.Session(c.specs(), hydro.make_policy("fixed", order=order, wave=2048, log_routes=1, reuse=1),
                      64, N)
    ids1, st1 = _query(s, c, 0, A)
    assert np.array_equal(ids1, ho.result_ids(c.P[:A]))
    assert all(x["cache_hits"] == 0 for x in st1)
    ids2, st2 = _query(s, c, 0, N)
    assert np.array_equal(ids2, c.expect)
    _, evA, _ = ho.short_circuit_eval(c.P[:A], order)
    _, evB, psB = ho.short_circuit_eval(c.P[A:], order)
    assert [x["cache_hits"] for x in st2] == list(evA)
    assert [x["evaluated"] for x in st2] == list(evB)
    assert [x["passed"] for x in st2] == list(psB)
    ev, _, _ = _replay(s, c, 0, N, c.P)
    assert list(ev) == [x["evaluated"] + x["cache_hits"] for x in st2]
    log(f"[gpu] reuse fixed {order}: hits {[x['cache_hits'] for x in st2]} evaluated {[x['evaluated'] for x in st2]}")
    # an emptied cache reuses nothing
    s.cache_clear()
    ids3, st3 = _query(s, c, 0, N)
    assert np.array_equal(ids3, c.expect)
    _, ev_all, _ = ho.short_circuit_eval(c.P, order)
    assert [x["evaluated"] for x in st3] == list(ev_all)
    assert all(x["cache_hits"] == 0 for x in st3)
    s.close()


def test_cached_decisions_follow_the_threshold_rule(c2):
    """Q2 raises the first predicate's thresholds: cached fails still decide (d <= theta0 <= theta),
    cached passes do not (d > theta0 says nothing about d > theta) and are evaluated again."""
    c = c2
    order = _expensive_first(c)
    j0 = order[0]
    s = hydro.Session(c.specs(), hydro.make_policy("fixed", order=order, wave=2048, log_routes=1, reuse=1),
                      64, N)
    _query(s, c, 0, A)
    th2 = c.pt.thresholds.copy()
    th2[:, j0] += 0.05
    ids, st = _query(s, c, 0, A, th2)
    theta_old = ho.tuple_thresholds(c.pt.thresholds, c.seg_len, np.arange(A))
    theta_new = ho.tuple_thresholds(th2, c.seg_len, np.arange(A))
    P2 = ho.decide(c.D[:A], theta_new)
    assert np.array_equal(ids, ho.result_ids(P2))
    dec = [ho.cached_decision(theta_old[t, j0], bool(c.P[t, j0]), theta_new[t, j0]) for t in range(A)]
    n_decided = sum(d for d, _ in dec)
    assert n_decided == int((~c.P[:A, j0]).sum())
    assert st[j0]["cache_hits"] == n_decided
    assert st[j0]["evaluated"] == A - n_decided
    _replay(s, c, 0, A, P2)
    s.close()


@pytest.mark.parametrize("route", ["cost", "score"])
def test_reuse_aware_routing_spends_fewer_flops(c2, route):
    """UC2's recurrent query: an exploratory query evaluates the most expensive predicate first on
    the middle range [L, H) (its decisions, and the others' on its survivors, are cached); the
    recurrent query then runs over [0, N) with static costs, once reuse-unaware (cached decisions
    are used when a tuple reaches them, the ranking ignores the cache) and once reuse-aware
    ((1 - hit rate) x cost per batch of 64).  Both return the oracle's ids with valid routes; on
    the cached range the reuse-aware one visits the expensive predicate first, the unaware one
    the cheapest, and the reuse-aware query spends fewer UDF FLOPs."""
    c = c2
    L, H = 4096, 12288
    order = _expensive_first(c)
    exp = order[0]
    flops = np.array(c.flops, dtype=np.float64)
    spent, first = {}, {}
    for reuse in (1, 2):
        s = hydro.Session(c.specs(), hydro.make_policy("fixed", order=order, wave=2048, log_routes=1, reuse=reuse,
                                                       cost_source="static"), 64, N)
        _query(s, c, L, H)                 # exploratory query
        s.set_route(route)
        ids, st = _query(s, c, 0, N)       # recurrent query
        assert np.array_equal(ids, c.expect)
        ev, _, routes = _replay(s, c, 0, N, c.P)
        assert list(ev) == [x["evaluated"] + x["cache_hits"] for x in st]
        spent[reuse] = float(np.dot([x["evaluated"] for x in st], flops))
        first[reuse] = float(np.mean([r[0] == exp for r in routes[L:H]]))
        log(f"[gpu] {route} reuse={reuse}: UDF GFLOP {spent[reuse] / 1e9:.3f} hits {[x['cache_hits'] for x in st]} "
            f"evaluated {[x['evaluated'] for x in st]}; cached range first visits the expensive predicate: {first[reuse]:.3f}")
        s.close()
    assert first[2] > 0.95 and first[1] < 0.05
    assert spent[2] < spent[1]


def test_reuse_policy_errors(c2):
    with pytest.raises(hydro.HydroError):
        hydro.Session(c2.specs(), hydro.make_policy("learned", reuse=1), 64, 1024)
    s = hydro.Session(c2.specs(), hydro.make_policy("score"), 64, 1024)
    with pytest.raises(hydro.HydroError):
        s.cache_clear()
    with pytest.raises(hydro.HydroError):
        s.set_route("learned")
    s.close()
