"""GPU checks of hydro_query_noalloc (the one-shot query that allocates no device memory and works
in the library's fixed per-GPU device array) against hydro_query, through the C ABI: ids equal to
the FP64 oracle's and to hydro_query's, statistics equal under deterministic routing, on two calls
in a row (the second smaller, so stale state from the first would show), plus its error paths."""
import numpy as np
import pytest

import hydro_synth as hs
from tests.gpu_util import case, check_stats, log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2403_14902_amd import hydro  # noqa: E402


def _both(c, n, start, pol, out_cap=None):
    dev = torch.from_numpy(c.frames[start - c.start:start - c.start + n]).cuda()
    ref_ids, ref_stats = hydro.query(dev, c.cfg.dtype, c.specs(), c.pt.thresholds, c.seg_len, pol, id_base=start)
    ids, stats = hydro.query_noalloc(dev, c.cfg.dtype, c.specs(), c.pt.thresholds, c.seg_len, pol,
                                     out_cap=n if out_cap is None else out_cap, id_base=start)
    return ref_ids, ref_stats, ids, stats


def _expect(c, n, start):
    lo = start - c.start
    from oracle import hydro_oracle as ho
    return ho.result_ids(c.P[lo:lo + n], id_base=start)


@pytest.mark.parametrize("wl,route,prec", [(2, "score", "bf16"), (1, "score", "fp32"), (1, "fixed", "bf16")])
def test_noalloc_equals_query_two_calls(wl, route, prec):
    c = case(wl, 2048 if wl == 1 else 6144)
    pol = hydro.make_policy(route, precision=prec, wave=512, cost_source="static")
    for n, start in ((c.n, c.start), (c.n // 3 + 5, c.start + 17)):
        log(f"[gpu] noalloc workload {wl} route={route} prec={prec} n={n} id_base={start}")
        ref_ids, ref_stats, ids, stats = _both(c, n, start, pol)
        exp = _expect(c, n, start)
        assert np.array_equal(ref_ids, exp)
        assert np.array_equal(ids, exp)
        check_stats(stats, n, ids.size)
        # static costs: routes are deterministic, so both entry points count the same evaluations
        for a, b in zip(stats, ref_stats):
            for key in ("evaluated", "passed", "rescored", "escalated"):
                assert a[key] == b[key], (key, a, b)


def test_noalloc_learned_router_and_explicit_bands():
    c = case(2, 6144)
    pol = hydro.make_policy("learned", precision="bf16", wave=512, tau=0.02, tau32=1e-5, explore=0.1)
    for n in (c.n, 2500):
        log(f"[gpu] noalloc learned n={n}")
        ref_ids, _, ids, stats = _both(c, n, c.start, pol)
        exp = _expect(c, n, c.start)
        assert np.array_equal(ref_ids, exp)
        assert np.array_equal(ids, exp)
        check_stats(stats, n, ids.size)


def test_noalloc_errors():
    c = case(1, 2048)
    dev = c.device_frames()
    pol = hydro.make_policy("score", precision="bf16", wave=512)
    exp = c.expect
    # output array too small: ECAPACITY and the size needed
    cm = (hydro.Model * c.cfg.k)(*[m.to_c() for m in c.specs()])
    fr = hydro._frames_struct(dev, c.cfg.dtype, 0)
    th = np.ascontiguousarray(c.pt.thresholds, dtype=np.float32)
    out = np.zeros(4, dtype=np.int64)
    n = hydro.C.c_int64()
    rc = hydro.lib().hydro_query_noalloc(hydro.C.byref(fr), cm, c.cfg.k, hydro._fp(th), th.shape[0], c.seg_len,
                                         hydro.C.byref(pol), out.ctypes.data_as(hydro.C.POINTER(hydro.C.c_int64)), 4,
                                         hydro.C.byref(n), None)
    assert rc == hydro.ECAPACITY and n.value == exp.size
    # host frames, graphs: refused
    with pytest.raises(hydro.HydroError):
        hydro.query_noalloc(c.frames, c.cfg.dtype, c.specs(), c.pt.thresholds, c.seg_len, pol, out_cap=c.n)
    with pytest.raises(hydro.HydroError):
        hydro.query_noalloc(dev, c.cfg.dtype, c.specs(), c.pt.thresholds, c.seg_len,
                            hydro.make_policy("score", use_graph=1), out_cap=c.n)
    # a model whose packed weights exceed the device array (12288-2048 MLP: ~250 MB of packed forms)
    big = hs.workload(3)
    d = big.models[5]
    w = hs.make_model(d)
    spec = hydro.ModelSpec.from_weights(w, 1)
    frames = torch.zeros((8, 64, 64, 3), dtype=torch.int16, device="cuda")
    with pytest.raises(hydro.HydroError) as e:
        hydro.query_noalloc(frames, "bf16", [spec], np.zeros((1, 1), np.float32), 8, pol, out_cap=8)
    assert e.value.code == hydro.ECAPACITY
    # the library is usable afterwards, and the array's previous contents do not leak into a call
    ids, _ = hydro.query_noalloc(dev, c.cfg.dtype, c.specs(), c.pt.thresholds, c.seg_len, pol, out_cap=c.n)
    assert np.array_equal(ids, exp)
