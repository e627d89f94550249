"""The C-ABI library loads, exports every function include/hydro.h declares, and rejects bad
arguments before touching the device.  CPU only (no compute calls)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2403_14902_amd import hydro

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "hydro.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hydro_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    L = hydro.lib()
    names = declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(L, n), f"{n} declared in hydro.h but not exported"
    assert set(hydro.EXPORTED) == set(names)


def test_version_and_no_error():
    L = hydro.lib()
    assert L.hydro_version().startswith(b"hydro-gfx950")


def test_policy_defaults():
    p = hydro.make_policy()
    assert p.route == hydro.ROUTE_SCORE and p.routing_batch == 64 and p.wave == 8192
    # bands default to automatic (<= 0): measured on the session's first push
    assert p.precision == hydro.PREC_BF16 and p.tau == 0.0 and p.tau32 == 0.0
    assert list(p.order)[:4] == [0, 1, 2, 3]


def _mlp_spec(mask=1, hidden=128, hw=8):
    rng = np.random.default_rng(0)
    d = hw * hw * 3
    t = {"W1": rng.standard_normal((d, hidden)), "b1": np.zeros(hidden), "W2": rng.standard_normal((hidden, 10)),
         "b2": np.zeros(10)}
    return hydro.ModelSpec("mlp", hw, mask, t, hidden=hidden)


def _create(models, policy, hw=8, max_push=64):
    cm = (hydro.Model * max(1, len(models)))(*[m.to_c() for m in models])
    h = C.c_void_p()
    rc = hydro.lib().hydro_session_create(cm if models else None, len(models), C.byref(policy) if policy else None,
                                          hw, hw, max_push, C.byref(h))
    return rc, hydro.lib().hydro_last_error().decode()


def test_create_rejects_bad_arguments():
    pol = hydro.make_policy()
    m = _mlp_spec()
    assert _create([], pol)[0] == hydro.EINVAL                     # K = 0 / NULL models
    assert _create([m] * 9, pol)[0] == hydro.EUNSUPPORTED           # K above 8
    assert _create([m], None)[0] == hydro.EINVAL                    # NULL policy
    assert _create([m], pol, max_push=0)[0] == hydro.EINVAL
    assert _create([m], pol, hw=16)[0] == hydro.EINVAL              # model shape != frame shape
    bad = _mlp_spec(mask=1 << 10)
    rc, msg = _create([bad], pol)
    assert rc == hydro.EINVAL and "class_mask" in msg
    odd = _mlp_spec(hidden=100)
    assert _create([odd], pol)[0] == hydro.EUNSUPPORTED
    fixed = hydro.make_policy("fixed", order=[0, 0])
    rc, msg = _create([m, m], fixed)
    assert rc == hydro.EINVAL and "permutation" in msg
    assert _create([m], hydro.make_policy(ewma_alpha=0.0))[0] == hydro.EINVAL
    assert _create([m], hydro.make_policy(routing_batch=0))[0] == hydro.EINVAL


def test_cnn_shape_support_is_checked():
    pol = hydro.make_policy()
    rng = np.random.default_rng(1)
    widths = (16, 32, 40)                     # not multiples of 16
    convs, cin = [], 3
    for co in widths:
        convs.append((rng.standard_normal((co, cin, 3, 3)), np.zeros(co)))
        cin = co
    spec = hydro.ModelSpec("cnn", 64, 1, {"convs": convs, "Wfc": np.zeros((cin, 10)), "bfc": np.zeros(10)},
                           widths=widths)
    rc, msg = _create([spec], pol, hw=64)
    assert rc == hydro.EUNSUPPORTED


def test_null_arguments_elsewhere():
    L = hydro.lib()
    assert L.hydro_session_push(None, None, None, 1, 1) == hydro.EINVAL
    assert L.hydro_session_finish(None, None, None, None) == hydro.EINVAL
    assert L.hydro_session_destroy(None) == hydro.EINVAL
    assert L.hydro_query(None, None, 0, None, 1, 1, None, None, None, None) == hydro.EINVAL
    assert L.hydro_last_error()


@pytest.mark.skipif(os.path.exists("/dev/kfd"), reason="checks the no-device error path only")
def test_valid_create_without_device_reports_device_error():
    rc, msg = _create([_mlp_spec()], hydro.make_policy())
    assert rc == hydro.EDEVICE and msg


def test_rescore3_rules():
    """The three-product re-score tier is opt-in, follows a BF16 first pass only, and only for
    4-layer 128x128 CNN predicates (checked before any device work)."""
    assert hydro.make_policy().rescore3 == 0
    m = _mlp_spec()
    assert _create([m], hydro.make_policy(rescore3=2))[0] == hydro.EINVAL
    for prec in ("fp32", "fp8"):
        assert _create([m], hydro.make_policy(precision=prec, rescore3=1))[0] == hydro.EUNSUPPORTED
    rc, msg = _create([m], hydro.make_policy(precision="bf16", rescore3=1))
    assert rc == hydro.EUNSUPPORTED and "three-product" in msg
