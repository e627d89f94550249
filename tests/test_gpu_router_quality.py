"""What the learned router (content-based routing, section 2.2) has learned: after a query with
route = LEARNED, its parameters are read back and its rejection probabilities are evaluated on
held-out frames (same ids and drift segments, another data seed) against the oracle's decisions:
binary cross-entropy against the base-rate predictor, and ROC AUC, per predicate.  The judge's
arm accounting (UDF FLOPs per finished tuple of the learned and control arms) is reported beside
it.  The figures are logged; the assertions are the exact ids and the consistency of what is
reported."""
import numpy as np
import pytest
from scipy.stats import rankdata

import hydro_synth as hs
from oracle import hydro_oracle as ho
from tests.gpu_util import case, check_stats, log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2403_14902_amd import hydro  # noqa: E402


def pooled_features(frames, dtype):
    """The router's input: the frame mean-pooled to 8x8x3 in (y, x, channel) order, normalised,
    rounded to bf16 (round to nearest even)."""
    x = ho.frames_to_f64(frames, dtype)
    n, h, w, _ = x.shape
    b = h // 8
    f = ho.normalize(x.reshape(n, 8, b, 8, b, 3).mean(axis=(2, 4)).reshape(n, 192)).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def router_logits(params, f, k):
    W1 = params[:192 * 64].reshape(192, 64).astype(np.float64)
    b1 = params[192 * 64:192 * 64 + 64].astype(np.float64)
    W2 = params[192 * 64 + 64:192 * 64 + 64 + 512].reshape(64, 8).astype(np.float64)
    b2 = params[-8:].astype(np.float64)
    return (np.maximum(f @ W1 + b1, 0.0) @ W2 + b2)[:, :k]


def bce(p, y):
    p = np.clip(p, 1e-7, 1 - 1e-7)
    return float(-(y * np.log(p) + (1 - y) * np.log(1 - p)).mean())


def auc(score, y):
    """Probability that a rejected tuple scores above an accepted one (ties count half)."""
    pos = y.sum()
    neg = y.size - pos
    if pos == 0 or neg == 0:
        return float("nan")
    r = rankdata(score)
    return float((r[y == 1].sum() - pos * (pos + 1) / 2) / (pos * neg))


@pytest.mark.parametrize("wl,n,wave,held", [(2, 32768, 2048, 4096), (4, 32768, 2048, 4096), (5, 4096, 256, 1024)])
def test_learned_router_held_out_quality(wl, n, wave, held):
    c = case(wl, n)
    pol = hydro.make_policy("learned", precision="bf16", wave=wave, explore=0.2)
    s = hydro.Session(c.specs(), pol, c.cfg.hw, c.n)
    s.push(c.device_frames(), c.cfg.dtype, c.pt.thresholds, c.seg_len)
    ids, stats = s.finish()
    assert np.array_equal(ids, c.expect)
    check_stats(stats, c.n, ids.size)
    info = s.info()
    params = s.router_params()
    s.close()
    assert np.all(np.isfinite(params))
    k = c.cfg.k
    # held-out frames: the last `held` ids of the query's range, drawn with another data seed
    lo = n - held
    fr = hs.make_frames(c.cfg, lo, held, data_seed=c.cfg.data_seed + 101)
    P, D = ho.truth_table(fr, c.cfg.dtype, c.weights, c.pt.class_masks, c.pt.thresholds, c.seg_len, id_base=lo)[:2]
    z = router_logits(params, pooled_features(fr, c.cfg.dtype), k)
    prob = 1.0 / (1.0 + np.exp(-z))
    log(f"[gpu] c{wl} learned router: steps={info['train_steps']} active={info['learned_active']} "
        f"learned_routed={info['learned_routed']} stats_routed={info['stats_routed']}")
    for j in range(k):
        y = (~P[:, j]).astype(np.float64)           # 1 = predicate j rejects
        rate = y.mean()
        base = bce(np.full_like(y, rate), y)
        log(f"  predicate {j}: reject rate {rate:.3f}  held-out BCE {bce(prob[:, j], y):.4f} "
            f"(base rate {base:.4f})  AUC {auc(z[:, j], y):.3f}")
    if info["arm_tuples"][0] > 0 and info["arm_tuples"][1] > 0:
        per = [info["arm_flops"][a] / info["arm_tuples"][a] / 1e6 for a in range(2)]
        log(f"  MFLOP per finished tuple: control {per[0]:.3f}  learned {per[1]:.3f}  "
            f"(tuples {int(info['arm_tuples'][0])} / {int(info['arm_tuples'][1])})")
        assert info["arm_tuples"][0] + info["arm_tuples"][1] <= c.n
