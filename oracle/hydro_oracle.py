"""FP64 reference evaluation of a conjunction of ML-UDF predicates (TEST INFRASTRUCTURE).

Only tests, the smoke check and the benchmark's CPU-baseline leg use this
module.  It is deliberately plain: every predicate is evaluated on every tuple,
in the conjunction's written order, in float64, with numpy matmuls as the only
library primitive.  No blocking, fusion or reordering beyond chunking the
tuple axis (tuples are independent).

Definitions and the passage of the paper (Hydro, arXiv 2403.14902) each
function follows:

* ``truth_table`` / ``result_ids``: the query keeps tuples on which all UDF
  predicates hold (section 1, motivating query; section 4.1, the UC1 query with
  two UDF predicates joined by AND).  Routing changes only the order of
  evaluation (section 4.1, "System Variants": no-reordering evaluates left to
  right; the adaptive variants reorder at run time) and failing rows are
  dropped at once (section 3.3, "Eager Materialization"), so the answer is
  order independent and equals this plain definition.
* ``predicate_margin`` / ``decide``: the paper's predicates compare a
  classifier's label with a constant (UDF(frame) = 'label').  The synthetic
  predicates generalise the label to a class subset S and a threshold theta:
  d = max_{c in S} z_c - max_{c not in S} z_c, pass iff d > theta (strict).  With
  theta = 0 this is "argmax in S" with ties rejected.
* ``policy_keys`` / ``policy_order``: section 4.1, "Cost-Driven Routing Policy"
  (score = cost/(1 - selectivity), lowest first) and "System Variants" (cost-
  driven ranks by cost alone, selectivity-driven by selectivity alone).
* ``fixed_order_counts``: "No Reordering" evaluates the written order with
  short-circuit (section 4.1, "System Variants"); section 4.1 "System
  Variants" also computes selectivity from the count of filtered rows.
* ``reuse_aware_cost`` / ``reuse_aware_order`` / ``cached_decision``:
  section 4.3, "Reuse-aware Routing": cached UDF results are reused, and the
  estimated cost of a predicate for a routing batch is (1 - cache hit rate)
  times the cost of computing it (cache access taken as free).  A cached
  decision taken at one threshold answers another threshold only where the
  comparison is implied (the reading taken here: its cache holds decisions, not
  raw UDF outputs).
* ``color_fraction``: a cheap CPU predicate beside the GPU UDFs (section 4.1:
  the colour classifier runs on the CPU concurrently with the breed model on
  the GPU); the reading taken here is a channel box, the fraction of pixels whose
  three values all lie inside it, compared with theta like the UDF margins.
* ``crop_logits``: a CNN on each tuple's crop of its frame, the variable-size
  inputs of section 5.3 (UDF composition, a classifier on Crop(frame, bbox)).
* ``replay_route``: checks a per-tuple visit sequence against the routing
  rules of section 3.3 ("Metadata for Data Routing": a batch visits each
  predicate at most once and is complete when all are visited; "Eager
  Materialization": a failing tuple goes no further) and derives the exact
  per-predicate counts that route implies.

Model arithmetic (inputs are synthetic classifiers, see ``hydro_synth``):
normalisation x' = (x - 0.5) * 4 for every predicate; zero padding in
normalised space; MLP h = ReLU(x' W1 + b1), z = h W2 + b2 with x' flattened
NHWC; CNN layers y[o,i,j] = ReLU(b[o] + sum_{c,u,v} W[o,c,u,v] x~[c,2i+u-1,2j+v-1])
(cross-correlation, stride 2, pad 1), global average pool, z = g Wfc + bfc.
"""
from __future__ import annotations

import itertools
import math
import os
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

N_CLASSES = 10

POLICY_FIXED = "fixed"
POLICY_SEL = "selectivity"
POLICY_SCORE = "score"
POLICY_COST = "cost"


# --------------------------------------------------------------------------
# O1/O2: frames to fp64 and normalisation
# --------------------------------------------------------------------------
def frames_to_f64(frames: np.ndarray, dtype: str) -> np.ndarray:
    """Exact fp64 value of stored frames.

    bf16 frames arrive as uint16 bit patterns (exact widening); uint8 v means
    v/255 (one IEEE fp64 division, round to nearest); fp32 widens exactly.
    """
    if dtype == "bf16":
        return (np.asarray(frames, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    if dtype == "u8":
        return np.asarray(frames).astype(np.float64) / 255.0
    return np.asarray(frames, dtype=np.float32).astype(np.float64)


def normalize(x: np.ndarray) -> np.ndarray:
    """x' = (x - 0.5) * 4, applied by every predicate before its model."""
    return (x - 0.5) * 4.0


# --------------------------------------------------------------------------
# O3/O4: model logits in fp64
# --------------------------------------------------------------------------
def mlp_logits(t: dict, xn: np.ndarray) -> np.ndarray:
    """z = ReLU(x' W1 + b1) W2 + b2; x' is the normalised frame flattened NHWC."""
    n = xn.shape[0]
    x = xn.reshape(n, -1)
    h = np.maximum(x @ t["W1"] + t["b1"], 0.0)
    return h @ t["W2"] + t["b2"]


def conv3x3_s2_relu(a: np.ndarray, w: np.ndarray, b: np.ndarray) -> np.ndarray:
    """One layer: y[n,i,j,o] = ReLU(b[o] + sum_{c,u,v} w[o,c,u,v] * a~[n, 2i+u-1, 2j+v-1, c]).

    ``a`` is NHWC fp64 (already normalised); a~ is ``a`` with a zero border;
    ``w`` [o][c][3][3] and ``b`` are fp64.
    The sum is written as im2col followed by one matmul.
    """
    n, hgt, wid, cin = a.shape
    ho, wo = (hgt + 1) // 2, (wid + 1) // 2
    ap = np.zeros((n, hgt + 2, wid + 2, cin), dtype=np.float64)
    ap[:, 1:hgt + 1, 1:wid + 1, :] = a
    cols = np.empty((n, ho, wo, 3, 3, cin), dtype=np.float64)
    for u in range(3):
        for v in range(3):
            # padded row of input row 2i+u-1 is 2i+u
            cols[:, :, :, u, v, :] = ap[:, u:u + 2 * ho:2, v:v + 2 * wo:2, :]
    wm = np.transpose(w, (2, 3, 1, 0)).reshape(9 * cin, -1)  # [(u,v,c)][o]
    y = cols.reshape(n * ho * wo, 9 * cin) @ wm + b
    return np.maximum(y, 0.0).reshape(n, ho, wo, -1)


def cnn_logits(t: dict, xn: np.ndarray) -> np.ndarray:
    """Conv stack, then the arithmetic mean over all final positions, then FC."""
    a = xn
    for w, b in t["convs"]:
        a = conv3x3_s2_relu(a, w, b)
    g = a.mean(axis=(1, 2))
    return g @ t["Wfc"] + t["bfc"]


def _f64_tensors(t: dict) -> dict:
    """The model's fp32 parameters widened (exactly) to fp64, once per call."""
    out = {}
    for k, v in t.items():
        if k == "convs":
            out[k] = [(w.astype(np.float64), b.astype(np.float64)) for w, b in v]
        else:
            out[k] = v.astype(np.float64)
    return out


def model_logits(model, frames: np.ndarray, dtype: str, chunk: int = 0, workers: int = 0) -> np.ndarray:
    """fp64 logits [n][10] of one predicate model on stored frames.

    Tuples are independent, so chunks of tuples are evaluated by a thread pool
    (BLAS limited to one thread per worker); each chunk's arithmetic is the
    plain definition above.
    """
    from concurrent.futures import ThreadPoolExecutor
    from threadpoolctl import threadpool_limits
    n = frames.shape[0]
    arch = model.desc.arch
    if chunk <= 0:
        chunk = 128 if arch == "mlp" else 16
    if workers <= 0:
        workers = min(16, os.cpu_count() or 1)
    t64 = _f64_tensors(model.tensors)
    fn = mlp_logits if arch == "mlp" else cnn_logits
    out = np.empty((n, N_CLASSES), dtype=np.float64)

    def job(s):
        xn = normalize(frames_to_f64(frames[s:s + chunk], dtype))
        out[s:s + chunk] = fn(t64, xn)

    with threadpool_limits(1):
        with ThreadPoolExecutor(workers) as ex:
            list(ex.map(job, range(0, n, chunk)))
    return out


def crop_logits(model, frames: np.ndarray, dtype: str, crops: np.ndarray) -> np.ndarray:
    """fp64 logits [n][10] of a CNN model applied to each tuple's crop (y0, x0, h, w) of its
    frame: the crop is the image (zero padding at its border in normalised space), the mean runs
    over the crop's final positions (section 5.3: a classifier on Crop(frame, bbox))."""
    t64 = _f64_tensors(model.tensors)
    out = np.empty((frames.shape[0], N_CLASSES), dtype=np.float64)
    for i, (y0, x0, h, w) in enumerate(np.asarray(crops, dtype=np.int64)):
        xn = normalize(frames_to_f64(frames[i:i + 1, y0:y0 + h, x0:x0 + w], dtype))
        out[i] = cnn_logits(t64, xn)[0]
    return out


# --------------------------------------------------------------------------
# O5: margin and decision
# --------------------------------------------------------------------------
def predicate_margin(z: np.ndarray, class_mask: int) -> np.ndarray:
    """d = max_{c in S} z_c - max_{c not in S} z_c; a max over no classes is -inf."""
    inside = np.array([(class_mask >> c) & 1 == 1 for c in range(N_CLASSES)])
    neg = -np.inf
    zin = np.where(inside[None, :], z, neg).max(axis=1) if inside.any() else np.full(z.shape[0], neg)
    zout = np.where(~inside[None, :], z, neg).max(axis=1) if (~inside).any() else np.full(z.shape[0], neg)
    with np.errstate(invalid="ignore"):
        d = zin - zout
    return d


def decide(d: np.ndarray, theta) -> np.ndarray:
    """pass iff d > theta (strict); theta is the fp32 threshold widened to fp64."""
    return d > np.asarray(theta, dtype=np.float64)


def color_fraction(frames: np.ndarray, dtype: str, lo: Sequence[float], hi: Sequence[float],
                   stride: int = 1) -> np.ndarray:
    """Fraction of each frame's sampled pixels (rows and columns 0, stride, 2 stride, ...) with
    lo[c] <= x_c <= hi[c] for all three channels (fp64)."""
    x = frames_to_f64(np.asarray(frames)[:, ::stride, ::stride], dtype)
    lo64 = np.asarray(lo, dtype=np.float32).astype(np.float64)
    hi64 = np.asarray(hi, dtype=np.float32).astype(np.float64)
    inside = np.all((x >= lo64) & (x <= hi64), axis=-1)
    return inside.reshape(x.shape[0], -1).mean(axis=1)


# --------------------------------------------------------------------------
# O6/O7: truth table and result
# --------------------------------------------------------------------------
def tuple_thresholds(thresholds: np.ndarray, seg_len: int, ids: np.ndarray) -> np.ndarray:
    """theta of every tuple: the row of its segment, segment = min(id // seg_len, n_seg - 1)."""
    th = np.asarray(thresholds, dtype=np.float32).astype(np.float64)
    seg = np.minimum(np.asarray(ids) // seg_len, th.shape[0] - 1)
    return th[seg]                                                      # [n][K]


def truth_table(frames: np.ndarray, dtype: str, models: Sequence, class_masks: Sequence[int],
                thresholds: np.ndarray, seg_len: int, id_base: int = 0,
                return_logits: bool = False):
    """Evaluate every predicate on every tuple (no short-circuit).

    Returns (P bool [n][K], D fp64 [n][K]) and optionally logits [K][n][10].
    """
    n = frames.shape[0]
    k = len(models)
    ids = id_base + np.arange(n)
    th = tuple_thresholds(thresholds, seg_len, ids)
    P = np.zeros((n, k), dtype=bool)
    D = np.zeros((n, k), dtype=np.float64)
    Z = [] if return_logits else None
    for j, m in enumerate(models):
        z = model_logits(m, frames, dtype)
        D[:, j] = predicate_margin(z, class_masks[j])
        P[:, j] = decide(D[:, j], th[:, j])
        if return_logits:
            Z.append(z)
    if return_logits:
        return P, D, Z
    return P, D


def result_ids(P: np.ndarray, id_base: int = 0) -> np.ndarray:
    """Ascending int64 ids of tuples that pass every predicate."""
    return (id_base + np.nonzero(P.all(axis=1))[0]).astype(np.int64)


def near_tie_gap(D: np.ndarray, thresholds: np.ndarray, seg_len: int, id_base: int = 0) -> float:
    """min over tuples and predicates of |d - theta| (finite margins only)."""
    ids = id_base + np.arange(D.shape[0])
    th = tuple_thresholds(thresholds, seg_len, ids)
    gap = np.abs(D - th)
    gap = gap[np.isfinite(gap)]
    return float(gap.min()) if gap.size else math.inf


# --------------------------------------------------------------------------
# Short-circuit evaluation in a static order, statistics
# --------------------------------------------------------------------------
def short_circuit_eval(P: np.ndarray, order: Sequence[int], id_base: int = 0):
    """Evaluate predicates in ``order``, dropping a tuple at its first failure.

    Returns (result ids, evaluated[K], passed[K]).  Computed tuple by tuple
    over the truth table, independent of ``result_ids``.
    """
    n, k = P.shape
    evaluated = np.zeros(k, dtype=np.int64)
    passed = np.zeros(k, dtype=np.int64)
    alive = np.ones(n, dtype=bool)
    for j in order:
        evaluated[j] += int(alive.sum())
        ok = alive & P[:, j]
        passed[j] += int(ok.sum())
        alive = ok
    return (id_base + np.nonzero(alive)[0]).astype(np.int64), evaluated, passed


def fixed_order_counts(P: np.ndarray, order: Sequence[int]):
    _, ev, ps = short_circuit_eval(P, order)
    return ev, ps


def stats_invariants(evaluated: Sequence[int], passed: Sequence[int], n: int, n_result: int) -> List[str]:
    """Properties every valid route's counts satisfy; returns the violated ones.

    Each tuple is dropped by exactly one failing evaluation or reaches the
    output, so sum_k (evaluated_k - passed_k) = n - |R|; every result tuple
    was evaluated and passed by every predicate.
    """
    bad = []
    ev = np.asarray(evaluated, dtype=np.int64)
    ps = np.asarray(passed, dtype=np.int64)
    if int((ev - ps).sum()) != n - n_result:
        bad.append("sum(evaluated - passed) != n - |R|")
    if (ps < n_result).any():
        bad.append("passed_k < |R|")
    if (ev < ps).any():
        bad.append("evaluated_k < passed_k")
    if (ev > n).any():
        bad.append("evaluated_k > n")
    return bad


def replay_route(P: np.ndarray, routes: Sequence[Sequence[int]]):
    """Check per-tuple visit sequences and derive the counts they imply.

    A valid sequence visits distinct predicates; every visit but the last
    passed; the last visit failed, or the sequence covers all K predicates
    (then the tuple is in the result).  Returns (ok, evaluated[K], passed[K],
    result indices, message).
    """
    n, k = P.shape
    evaluated = np.zeros(k, dtype=np.int64)
    passed = np.zeros(k, dtype=np.int64)
    out = []
    for t, seq in enumerate(routes):
        seq = list(seq)
        if len(set(seq)) != len(seq) or any(j < 0 or j >= k for j in seq):
            return False, evaluated, passed, None, f"tuple {t}: invalid sequence {seq}"
        if not seq:
            return False, evaluated, passed, None, f"tuple {t}: never evaluated"
        for i, j in enumerate(seq):
            evaluated[j] += 1
            if P[t, j]:
                passed[j] += 1
            elif i != len(seq) - 1:
                return False, evaluated, passed, None, f"tuple {t}: continued after failing {j}"
        last_ok = bool(P[t, seq[-1]])
        if last_ok and len(seq) != k:
            return False, evaluated, passed, None, f"tuple {t}: stopped early after passing"
        if last_ok:
            out.append(t)
    return True, evaluated, passed, np.asarray(out, dtype=np.int64), ""


# --------------------------------------------------------------------------
# Routing-policy keys (lowest key first)
# --------------------------------------------------------------------------
def smoothed_selectivity(passed, evaluated) -> np.ndarray:
    """(passed + 1) / (evaluated + 2): the pass fraction with a uniform prior.

    The paper estimates selectivity from counts of filtered rows; the +1/+2
    prior is the reading taken here for predicates that have seen few tuples.
    """
    return (np.asarray(passed, dtype=np.float64) + 1.0) / (np.asarray(evaluated, dtype=np.float64) + 2.0)


def policy_keys(policy: str, cost, selectivity) -> np.ndarray:
    """Ranking key of each predicate.

    score: cost / (1 - selectivity), +inf when selectivity = 1;
    cost: cost; selectivity: selectivity.
    """
    c = np.asarray(cost, dtype=np.float64)
    s = np.asarray(selectivity, dtype=np.float64)
    if policy == POLICY_SCORE:
        with np.errstate(divide="ignore"):
            return np.where(s >= 1.0, np.inf, c / (1.0 - s))
    if policy == POLICY_COST:
        return c.copy()
    if policy == POLICY_SEL:
        return s.copy()
    raise ValueError(policy)


def policy_order(policy: str, cost, selectivity) -> List[int]:
    """Predicates sorted by ascending key; equal keys go to the lower index."""
    key = policy_keys(policy, cost, selectivity)
    return sorted(range(len(key)), key=lambda j: (key[j], j))


def reuse_aware_cost(hit_rate, cost) -> np.ndarray:
    """Estimated cost of each predicate for a routing batch: (1 - cache hit rate) * cost."""
    return (1.0 - np.asarray(hit_rate, dtype=np.float64)) * np.asarray(cost, dtype=np.float64)


def reuse_aware_order(policy: str, cost, selectivity, hit_rate) -> List[int]:
    """The policy's order with the reuse-aware estimate in place of the cost (cost and score
    policies; the selectivity policy does not use the cost)."""
    return policy_order(policy, reuse_aware_cost(hit_rate, cost), selectivity)


def cached_decision(theta_cached: float, passed_cached: bool, theta: float) -> Tuple[bool, bool]:
    """(decided, pass) for a tuple whose margin d was found to satisfy d > theta_cached
    (passed_cached) or d <= theta_cached (not passed_cached), now compared with theta.

    d > theta_cached implies d > theta when theta <= theta_cached; d <= theta_cached implies
    d <= theta when theta >= theta_cached.  Otherwise the cached outcome does not decide.
    """
    if passed_cached and theta <= theta_cached:
        return True, True
    if not passed_cached and theta >= theta_cached:
        return True, False
    return False, False


def concurrent_makespan(order: Sequence[int], passes: np.ndarray, cost: Sequence[float]) -> float:
    """Predicates on separate resources running concurrently (section 4.1, "Example comparison"):
    each predicate has one worker that takes its tuples first come, first served, cost[j] time
    units each; every tuple starts at the first predicate of ``order`` at time 0, moves to the
    next one when it passes and is dropped when it fails.  passes[t, j]: tuple t passes j.
    Returns the time the last evaluation ends."""
    passes = np.asarray(passes, dtype=bool)
    n = passes.shape[0]
    arrive = np.zeros(n)                    # arrival time of each live tuple at the current stage
    live = np.arange(n)
    end = 0.0
    for j in order:
        free = 0.0
        done = np.empty(live.size)
        for q, t in enumerate(live):         # first come, first served (arrival order; ties by id)
            start = max(free, arrive[q])
            free = start + cost[j]
            done[q] = free
        end = max(end, free if live.size else 0.0)
        keep = passes[live, j]
        live, arrive = live[keep], done[keep]
        o = np.lexsort((live, arrive))
        live, arrive = live[o], arrive[o]
    return float(end)


def policy_first(policy: str, cost, selectivity) -> int:
    """The predicate a policy evaluates first (lowest key, lowest index on ties)."""
    return policy_order(policy, cost, selectivity)[0]


# --------------------------------------------------------------------------
# Derived analysis quantities
# --------------------------------------------------------------------------
def best_static_order(P: np.ndarray, flops: Sequence[float]):
    """Static order with the least total FLOPs over all K! orders, and that total."""
    k = P.shape[1]
    best = None
    for order in itertools.permutations(range(k)):
        ev, _ = fixed_order_counts(P, order)
        f = float(np.dot(ev, flops))
        if best is None or f < best[1]:
            best = (list(order), f)
    return best


def clairvoyant_flops(P: np.ndarray, flops: Sequence[float]) -> float:
    """Per-tuple optimal routing: a failing tuple pays its cheapest failing predicate,
    a passing tuple pays every predicate."""
    f = np.asarray(flops, dtype=np.float64)
    allpass = P.all(axis=1)
    fail_cost = np.where(~P, f[None, :], np.inf).min(axis=1)
    return float(fail_cost[~allpass].sum() + allpass.sum() * f.sum())


__all__ = [name for name in dir() if not name.startswith("_") and name not in ("annotations",)]
