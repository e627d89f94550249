"""ctypes binding of libhydro.so (the gfx950 engine declared in include/hydro.h).

Argument marshalling only: every step of the query runs in the library's HIP kernels.
torch is used for device memory (frames may be CUDA/HIP tensors) and streams.  The binding
raises if the library has not been built; there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhydro.so")

MAX_PREDICATES = 8
MAX_LAYERS = 4

OK, EINVAL, ENOMEM, EDEVICE, EUNSUPPORTED, ECAPACITY, ESTATE = 0, -1, -2, -3, -4, -5, -6
DTYPE_F32, DTYPE_BF16, DTYPE_U8 = 0, 1, 2
MEM_DEVICE, MEM_HOST = 0, 1
ARCH_MLP, ARCH_CNN, ARCH_HOST = 0, 1, 2
ROUTE_FIXED, ROUTE_SEL, ROUTE_SCORE, ROUTE_COST, ROUTE_LEARNED = 0, 1, 2, 3, 4
PREC_FP32, PREC_BF16, PREC_FP8 = 0, 1, 2
COST_MEASURED, COST_STATIC = 0, 1

ROUTES = {"fixed": ROUTE_FIXED, "selectivity": ROUTE_SEL, "score": ROUTE_SCORE, "cost": ROUTE_COST,
          "learned": ROUTE_LEARNED}
PRECISIONS = {"fp32": PREC_FP32, "bf16": PREC_BF16, "fp8": PREC_FP8}
DTYPES = {"f32": DTYPE_F32, "bf16": DTYPE_BF16, "u8": DTYPE_U8}


class HydroError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"hydro status {code}: {msg}")
        self.code = code


class Frames(C.Structure):
    _fields_ = [("data", C.c_void_p), ("dtype", C.c_int32), ("where", C.c_int32), ("n", C.c_int64),
                ("h", C.c_int32), ("w", C.c_int32), ("id_base", C.c_int64), ("host_data", C.c_void_p),
                ("crops", C.c_void_p)]


FP = C.POINTER(C.c_float)


class Model(C.Structure):
    _fields_ = [("arch", C.c_int32), ("in_h", C.c_int32), ("in_w", C.c_int32), ("hidden", C.c_int32),
                ("w1", FP), ("b1", FP), ("w2", FP), ("b2", FP),
                ("n_layers", C.c_int32), ("widths", C.c_int32 * MAX_LAYERS),
                ("conv_w", FP * MAX_LAYERS), ("conv_b", FP * MAX_LAYERS),
                ("fc_w", FP), ("fc_b", FP), ("class_mask", C.c_uint32),
                ("color_lo", C.c_float * 3), ("color_hi", C.c_float * 3), ("color_stride", C.c_int32),
                ("on_crop", C.c_int32)]


class Policy(C.Structure):
    _fields_ = [("route", C.c_int32), ("order", C.c_int32 * MAX_PREDICATES), ("routing_batch", C.c_int32),
                ("wave", C.c_int32), ("warmup_batches", C.c_int32), ("ewma_alpha", C.c_float),
                ("cost_source", C.c_int32), ("precision", C.c_int32), ("tau", C.c_float), ("tau32", C.c_float),
                ("grouped", C.c_int32), ("use_graph", C.c_int32), ("log_routes", C.c_int32),
                ("time_kernels", C.c_int32), ("autotune", C.c_int32),
                ("explore", C.c_float), ("seed", C.c_uint64), ("stream", C.c_void_p), ("tau16", C.c_float),
                ("reuse", C.c_int32), ("cache_log2", C.c_int32), ("balance", C.c_int32), ("rescore3", C.c_int32)]


class PredStats(C.Structure):
    _fields_ = [("evaluated", C.c_uint64), ("passed", C.c_uint64), ("rescored", C.c_uint64),
                ("escalated", C.c_uint64), ("device_us", C.c_double), ("cost_us_per_tuple", C.c_double),
                ("selectivity", C.c_double), ("rescored16", C.c_uint64), ("cache_hits", C.c_uint64)]


class QueryInfo(C.Structure):
    _fields_ = [("n_tuples", C.c_uint64), ("n_result", C.c_uint64), ("rounds", C.c_uint32), ("k", C.c_uint32),
                ("learned_routed", C.c_uint64), ("stats_routed", C.c_uint64), ("learned_active", C.c_uint32),
                ("train_steps", C.c_uint32), ("elapsed_us", C.c_double), ("route_ms", C.c_double),
                ("first_pass_ms", C.c_double), ("f32_pass_ms", C.c_double), ("f64_pass_ms", C.c_double),
                ("timed_rounds", C.c_uint32), ("pad_", C.c_uint32), ("learned_stale", C.c_uint64),
                ("mid_pass_ms", C.c_double), ("arm_flops", C.c_double * 2), ("arm_tuples", C.c_double * 2)]


class RoundRecord(C.Structure):
    _fields_ = [("order", C.c_int32 * MAX_PREDICATES), ("folded_evaluated", C.c_uint64 * MAX_PREDICATES),
                ("folded_passed", C.c_uint64 * MAX_PREDICATES), ("selectivity", C.c_double * MAX_PREDICATES),
                ("cost", C.c_double * MAX_PREDICATES), ("seen_mask", C.c_uint32), ("pad_", C.c_uint32)]


_lib = None


def lib():
    """Load libhydro.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2403_14902_amd/build.py")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        L.hydro_policy_default.argtypes = [C.POINTER(Policy)]
        L.hydro_policy_default.restype = None
        L.hydro_query.argtypes = [C.POINTER(Frames), C.POINTER(Model), i32, FP, i32, i64, C.POINTER(Policy),
                                  C.POINTER(C.POINTER(C.c_int64)), C.POINTER(C.c_int64), C.POINTER(PredStats)]
        L.hydro_query_noalloc.argtypes = [C.POINTER(Frames), C.POINTER(Model), i32, FP, i32, i64, C.POINTER(Policy),
                                          C.POINTER(C.c_int64), i64, C.POINTER(C.c_int64), C.POINTER(PredStats)]
        L.hydro_session_create.argtypes = [C.POINTER(Model), i32, C.POINTER(Policy), i32, i32, i64, C.POINTER(vp)]
        L.hydro_session_reset.argtypes = [vp]
        L.hydro_session_push.argtypes = [vp, C.POINTER(Frames), FP, i32, i64]
        L.hydro_session_finish.argtypes = [vp, C.POINTER(C.POINTER(C.c_int64)), C.POINTER(C.c_int64),
                                           C.POINTER(PredStats)]
        L.hydro_session_info.argtypes = [vp, C.POINTER(QueryInfo)]
        L.hydro_session_routes.argtypes = [vp, i64, i64, C.POINTER(C.c_uint32)]
        L.hydro_session_round_log.argtypes = [vp, i32, i32, C.POINTER(RoundRecord)]
        L.hydro_session_set_order.argtypes = [vp, C.POINTER(C.c_int32)]
        L.hydro_router_train_debug.argtypes = [i32, C.POINTER(C.c_uint16), C.POINTER(C.c_int32),
                                               C.POINTER(C.c_uint8), i32, FP, FP, FP, i32, C.c_float]
        L.hydro_compaction_debug.argtypes = [i32, i64, vp, i32, i32, vp, C.POINTER(C.c_int64), C.POINTER(PredStats),
                                             C.POINTER(C.c_double)]
        L.hydro_session_logits.argtypes = [vp, i32, i32, C.POINTER(Frames), C.POINTER(C.c_double)]
        L.hydro_session_calibrate.argtypes = [vp, C.POINTER(Frames), C.c_float, FP, FP]
        L.hydro_session_bands.argtypes = [vp, FP, FP, FP]
        L.hydro_session_router_params.argtypes = [vp, FP, i32]
        L.hydro_session_cache_clear.argtypes = [vp]
        L.hydro_session_set_route.argtypes = [vp, i32]
        L.hydro_session_destroy.argtypes = [vp]
        L.hydro_free.argtypes = [vp]
        L.hydro_free.restype = None
        L.hydro_last_error.restype = C.c_char_p
        L.hydro_version.restype = C.c_char_p
        for name in ("hydro_query", "hydro_query_noalloc", "hydro_session_create", "hydro_session_reset", "hydro_session_push",
                     "hydro_session_finish", "hydro_session_info", "hydro_session_routes",
                     "hydro_session_round_log", "hydro_session_set_order", "hydro_router_train_debug",
                     "hydro_compaction_debug", "hydro_session_logits",
                     "hydro_session_calibrate", "hydro_session_bands", "hydro_session_router_params",
                     "hydro_session_cache_clear", "hydro_session_set_route", "hydro_session_destroy"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


EXPORTED = ("hydro_policy_default", "hydro_query", "hydro_query_noalloc", "hydro_session_create", "hydro_session_reset",
            "hydro_session_push", "hydro_session_finish", "hydro_session_info", "hydro_session_routes",
            "hydro_session_round_log", "hydro_session_set_order", "hydro_router_train_debug",
            "hydro_compaction_debug", "hydro_session_logits", "hydro_session_calibrate", "hydro_session_bands",
            "hydro_session_router_params", "hydro_session_cache_clear", "hydro_session_set_route",
            "hydro_session_destroy",
            "hydro_free",
            "hydro_last_error", "hydro_version")


def _check(rc: int):
    if rc != OK:
        raise HydroError(rc, lib().hydro_last_error().decode())


def _fp(a: Optional[np.ndarray]):
    if a is None:
        return FP()
    return a.ctypes.data_as(FP)


class ModelSpec:
    """A predicate model held as contiguous fp32 numpy arrays (kept alive by this object)."""

    def __init__(self, arch: str, in_hw: int, class_mask: int, tensors: dict, hidden: int = 0,
                 widths: Sequence[int] = (), on_crop: bool = False):
        self.arch, self.in_hw, self.class_mask = arch, in_hw, int(class_mask)
        self.on_crop = bool(on_crop)
        self.hidden, self.widths = hidden, tuple(widths)
        f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
        if arch == "host":
            self.t = {"lo": [float(x) for x in tensors["lo"]], "hi": [float(x) for x in tensors["hi"]],
                      "stride": int(tensors.get("stride", 1))}
        elif arch == "mlp":
            self.t = {k: f32(tensors[k]) for k in ("W1", "b1", "W2", "b2")}
        else:
            self.t = {"convs": [(f32(w), f32(b)) for w, b in tensors["convs"]],
                      "Wfc": f32(tensors["Wfc"]), "bfc": f32(tensors["bfc"])}

    @classmethod
    def host_color(cls, in_hw: int, lo: Sequence[float], hi: Sequence[float], stride: int = 1) -> "ModelSpec":
        """A HOST predicate: the fraction of sampled pixels (every stride-th row and column) inside
        the channel box [lo, hi], decided by CPU threads."""
        return cls("host", in_hw, 0, {"lo": lo, "hi": hi, "stride": stride})

    @classmethod
    def from_weights(cls, weights, class_mask: int, on_crop: bool = False, in_hw: int = 0) -> "ModelSpec":
        """From a ``hydro_synth.ModelWeights`` (on_crop: a CNN on each tuple's crop of frames of
        side in_hw)."""
        d = weights.desc
        if on_crop:
            return cls("cnn", in_hw or d.in_hw, class_mask, weights.tensors, widths=d.widths, on_crop=True)
        if d.arch == "mlp":
            hw = int(round((d.d_in / 3) ** 0.5))
            return cls("mlp", hw, class_mask, weights.tensors, hidden=d.hidden)
        return cls("cnn", d.in_hw, class_mask, weights.tensors, widths=d.widths)

    def to_c(self) -> Model:
        m = Model()
        m.in_h = m.in_w = self.in_hw
        m.class_mask = self.class_mask
        if self.arch == "host":
            m.arch = ARCH_HOST
            for c in range(3):
                m.color_lo[c], m.color_hi[c] = self.t["lo"][c], self.t["hi"][c]
            m.color_stride = self.t["stride"]
        elif self.arch == "mlp":
            m.arch = ARCH_MLP
            m.hidden = self.hidden
            m.w1, m.b1, m.w2, m.b2 = (_fp(self.t[k]) for k in ("W1", "b1", "W2", "b2"))
        else:
            m.arch = ARCH_CNN
            m.on_crop = int(self.on_crop)
            m.n_layers = len(self.widths)
            for i, w in enumerate(self.widths):
                m.widths[i] = w
                m.conv_w[i] = _fp(self.t["convs"][i][0])
                m.conv_b[i] = _fp(self.t["convs"][i][1])
            m.fc_w, m.fc_b = _fp(self.t["Wfc"]), _fp(self.t["bfc"])
        return m


def make_policy(route: str = "score", order: Optional[Sequence[int]] = None, precision: str = "bf16",
                **kw) -> Policy:
    p = Policy()
    lib().hydro_policy_default(C.byref(p))
    p.route = ROUTES[route] if isinstance(route, str) else int(route)
    if order is not None:
        for i, o in enumerate(order):
            p.order[i] = int(o)
    p.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    for k, v in kw.items():
        if k == "cost_source" and isinstance(v, str):
            v = COST_STATIC if v == "static" else COST_MEASURED
        setattr(p, k, v)
    return p


def _frames_struct(frames, dtype: str, id_base: int) -> Frames:
    fr = Frames()
    fr.dtype = DTYPES[dtype]
    fr.id_base = int(id_base)
    if hasattr(frames, "data_ptr"):          # torch tensor
        assert frames.is_contiguous(), "frames must be contiguous"
        fr.data = frames.data_ptr()
        fr.where = MEM_DEVICE if frames.is_cuda else MEM_HOST
        shape = tuple(frames.shape)
    else:
        assert frames.flags["C_CONTIGUOUS"], "frames must be contiguous"
        fr.data = frames.ctypes.data
        fr.where = MEM_HOST
        shape = frames.shape
    if len(shape) != 4 or shape[3] != 3:
        raise HydroError(EINVAL, f"frames must be [n, h, w, 3], got {shape}")
    fr.n, fr.h, fr.w = shape[0], shape[1], shape[2]
    return fr


def _stats_list(st, k) -> List[Dict]:
    return [{f: getattr(st[i], f) for f, _ in PredStats._fields_} for i in range(k)]


class Session:
    """A query session: models are uploaded once; each query is pushes + finish."""

    def __init__(self, models: Sequence[ModelSpec], policy: Policy, frame_hw: int, max_push: int):
        self.models = list(models)
        self.k = len(self.models)
        self._cm = (Model * self.k)(*[m.to_c() for m in self.models])
        self.policy = policy
        self._h = C.c_void_p()
        self._keep = []
        _check(lib().hydro_session_create(self._cm, self.k, C.byref(policy), frame_hw, frame_hw, int(max_push),
                                          C.byref(self._h)))

    def reset(self):
        self._keep = []
        _check(lib().hydro_session_reset(self._h))

    def push(self, frames, dtype: str, thresholds: np.ndarray, seg_len: int, id_base: int = 0, host_copy=None,
             crops=None):
        """host_copy: the same frames in host memory (numpy or CPU tensor) for HOST predicates when
        `frames` is on the device.  crops: int32 [n][4] (y0, x0, h, w) per tuple for on_crop
        predicates."""
        th = np.ascontiguousarray(thresholds, dtype=np.float32)
        if th.ndim == 1:
            th = th[None, :]
        fr = _frames_struct(frames, dtype, id_base)
        if crops is not None:
            cr = np.ascontiguousarray(crops, dtype=np.int32)
            fr.crops = cr.ctypes.data
            self._keep.append(cr)
        if host_copy is not None:
            hc = host_copy if hasattr(host_copy, "data_ptr") else np.ascontiguousarray(host_copy)
            fr.host_data = hc.data_ptr() if hasattr(hc, "data_ptr") else hc.ctypes.data
            self._keep.append(hc)
        self._keep.append((frames, th))
        _check(lib().hydro_session_push(self._h, C.byref(fr), _fp(th), th.shape[0], int(seg_len)))

    def finish(self):
        ptr = C.POINTER(C.c_int64)()
        n = C.c_int64()
        st = (PredStats * self.k)()
        _check(lib().hydro_session_finish(self._h, C.byref(ptr), C.byref(n), st))
        ids = np.ctypeslib.as_array(ptr, shape=(n.value,)).copy() if n.value > 0 else np.zeros(0, np.int64)
        lib().hydro_free(ptr)
        self._keep = []
        return ids, _stats_list(st, self.k)

    def info(self) -> Dict:
        q = QueryInfo()
        _check(lib().hydro_session_info(self._h, C.byref(q)))
        out = {f: getattr(q, f) for f, _ in QueryInfo._fields_}
        out["arm_flops"], out["arm_tuples"] = list(q.arm_flops), list(q.arm_tuples)
        return out

    def cache_clear(self):
        """Drop every cached decision (policy.reuse > 0)."""
        _check(lib().hydro_session_cache_clear(self._h))

    def router_params(self) -> np.ndarray:
        """The learned router's parameters W1 | b1 | W2 | b2 (see hydro_session_router_params)."""
        p = np.zeros(ROUTER_NPARAM, dtype=np.float32)
        _check(lib().hydro_session_router_params(self._h, _fp(p), p.size))
        return p

    def routes(self, first: int, n: int) -> np.ndarray:
        out = np.zeros(n, dtype=np.uint32)
        _check(lib().hydro_session_routes(self._h, first, n, out.ctypes.data_as(C.POINTER(C.c_uint32))))
        return out

    def set_order(self, order: Sequence[int]):
        """The FIXED route's order for the next queries."""
        o = (C.c_int32 * MAX_PREDICATES)(*[int(x) for x in order])
        _check(lib().hydro_session_set_order(self._h, o))

    def set_route(self, route: str):
        """The routing policy of the next queries (fixed, selectivity, score or cost)."""
        _check(lib().hydro_session_set_route(self._h, ROUTES[route] if isinstance(route, str) else int(route)))

    def round_log(self, first: int, n: int) -> List[Dict]:
        """Per-round rankings and folded statistics of the last query (policy.log_routes = 1)."""
        recs = (RoundRecord * max(1, n))()
        _check(lib().hydro_session_round_log(self._h, first, n, recs))
        k = self.k
        return [{"order": list(r.order)[:k], "folded_evaluated": list(r.folded_evaluated)[:k],
                 "folded_passed": list(r.folded_passed)[:k], "selectivity": list(r.selectivity)[:k],
                 "cost": list(r.cost)[:k], "seen_mask": r.seen_mask} for r in recs[:n]]

    def logits(self, pred: int, tier: int, frames, dtype: str) -> np.ndarray:
        fr = _frames_struct(frames, dtype, 0)
        out = np.zeros((fr.n, 10), dtype=np.float64)
        _check(lib().hydro_session_logits(self._h, pred, tier, C.byref(fr),
                                          out.ctypes.data_as(C.POINTER(C.c_double))))
        return out

    def calibrate(self, frames, dtype: str, safety: float = 2.0):
        """Per-predicate re-score bands from measured margin errors (see hydro.h)."""
        fr = _frames_struct(frames, dtype, 0)
        t = np.zeros(self.k, dtype=np.float32)
        t32 = np.zeros(self.k, dtype=np.float32)
        _check(lib().hydro_session_calibrate(self._h, C.byref(fr), float(safety), _fp(t), _fp(t32)))
        return t, t32

    def bands(self):
        """The per-predicate bands the next push uses: (tau, tau16, tau32)."""
        t, t16, t32 = (np.zeros(self.k, dtype=np.float32) for _ in range(3))
        _check(lib().hydro_session_bands(self._h, _fp(t), _fp(t16), _fp(t32)))
        return t, t16, t32

    def close(self):
        if self._h:
            lib().hydro_session_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def query(frames, dtype: str, models: Sequence[ModelSpec], thresholds: np.ndarray, seg_len: int,
          policy: Policy, id_base: int = 0):
    """One-shot query through hydro_query."""
    cm = (Model * len(models))(*[m.to_c() for m in models])
    th = np.ascontiguousarray(thresholds, dtype=np.float32)
    if th.ndim == 1:
        th = th[None, :]
    fr = _frames_struct(frames, dtype, id_base)
    ptr = C.POINTER(C.c_int64)()
    n = C.c_int64()
    st = (PredStats * len(models))()
    _check(lib().hydro_query(C.byref(fr), cm, len(models), _fp(th), th.shape[0], int(seg_len), C.byref(policy),
                             C.byref(ptr), C.byref(n), st))
    ids = np.ctypeslib.as_array(ptr, shape=(n.value,)).copy() if n.value > 0 else np.zeros(0, np.int64)
    lib().hydro_free(ptr)
    return ids, _stats_list(st, len(models))


def query_noalloc(frames, dtype: str, models: Sequence[ModelSpec], thresholds: np.ndarray, seg_len: int,
                  policy: Policy, out_cap: int, id_base: int = 0):
    """One-shot query through hydro_query_noalloc (no device allocation; ids into a host array of
    out_cap entries).  Returns (ids, stats)."""
    cm = (Model * len(models))(*[m.to_c() for m in models])
    th = np.ascontiguousarray(thresholds, dtype=np.float32)
    if th.ndim == 1:
        th = th[None, :]
    fr = _frames_struct(frames, dtype, id_base)
    out = np.zeros(max(1, int(out_cap)), dtype=np.int64)
    n = C.c_int64()
    st = (PredStats * len(models))()
    _check(lib().hydro_query_noalloc(C.byref(fr), cm, len(models), _fp(th), th.shape[0], int(seg_len),
                                     C.byref(policy), out.ctypes.data_as(C.POINTER(C.c_int64)), int(out_cap),
                                     C.byref(n), st))
    return out[:n.value].copy(), _stats_list(st, len(models))


ROUTER_NPARAM = 192 * 64 + 64 + 64 * 8 + 8


def router_train_debug(k: int, feats_bf16: np.ndarray, pred: np.ndarray, rejected: np.ndarray,
                       params: np.ndarray, adam_m: np.ndarray, adam_v: np.ndarray, steps_done: int, lr: float):
    """One launch of the learned router's training kernel (see hydro_router_train_debug);
    returns updated copies of (params, adam_m, adam_v)."""
    f = np.ascontiguousarray(feats_bf16, dtype=np.uint16)
    pr = np.ascontiguousarray(pred, dtype=np.int32)
    rj = np.ascontiguousarray(rejected, dtype=np.uint8)
    p, m, v = (np.array(a, dtype=np.float32, copy=True) for a in (params, adam_m, adam_v))
    _check(lib().hydro_router_train_debug(int(k), f.ctypes.data_as(C.POINTER(C.c_uint16)),
                                          pr.ctypes.data_as(C.POINTER(C.c_int32)),
                                          rj.ctypes.data_as(C.POINTER(C.c_uint8)), int(f.shape[0]),
                                          _fp(p), _fp(m), _fp(v), int(steps_done), float(lr)))
    return p, m, v


def compaction_debug(k: int, n: int, pass_bits, out_ids, route: str = "fixed", wave: int = 1 << 20):
    """The routing / forwarding / result path on given outcomes (see hydro_compaction_debug).
    pass_bits: device tensor of k * ceil(n / 32) 32-bit words (row j = predicate j); out_ids:
    device int64 tensor of at least n elements.  Returns (result count, per-predicate stats,
    [fold + route, decide + forward, results, total] device ms)."""
    words = (int(n) + 31) // 32
    if int(n) > 0:
        if pass_bits.numel() * pass_bits.element_size() < 4 * k * words:
            raise ValueError("pass_bits holds fewer than k * ceil(n / 32) words")
        if out_ids.numel() < n or out_ids.element_size() != 8:
            raise ValueError("out_ids must hold n int64 values")
    cnt = C.c_int64()
    st = (PredStats * max(1, int(k)))()
    ms = (C.c_double * 4)()
    _check(lib().hydro_compaction_debug(int(k), int(n), C.c_void_p(pass_bits.data_ptr() if n > 0 else 0),
                                        ROUTES[route], int(wave), C.c_void_p(out_ids.data_ptr() if n > 0 else 0),
                                        C.byref(cnt), st, ms))
    return cnt.value, _stats_list(st, int(k)), list(ms)


def decode_routes(codes: np.ndarray) -> List[List[int]]:
    """Per-tuple visit sequences from the packed route log."""
    out = []
    for c in codes.tolist():
        seq = []
        while c:
            seq.append((c & 15) - 1)
            c >>= 4
        out.append(seq)
    return out
