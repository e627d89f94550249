"""Seeded synthetic inputs for the conjunctive ML-UDF query.

This module produces the *inputs* of a query: frames, predicate model weights
and the static description of each workload (sizes, widths, target
selectivities, segment layout).  It holds none of the method's arithmetic: no
forward pass, no margin, no decision, no routing.  Class subsets and
thresholds are calibrated by the oracle and stored as data files under
``tests/golden/configs``; they are only *read* here.

Both sides of the parity check use this module: the FP64 CPU oracle and the
HIP path (tests, bench).  Nothing here imports either of them.

Frame recipe (structured, low-frequency content so that a random GAP-CNN gives
frame-dependent margins): per frame, z ~ N(0,1)^{3x8x8}, U = bilinear upsample
to HxH with half-pixel centres (two taps per axis, elementwise fp64 operations in
a fixed order, so the frames do not depend on the machine's BLAS), e ~ U[-1,1]
iid per pixel value; frame = clip(0.5 + 0.25*U(z) + 0.10*e, 0, 1), stored NHWC and quantised to
bf16 (fp64 -> fp32 RNE -> bf16 RNE) or uint8 (round-half-even of 255*x).
The small MLP workload uses iid uniform[0,1) fp32 frames instead.

Random streams are split in chunks of ``CHUNK`` frames, each seeded by
``SeedSequence([data_seed, chunk])``, so any chunk of a large stream can be
regenerated on its own.
"""
from __future__ import annotations

import json
import os
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

CHUNK = 1024           # frames per independently seeded chunk
N_CLASSES = 10         # every predicate model ends in 10 logits

DTYPE_F32 = "f32"
DTYPE_BF16 = "bf16"
DTYPE_U8 = "u8"

GOLDEN_DIR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                          "tests", "golden", "configs")


# --------------------------------------------------------------------------
# Workload descriptions
# --------------------------------------------------------------------------
@dataclass
class ModelDesc:
    """Architecture of one predicate model (weights come from ``make_model``)."""
    arch: str                    # "mlp" or "cnn"
    seed: int
    # mlp
    d_in: int = 0
    hidden: int = 0
    # cnn: input is in_hw x in_hw x 3; conv3x3 stride 2 pad 1 + ReLU per width
    in_hw: int = 0
    widths: Tuple[int, ...] = ()

    def flops(self) -> float:
        """Multiply-add FLOPs (2 per MAC) of one evaluation of this model."""
        if self.arch == "mlp":
            return 2.0 * (self.d_in * self.hidden + self.hidden * N_CLASSES)
        f = 0.0
        hw, cin = self.in_hw, 3
        for co in self.widths:
            hw //= 2
            f += 2.0 * hw * hw * co * cin * 9
            cin = co
        return f + 2.0 * cin * N_CLASSES


@dataclass
class WorkloadConfig:
    name: str
    index: int                   # 1-based workload number
    n: int                       # tuples (frames)
    hw: int                      # frame height = width
    dtype: str                   # f32 | bf16 | u8
    data_seed: int
    models: List[ModelDesc]
    targets: List[Tuple[float, ...]]   # per segment: target selectivity of each predicate
    frame_kind: str = "structured"     # "uniform" (iid U[0,1)) or "structured" (recipe G)
    predicates_from: Optional[str] = None   # share class subsets/thresholds with another workload
    push_batch: int = 0          # frames per host->device push (0 = device resident)
    calib_frames: int = 8192
    calib_seed_offset: int = 7777

    @property
    def k(self) -> int:
        return len(self.models)

    @property
    def n_seg(self) -> int:
        return len(self.targets)

    @property
    def frame_bytes(self) -> int:
        return self.hw * self.hw * 3 * {DTYPE_F32: 4, DTYPE_BF16: 2, DTYPE_U8: 1}[self.dtype]


def _cnn(seed, hw, widths):
    return ModelDesc(arch="cnn", seed=seed, in_hw=hw, widths=tuple(widths))


def _mlp(seed, d, h):
    return ModelDesc(arch="mlp", seed=seed, d_in=d, hidden=h)


def _drift_targets(base=(0.5, 0.2, 0.8), n_seg=8):
    import itertools
    perms = list(itertools.permutations(base))
    return [tuple(perms[s % len(perms)]) for s in range(n_seg)]


def workload(index: int) -> WorkloadConfig:
    """The five synthetic workloads, numbered 1..5."""
    if index == 1:
        return WorkloadConfig(
            name="mlp2_uniform32", index=1, n=2048, hw=32, dtype=DTYPE_F32, data_seed=1,
            models=[_mlp(1000 * 1 + k, 3072, 256) for k in range(2)],
            targets=[(0.3, 0.6)], frame_kind="uniform")
    if index == 2:
        return WorkloadConfig(
            name="cnn3_drift64", index=2, n=65536, hw=64, dtype=DTYPE_BF16, data_seed=2,
            models=[_cnn(1000 * 2 + k, 64, [16 * m, 32 * m, 64 * m]) for k, m in enumerate((1, 2, 4))],
            targets=_drift_targets())
    if index == 3:
        hs = (256, 512, 768, 1024, 1536, 2048)
        return WorkloadConfig(
            name="mlp6_batched64", index=3, n=262144, hw=64, dtype=DTYPE_BF16, data_seed=3,
            models=[_mlp(1000 * 3 + k, 12288, h) for k, h in enumerate(hs)],
            targets=[(0.58, 0.90, 0.10, 0.74, 0.26, 0.42)])
    if index == 4:
        base = workload(2)
        return WorkloadConfig(
            name="cnn3_drift64_large", index=4, n=524288, hw=64, dtype=DTYPE_BF16, data_seed=4,
            models=base.models, targets=base.targets, predicates_from=base.name)
    if index == 5:
        return WorkloadConfig(
            name="cnn4_u8_128", index=5, n=1048576, hw=128, dtype=DTYPE_U8, data_seed=5,
            models=[_cnn(1000 * 5 + k, 128, [32, 64, 128, 256]) for k in range(4)],
            targets=[(0.8, 0.6, 0.4, 0.2)], push_batch=16384)
    raise ValueError(f"unknown workload {index}")


ALL_WORKLOADS = (1, 2, 3, 4, 5)


# --------------------------------------------------------------------------
# Frames
# --------------------------------------------------------------------------
def _upsample_matrix(src: int, dst: int) -> np.ndarray:
    """Bilinear interpolation matrix A (dst x src), half-pixel centres, edge clamp."""
    a = np.zeros((dst, src), dtype=np.float64)
    scale = src / dst
    for i in range(dst):
        s = (i + 0.5) * scale - 0.5
        s = min(max(s, 0.0), src - 1.0)
        lo = int(np.floor(s))
        hi = min(lo + 1, src - 1)
        w = s - lo
        a[i, lo] += 1.0 - w
        a[i, hi] += w
    return a


def _upsample_taps(src: int, dst: int):
    """The two taps of every output index of the interpolation matrix: (lo, hi, w_lo, w_hi),
    with w_hi = 0 where the edge clamp leaves a single tap."""
    a = _upsample_matrix(src, dst)
    rows = np.arange(dst)
    lo = np.argmax(a != 0.0, axis=1)
    hi = np.minimum(lo + 1, src - 1)
    w_lo = a[rows, lo]
    w_hi = np.where(hi != lo, a[rows, hi], 0.0)
    return lo, hi, w_lo, w_hi


def _upsample(z: np.ndarray, dst: int) -> np.ndarray:
    """Bilinear upsample of z [n][3][8][8] to [n][dst][dst][3] (NHWC), columns then rows.

    Every output is the two-tap sum w_lo * v[lo] + w_hi * v[hi] of the interpolation matrix's
    nonzero entries, built from elementwise fp64 multiplies and adds only (no BLAS), so the frames
    are bit-identical on every machine and thread count.
    """
    src = z.shape[-1]
    lo, hi, w_lo, w_hi = _upsample_taps(src, dst)
    zt = z.transpose(0, 2, 3, 1)                                           # n, i, j, c
    t = (w_lo[None, None, :, None] * np.take(zt, lo, axis=2)
         + w_hi[None, None, :, None] * np.take(zt, hi, axis=2))           # n, i, x, c
    return (w_lo[None, :, None, None] * np.take(t, lo, axis=1)
            + w_hi[None, :, None, None] * np.take(t, hi, axis=1))         # n, y, x, c


def f64_to_bf16_bits(x: np.ndarray) -> np.ndarray:
    """fp64 -> fp32 (round to nearest even) -> bf16 (round to nearest even), as uint16 bits."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return r.astype(np.uint16)


def _chunk_frames(cfg: WorkloadConfig, chunk: int, data_seed: int) -> np.ndarray:
    """All CHUNK frames of one chunk, in storage dtype (f32, bf16 bits as uint16, or uint8)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([data_seed, chunk])))
    hw = cfg.hw
    if cfg.frame_kind == "uniform":
        x = rng.random((CHUNK, hw, hw, 3))                       # U[0,1) fp64
        return x.astype(np.float32)
    z = rng.standard_normal((CHUNK, 3, 8, 8))
    e = rng.uniform(-1.0, 1.0, size=(CHUNK, hw, hw, 3))
    up = _upsample(z, hw)                                       # (n, hw, hw, 3)
    x = np.clip(0.5 + 0.25 * up + 0.10 * e, 0.0, 1.0)
    if cfg.dtype == DTYPE_BF16:
        return f64_to_bf16_bits(x)
    if cfg.dtype == DTYPE_U8:
        return np.rint(255.0 * x).astype(np.uint8)
    return x.astype(np.float32)


def storage_dtype(cfg: WorkloadConfig):
    return {DTYPE_F32: np.float32, DTYPE_BF16: np.uint16, DTYPE_U8: np.uint8}[cfg.dtype]


def make_frames(cfg: WorkloadConfig, start: int = 0, count: Optional[int] = None,
                data_seed: Optional[int] = None, out: Optional[np.ndarray] = None) -> np.ndarray:
    """Frames [start, start+count) of the workload's stream, NHWC, storage dtype.

    bf16 frames are returned as their uint16 bit patterns.
    """
    if count is None:
        count = cfg.n - start
    seed = cfg.data_seed if data_seed is None else data_seed
    if out is None:
        out = np.empty((count, cfg.hw, cfg.hw, 3), dtype=storage_dtype(cfg))
    c0, c1 = start // CHUNK, (start + count + CHUNK - 1) // CHUNK
    for c in range(c0, c1):
        blk = _chunk_frames(cfg, c, seed)
        lo = max(start, c * CHUNK)
        hi = min(start + count, (c + 1) * CHUNK)
        out[lo - start:hi - start] = blk[lo - c * CHUNK:hi - c * CHUNK]
    return out


def make_frames_parallel(cfg: WorkloadConfig, start: int = 0, count: Optional[int] = None,
                         data_seed: Optional[int] = None, workers: int = 0,
                         out: Optional[np.ndarray] = None) -> np.ndarray:
    """Same values as ``make_frames``; chunks are produced by a thread pool."""
    from concurrent.futures import ThreadPoolExecutor
    if count is None:
        count = cfg.n - start
    if out is None:
        out = np.empty((count, cfg.hw, cfg.hw, 3), dtype=storage_dtype(cfg))
    if workers <= 0:
        workers = min(16, os.cpu_count() or 1)
    c0, c1 = start // CHUNK, (start + count + CHUNK - 1) // CHUNK

    def job(c):
        lo = max(start, c * CHUNK)
        hi = min(start + count, (c + 1) * CHUNK)
        make_frames(cfg, lo, hi - lo, data_seed, out=out[lo - start:hi - start])

    with ThreadPoolExecutor(workers) as ex:
        list(ex.map(job, range(c0, c1)))
    return out


def calibration_frames(cfg: WorkloadConfig) -> np.ndarray:
    return make_frames(cfg, 0, cfg.calib_frames, data_seed=cfg.data_seed + cfg.calib_seed_offset)


# --------------------------------------------------------------------------
# Predicate models
# --------------------------------------------------------------------------
@dataclass
class ModelWeights:
    desc: ModelDesc
    # mlp: W1 [D][h], b1 [h], W2 [h][10], b2 [10]
    # cnn: convs = [(W [co][ci][3][3], b [co]) ...], fc = (W [c_last][10], b [10])
    tensors: dict = field(default_factory=dict)


def _he(rng, shape, fan_in):
    return (rng.standard_normal(shape) * np.sqrt(2.0 / fan_in)).astype(np.float32)


def _bias(rng, n):
    return rng.uniform(-0.05, 0.05, size=n).astype(np.float32)


def make_model(desc: ModelDesc) -> ModelWeights:
    """He-normal fp32 weights and small uniform biases, drawn in fp64 from PCG64(seed).

    Draw order is fixed: MLP (W1, b1, W2, b2); CNN per layer (W, b) then (Wfc, bfc).
    """
    rng = np.random.Generator(np.random.PCG64(desc.seed))
    t = {}
    if desc.arch == "mlp":
        t["W1"] = _he(rng, (desc.d_in, desc.hidden), desc.d_in)
        t["b1"] = _bias(rng, desc.hidden)
        t["W2"] = _he(rng, (desc.hidden, N_CLASSES), desc.hidden)
        t["b2"] = _bias(rng, N_CLASSES)
    else:
        cin = 3
        convs = []
        for co in desc.widths:
            w = _he(rng, (co, cin, 3, 3), cin * 9)
            b = _bias(rng, co)
            convs.append((w, b))
            cin = co
        t["convs"] = convs
        t["Wfc"] = _he(rng, (cin, N_CLASSES), cin)
        t["bfc"] = _bias(rng, N_CLASSES)
    return ModelWeights(desc=desc, tensors=t)


# --------------------------------------------------------------------------
# Calibrated predicate tables (written by the oracle's calibration script)
# --------------------------------------------------------------------------
@dataclass
class PredicateTable:
    class_masks: List[int]          # per predicate: bit c set <=> class c in the subset
    thresholds: np.ndarray          # fp32 [n_seg][K]


def predicate_table_path(cfg: WorkloadConfig) -> str:
    name = cfg.predicates_from or cfg.name
    return os.path.join(GOLDEN_DIR, f"{name}.json")


def load_predicates(cfg: WorkloadConfig) -> PredicateTable:
    with open(predicate_table_path(cfg)) as f:
        d = json.load(f)
    th = np.array(d["thresholds"], dtype=np.float32).reshape(len(d["thresholds"]), -1)
    return PredicateTable(class_masks=[int(m) for m in d["class_masks"]], thresholds=th)


def segment_of(cfg: WorkloadConfig, ids: np.ndarray) -> np.ndarray:
    """Segment index of each tuple id: segment s covers [s*n/n_seg, (s+1)*n/n_seg)."""
    seg_len = cfg.n // cfg.n_seg
    return np.minimum(np.asarray(ids) // seg_len, cfg.n_seg - 1)
