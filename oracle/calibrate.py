"""Choose each predicate's class subset and thresholds (TEST INFRASTRUCTURE).

Writes ``tests/golden/configs/<workload>.json``; the stored values come only
from this script, which calls only the oracle and the seeded input generator.

For every predicate of a workload, on ``calib_frames`` separate calibration
frames (own data seed), in fp64:

1. class subset S: classes sorted by how often they are the argmax (most
   frequent first, ties to the lower class); add classes while the cumulative
   argmax share stays <= the target selectivity r; at least one class, never
   all ten.  (The workloads only state "argmax in a class subset sized for
   selectivity r"; random networks are strongly class-skewed, so a subset alone
   cannot hit r and a threshold on the margin finishes the job.)
2. threshold for each segment s with target r_s: sort the calibration margins
   d ascending, i = round((1 - r_s) * n), theta = midpoint of d[i-1] and d[i],
   rounded to fp32.  The predicate then passes about r_s of the calibration
   frames.

Usage: python -m oracle.calibrate [workload ...]
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np

from hydro_synth import (GOLDEN_DIR, calibration_frames, make_model, predicate_table_path,
                         workload)

from .hydro_oracle import model_logits, predicate_margin


def choose_subset(z: np.ndarray, target: float) -> int:
    am = np.argmax(z, axis=1)
    freq = np.bincount(am, minlength=z.shape[1]) / z.shape[0]
    order = sorted(range(z.shape[1]), key=lambda c: (-freq[c], c))
    mask, cum = 0, 0.0
    for i, c in enumerate(order):
        if i == 0 or (cum + freq[c] <= target and i < z.shape[1] - 1):
            mask |= 1 << c
            cum += freq[c]
        else:
            break
    return mask


def threshold_for(d: np.ndarray, target: float) -> float:
    ds = np.sort(d[np.isfinite(d)])
    n = ds.size
    i = int(round((1.0 - target) * n))
    i = min(max(i, 1), n - 1)
    return float(np.float32(0.5 * (ds[i - 1] + ds[i])))


def calibrate(index: int) -> dict:
    cfg = workload(index)
    frames = calibration_frames(cfg)
    masks, theta = [], np.zeros((cfg.n_seg, cfg.k), dtype=np.float32)
    for j, desc in enumerate(cfg.models):
        z = model_logits(make_model(desc), frames, cfg.dtype)
        r_ref = cfg.targets[0][j]
        mask = choose_subset(z, r_ref)
        d = predicate_margin(z, mask)
        masks.append(mask)
        for s in range(cfg.n_seg):
            theta[s, j] = threshold_for(d, cfg.targets[s][j])
    return {"workload": cfg.name, "class_masks": masks,
            "thresholds": [[float(v) for v in row] for row in theta],
            "targets": [list(t) for t in cfg.targets],
            "calib_frames": cfg.calib_frames,
            "calib_seed": cfg.data_seed + cfg.calib_seed_offset}


def main(argv):
    idx = [int(a) for a in argv] or [1, 2, 3, 5]
    os.makedirs(GOLDEN_DIR, exist_ok=True)
    for i in idx:
        cfg = workload(i)
        if cfg.predicates_from:
            print(f"workload {i} shares predicates with {cfg.predicates_from}")
            continue
        d = calibrate(i)
        with open(predicate_table_path(cfg), "w") as f:
            json.dump(d, f, indent=1)
        print(f"workload {i}: masks {d['class_masks']} thresholds {d['thresholds']}")


if __name__ == "__main__":
    main(sys.argv[1:])
