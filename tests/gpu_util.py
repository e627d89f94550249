"""Shared helpers of the GPU parity tests (oracle side computed on the CPU)."""
import functools
import sys

import numpy as np

import hydro_synth as hs
from oracle import hydro_oracle as ho


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


class Case:
    """A workload prefix with its oracle truth table."""

    def __init__(self, wl: int, n: int, start: int = 0, logits: bool = False):
        self.cfg = cfg = hs.workload(wl)
        self.n, self.start = n, start
        self.frames = hs.make_frames_parallel(cfg, start, n)
        self.pt = hs.load_predicates(cfg)
        self.weights = [hs.make_model(d) for d in cfg.models]
        self.seg_len = cfg.n // cfg.n_seg
        out = ho.truth_table(self.frames, cfg.dtype, self.weights, self.pt.class_masks, self.pt.thresholds,
                             self.seg_len, id_base=start, return_logits=logits)
        self.P, self.D = out[0], out[1]
        self.Z = out[2] if logits else None
        self.expect = ho.result_ids(self.P, id_base=start)
        self.flops = [d.flops() for d in cfg.models]
        # near-tie audit: "bit-exact against FP64" is well defined only when no margin lies within
        # FP64 summation-order noise of its threshold
        self.gap = ho.near_tie_gap(self.D, self.pt.thresholds, self.seg_len, id_base=start)
        assert self.gap > 1e-9, f"workload {wl} [{start}, {start + n}): margin within {self.gap:.3g} of a threshold"

    def specs(self):
        from paper_2403_14902_amd import hydro
        return [hydro.ModelSpec.from_weights(w, m) for w, m in zip(self.weights, self.pt.class_masks)]

    def device_frames(self):
        import torch
        return torch.from_numpy(self.frames).cuda()


@functools.lru_cache(maxsize=8)
def case(wl: int, n: int, start: int = 0, logits: bool = False) -> Case:
    log(f"[oracle] workload {wl} tuples [{start}, {start + n}) ...")
    c = Case(wl, n, start, logits)
    log(f"[oracle] workload {wl}: |R| = {c.expect.size}, min |d - theta| = {c.gap:.3g}")
    return c


def check_stats(stats, n, n_result):
    ev = [s["evaluated"] for s in stats]
    ps = [s["passed"] for s in stats]
    bad = ho.stats_invariants(ev, ps, n, n_result)
    assert bad == [], bad
