"""The device frame generator writes the same bytes as the numpy recipe (both sides of every GPU
parity check read frames from one recipe)."""
import time

import numpy as np
import pytest

import hydro_synth as hs
from tests.gpu_util import log

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from hydro_synth import device as hd  # noqa: E402


@pytest.mark.parametrize("w,start,count", [(2, 1000, 2100), (5, 0, 1030), (5, 1046000, 2576)])
def test_device_frames_equal_numpy(w, start, count):
    cfg = hs.workload(w)
    dev = hd.make_frames_device(cfg, start, count, chunks_per_call=2)
    got = dev.cpu().numpy().view(hs.storage_dtype(cfg))
    want = hs.make_frames_parallel(cfg, start, count)
    bad = np.argwhere((got != want).reshape(count, -1).any(axis=1)).ravel()
    assert bad.size == 0, f"{bad.size} frames differ, first {start + bad[0]}"


def test_device_generation_rate():
    cfg = hs.workload(5)
    n = 65536
    out = torch.empty((n, cfg.hw, cfg.hw, 3), dtype=torch.uint8, device="cuda")
    hd.make_frames_device(cfg, 0, 1024, out=out[:1024])
    t = time.perf_counter()
    hd.make_frames_device(cfg, 0, n, out=out)
    dt = time.perf_counter() - t
    log(f"[gpu] device frame generator: {n / dt:.0f} frames/s of 128x128x3 u8 ({n * cfg.hw * cfg.hw * 3 / dt / 1e9:.2f} GB/s)")
    sample = out[n - 3:].cpu().numpy()
    assert np.array_equal(sample, hs.make_frames(cfg, n - 3, 3))
