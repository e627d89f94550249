"""Structured frames written straight into device memory (or evaluated on the host by the same
compiled code), bit-identical to ``hydro_synth.make_frames``.

The numpy recipe draws, per chunk of ``CHUNK`` frames, the low-frequency field z and then one
uniform double per frame value from the chunk's PCG64 stream.  Here the host still draws z (and
reads the stream's state right after it); ``framegen.hip`` jumps the stream ahead to each frame
row and evaluates the noise, the upsample, the clip and the quantisation with the same fp64
operations in the same order.  Only the structured bf16 / uint8 workloads are supported (the
uniform fp32 workload is small enough for numpy).
"""
from __future__ import annotations

import ctypes
import os
from concurrent.futures import ThreadPoolExecutor
from typing import Optional

import numpy as np

from . import CHUNK, DTYPE_BF16, DTYPE_U8, WorkloadConfig, _upsample_taps, storage_dtype

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhydro_synth.so")
_DT = {DTYPE_BF16: 1, DTYPE_U8: 2}
_M64 = (1 << 64) - 1
_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with hydro_synth.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        args = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int64,
                ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                ctypes.c_void_p, ctypes.c_void_p]
        L.hs_frames_host.argtypes = args
        L.hs_frames_host.restype = ctypes.c_int
        L.hs_frames_device.argtypes = args + [ctypes.c_void_p]
        L.hs_frames_device.restype = ctypes.c_int
        L.hs_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def chunk_field_and_state(chunk: int, data_seed: int):
    """z [CHUNK][3][8][8] of one chunk and its PCG64 state after drawing z, as
    (state lo, state hi, increment lo, increment hi)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([data_seed, chunk])))
    z = rng.standard_normal((CHUNK, 3, 8, 8))
    st = rng.bit_generator.state["state"]
    s, inc = int(st["state"]), int(st["inc"])
    return z, np.array([s & _M64, s >> 64, inc & _M64, inc >> 64], dtype=np.uint64)


def _prepare(cfg: WorkloadConfig, c0: int, c1: int, data_seed: int, workers: int):
    if cfg.frame_kind == "uniform" or cfg.dtype not in _DT:
        raise ValueError(f"workload {cfg.name}: only structured bf16 / uint8 frames are generated here")
    z = np.empty((c1 - c0, CHUNK, 3, 8, 8), dtype=np.float64)
    st = np.empty((c1 - c0, 4), dtype=np.uint64)

    def job(c):
        z[c - c0], st[c - c0] = chunk_field_and_state(c, data_seed)

    with ThreadPoolExecutor(max(1, workers)) as ex:
        list(ex.map(job, range(c0, c1)))
    lo, hi, w_lo, w_hi = _upsample_taps(8, cfg.hw)
    tabs = (np.ascontiguousarray(w_lo, dtype=np.float64), np.ascontiguousarray(w_hi, dtype=np.float64),
            np.ascontiguousarray(lo, dtype=np.int32), np.ascontiguousarray(hi, dtype=np.int32))
    return z, st, tabs


def make_frames_host(cfg: WorkloadConfig, start: int, count: int, data_seed: Optional[int] = None) -> np.ndarray:
    """Frames [start, start + count) evaluated on the host by the compiled generator."""
    seed = cfg.data_seed if data_seed is None else data_seed
    out = np.empty((count, cfg.hw, cfg.hw, 3), dtype=storage_dtype(cfg))
    if count == 0:
        return out
    c0, c1 = start // CHUNK, (start + count + CHUNK - 1) // CHUNK
    z, st, (w_lo, w_hi, lo, hi) = _prepare(cfg, c0, c1, seed, 4)
    rc = lib().hs_frames_host(_DT[cfg.dtype], cfg.hw, CHUNK, c1 - c0, start - c0 * CHUNK, count,
                              z.ctypes.data, st.ctypes.data, w_lo.ctypes.data, w_hi.ctypes.data,
                              lo.ctypes.data, hi.ctypes.data, out.ctypes.data)
    if rc != 0:
        raise RuntimeError(lib().hs_last_error().decode())
    return out


def make_frames_device(cfg: WorkloadConfig, start: int, count: int, out=None, data_seed: Optional[int] = None,
                       chunks_per_call: int = 64, workers: int = 16, progress=None):
    """Frames [start, start + count) generated on the current CUDA device into `out` (a torch
    tensor [count][hw][hw][3] of the storage dtype, allocated when None); returns `out`.
    Synchronises the current stream after every call of `chunks_per_call` chunks."""
    import torch
    seed = cfg.data_seed if data_seed is None else data_seed
    tdt = {DTYPE_BF16: torch.int16, DTYPE_U8: torch.uint8}[cfg.dtype]
    if out is None:
        out = torch.empty((count, cfg.hw, cfg.hw, 3), dtype=tdt, device="cuda")
    assert out.is_cuda and out.is_contiguous() and tuple(out.shape) == (count, cfg.hw, cfg.hw, 3)
    assert out.element_size() == np.dtype(storage_dtype(cfg)).itemsize
    stream = torch.cuda.current_stream().cuda_stream
    pos = start
    while pos < start + count:
        c0 = pos // CHUNK
        c1 = min(c0 + chunks_per_call, (start + count + CHUNK - 1) // CHUNK)
        n = min(c1 * CHUNK, start + count) - pos
        z, st, tabs = _prepare(cfg, c0, c1, seed, workers)
        dz = torch.from_numpy(z).cuda()
        dst = torch.from_numpy(st.view(np.int64)).cuda()
        dt = [torch.from_numpy(t).cuda() for t in tabs]
        dst_out = out[pos - start:pos - start + n]
        rc = lib().hs_frames_device(_DT[cfg.dtype], cfg.hw, CHUNK, c1 - c0, pos - c0 * CHUNK, n,
                                    dz.data_ptr(), dst.data_ptr(), dt[0].data_ptr(), dt[1].data_ptr(),
                                    dt[2].data_ptr(), dt[3].data_ptr(), dst_out.data_ptr(), stream)
        if rc != 0:
            raise RuntimeError(lib().hs_last_error().decode())
        torch.cuda.current_stream().synchronize()
        pos += n
        if progress is not None:
            progress(pos - start, count)
    return out
