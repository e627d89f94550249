"""The seeded input generator: frames are bit-identical whatever the machine, its BLAS or the
number of threads (the predicate tables under tests/golden were calibrated on these frames, and
the GPU path and the oracle must see the same bytes).  CPU only."""
import hashlib

import numpy as np
import pytest

import hydro_synth as hs

# sha256 of the first 256 frames of three workloads (fp32 uniform, bf16 structured, uint8 128x128)
FRAME_SHA = {
    1: "02237e6bc14e4b58048018b42969dd4191fd77969f010e031f3120fab0090369",
    2: "e6f1eba7b7b63b6b2d46ed69aa11fb9bb92306e57c8b4dca891f752d3c4cb2b0",
    5: "97bcbe2f1f7da5ab827d4c7913fefdd76d342a6a82893a4e3dfb97e7f8c853d7",
}


@pytest.mark.parametrize("w", sorted(FRAME_SHA))
def test_frames_bit_reproducible(w):
    cfg = hs.workload(w)
    assert hashlib.sha256(hs.make_frames(cfg, 0, 256).tobytes()).hexdigest() == FRAME_SHA[w]


def test_parallel_generation_matches_serial():
    cfg = hs.workload(2)
    a = hs.make_frames(cfg, 1000, 1500)
    for workers in (1, 3, 8):
        assert np.array_equal(hs.make_frames_parallel(cfg, 1000, 1500, workers=workers), a)


@pytest.mark.parametrize("dst", [32, 64, 128])
def test_two_tap_upsample_equals_interpolation_matrix(dst):
    """The two-tap evaluation is the dense product A z A^T with the interpolation matrix, to
    rounding (each output is a convex combination of at most four source values)."""
    z = np.random.default_rng(dst).standard_normal((5, 3, 8, 8))
    a = hs._upsample_matrix(8, dst)
    assert np.allclose(a.sum(axis=1), 1.0) and ((a != 0).sum(axis=1) <= 2).all()
    dense = np.einsum("yi,ncij,xj->nyxc", a, z, a)
    assert np.abs(hs._upsample(z, dst) - dense).max() < 1e-13


# ---------------------------------------------------------------- compiled frame generator
@pytest.fixture(scope="module")
def framegen():
    from hydro_synth import build, device
    if not __import__("os").path.exists(device.LIB_PATH):
        build.build()
    return device


@pytest.mark.parametrize("w,start,count", [(2, 0, 3), (2, 1022, 4), (4, 524286, 2), (5, 0, 2), (5, 3071, 3),
                                           (5, 1048574, 2)])
def test_compiled_generator_equals_numpy(framegen, w, start, count):
    """The compiled generator (PCG64 jump-ahead to each frame row, the same fp64 expressions) is
    bit-identical to the numpy recipe, across chunk boundaries and at the end of the largest stream."""
    cfg = hs.workload(w)
    assert np.array_equal(framegen.make_frames_host(cfg, start, count), hs.make_frames(cfg, start, count))


def test_compiled_generator_calibration_seed(framegen):
    cfg = hs.workload(5)
    seed = cfg.data_seed + cfg.calib_seed_offset
    assert np.array_equal(framegen.make_frames_host(cfg, 2047, 2, data_seed=seed),
                          hs.make_frames(cfg, 2047, 2, data_seed=seed))


def test_pcg_jump_ahead_matches_stepping(framegen):
    """A planted check of the draw positions: frame 1 of a chunk is not frame 0 of it."""
    cfg = hs.workload(5)
    a = framegen.make_frames_host(cfg, 0, 2)
    assert not np.array_equal(a[0], a[1])
