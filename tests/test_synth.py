"""Seeded synthetic workloads: shapes, reproducibility and physical consistency."""

import numpy as np
import pytest

import oracle
import synth


def test_burst_frame_shapes_and_seed():
    a = synth.burst_frame()
    b = synth.burst_frame()
    assert a.x.shape == (8, 1024) and a.dirs.shape == (64, 3) and a.mic_pos.shape == (8, 3)
    assert np.array_equal(a.x, b.x) and np.array_equal(a.mic_pos, b.mic_pos)
    assert not np.array_equal(a.x, synth.burst_frame(seed_salt=1).x)
    assert np.all(np.hypot(a.mic_pos[:, 0], a.mic_pos[:, 1]) <= 0.025)
    np.testing.assert_allclose(np.linalg.norm(a.dirs, axis=1), 1.0)


def test_burst_frame_das_peaks_at_reflectors():
    """Delay-and-sum of the generated frame peaks within 1.5 grid steps of a reflector.

    The three echoes overlap in time, so only the global peak is checked; exact
    alignment of a single plane wave is pinned in the oracle tests.
    """
    f = synth.burst_frame()
    y = oracle.dmas_rows(f.x, f.mic_pos, f.dirs, f.fs, f.c, 1, use_cf=False)
    az_grid = np.linspace(-60, 60, 64)
    step = az_grid[1] - az_grid[0]
    best = az_grid[int(np.argmax(np.abs(y).max(axis=1)))]
    assert min(abs(best - r["az"]) for r in f.truth["reflectors"]) <= 1.5 * step


def test_ertis_frame_shapes():
    f = synth.ertis_frame()
    assert f.x.shape == (32, 16384) and f.dirs.shape == (91 * 46, 3)
    d = np.hypot(f.mic_pos[:, 0] - f.mic_pos[:, 0][:, None], f.mic_pos[:, 1] - f.mic_pos[:, 1][:, None])
    assert d[~np.eye(32, dtype=bool)].min() >= 0.004
    assert np.all(np.hypot(f.mic_pos[:, 0], f.mic_pos[:, 1]) <= 0.06)
    assert len(f.truth["reflectors"]) == 20 and f.order == 5 and f.use_cf
    assert np.isfinite(f.x).all() and np.abs(f.x).max() > 0


def test_nearfield_frame_shapes():
    f = synth.nearfield_frame(voxels=(8, 8, 4))
    assert f.x.shape == (1024, 2048) and f.dirs.shape == (256, 3) and f.nearfield
    assert f.dirs[:, 2].min() > 1.0 and f.dirs[:, 2].max() < 1.5


def test_serving_pool_mix():
    pool = synth.serving_pool(n_arrays_per_m=1, max_frames=6, sample_choices=(4096,), dir_choices=(1024, 2048))
    assert len(pool) == 6
    assert {f.num_mics for f in pool} <= {16, 32, 64}
    assert {f.order for f in pool} <= {3, 5}
    for f in pool:
        assert f.num_dirs in (1024, 2048) and f.num_samples == 4096


def test_hex_array_counts():
    """Hexagonal lattice with 5 mm edge: 1 cm radius holds 19 microphones."""
    assert synth.hex_disc_array(0.01).shape[0] == 19
