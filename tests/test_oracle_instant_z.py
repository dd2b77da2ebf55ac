"""Pins of the per-frame slice binning (atoms within each frame's slice
z-bounds, Methods 2.2) against the frame-mean binning the path uses by
default."""
import dataclasses

import numpy as np

from oracle import tacaw_oracle as o
from paper_2602_10064_amd import workloads as w


def straddling_job(seed, n_frames=6):
    # atoms oscillating across slice boundaries (dz = 1 A)
    job = w.random_small_job(seed, nx=24, ny=24, n_slices=4, n_frames=n_frames, n_atoms=6, cell=(5.0, 5.0, 4.0))
    rng = np.random.default_rng(seed)
    pos = job.positions.copy()
    bound = rng.integers(1, 4, size=job.n_atoms).astype(float)
    t = np.arange(n_frames)[:, None]
    pos[:, :, 2] = bound[None, :] + 0.3 * np.sin(2 * np.pi * t / n_frames + rng.uniform(0, 6, job.n_atoms)[None])
    return dataclasses.replace(job, positions=pos, slice_by_instant_z=True)


def test_instant_binning_by_hand():
    pos = np.zeros((3, 2, 3))
    pos[:, 0, 2] = [0.9, 1.1, 0.95]      # crosses the boundary at 1.0 (dz = 1)
    pos[:, 1, 2] = [3.99, 4.01, 2.5]     # wraps past Lz = 4 back to slice 0
    inst = o.slice_index(pos, 4.0, 4, instant=True)
    assert inst.tolist() == [[0, 3], [1, 0], [0, 2]]
    assert o.slice_index(pos, 4.0, 4).tolist() == [0, 3]      # means 0.983 and 3.5


def test_instant_frame_equals_a_one_frame_job():
    # with one frame the mean z is that frame's z, so each frame of the
    # per-frame binning equals a one-frame job binned by its mean
    job = straddling_job(7)
    ex = o.exit_waves(job)
    for f in range(job.n_frames):
        single = dataclasses.replace(job, positions=job.positions[f:f + 1].copy(), slice_by_instant_z=False)
        assert np.allclose(ex[:, f:f + 1], o.exit_waves(single), atol=1e-13)
    # and the binnings do differ on this trajectory
    mean = o.exit_waves(dataclasses.replace(job, slice_by_instant_z=False))
    assert np.max(np.abs(mean - ex)) > 1e-6


def test_instant_equals_mean_when_no_atom_crosses():
    job = w.random_small_job(8, nx=16, ny=16, n_slices=3, n_frames=4, n_atoms=5)
    a = o.exit_waves(job)
    b = o.exit_waves(dataclasses.replace(job, slice_by_instant_z=True))
    assert np.array_equal(a, b)
