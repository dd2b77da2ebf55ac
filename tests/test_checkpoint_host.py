"""Host logic of the frame-granular checkpoints (no GPU): a stand-in job that
keeps its exit store in numpy records which frames were computed."""
import json

import numpy as np
import pytest

from paper_2602_10064_amd.checkpoint import run_with_checkpoints


from paper_2602_10064_amd import workloads as w


class FakeJob:
    def __init__(self, n_probes=2, n_frames=10, ny=3, nx=4, seed=7, aberrations=None):
        self.n_probes, self.n_frames, self.ny, self.nx = n_probes, n_frames, ny, nx
        # the description the digest reads (the stand-in's waves do not depend on it)
        self.job = w.random_small_job(seed, nx=nx, ny=ny, n_frames=n_frames, aperture_mrad=20.0,
                                      n_probes=n_probes)
        self.aberrations = aberrations
        self.store = np.zeros((n_probes, n_frames, ny, nx), np.complex64)
        self.present = np.zeros(n_frames, bool)
        self.computed = []
        self.finished = False

    def _wave(self, f):
        return (f + 1) * (1 + 1j) * np.ones((self.n_probes, self.ny, self.nx), np.complex64)

    def run_frames(self, f0, f1, stream=None):
        for f in range(f0, f1):
            self.store[:, f] = self._wave(f)
            self.computed.append(f)
        self.present[f0:f1] = True

    def exit_frames(self, f0, f1):
        assert self.present[f0:f1].all()
        return self.store[:, f0:f1].copy()

    def put_exit_frames(self, f0, waves):
        self.store[:, f0:f0 + waves.shape[1]] = waves
        self.present[f0:f0 + waves.shape[1]] = True

    def finish(self, stream=None):
        assert self.present.all()
        self.finished = True


def test_restart_computes_only_missing_chunks(tmp_path):
    a = FakeJob()
    assert run_with_checkpoints(a, str(tmp_path), 4) == 3          # chunks 0-3, 4-7, 8-9
    assert a.finished and a.computed == list(range(10))
    (tmp_path / "frames_000004_000008.npy").unlink()                # an interrupted run
    b = FakeJob()
    assert run_with_checkpoints(b, str(tmp_path), 4) == 1
    assert b.computed == [4, 5, 6, 7]
    assert np.array_equal(b.store, a.store) and b.finished
    assert json.loads((tmp_path / "manifest.json").read_text())["chunk_frames"] == 4


def test_other_job_or_chunking_is_refused(tmp_path):
    run_with_checkpoints(FakeJob(), str(tmp_path), 4)
    with pytest.raises(ValueError):
        run_with_checkpoints(FakeJob(n_frames=12), str(tmp_path), 4)
    with pytest.raises(ValueError):
        run_with_checkpoints(FakeJob(), str(tmp_path), 5)
    with pytest.raises(ValueError):
        run_with_checkpoints(FakeJob(), str(tmp_path / "x"), 0)


def test_changed_job_in_same_directory_is_refused(tmp_path):
    # same exit-store shape and chunking, different inputs: restoring the first
    # job's waves would give a wrong spectrum silently
    run_with_checkpoints(FakeJob(), str(tmp_path), 4)
    assert run_with_checkpoints(FakeJob(), str(tmp_path), 4) == 0       # the same job restores
    with pytest.raises(ValueError):
        run_with_checkpoints(FakeJob(seed=8), str(tmp_path), 4)         # another trajectory
    other = FakeJob()
    other.job = other.job.replace(voltage_V=200e3)
    with pytest.raises(ValueError):
        run_with_checkpoints(other, str(tmp_path), 4)
    ab = (np.r_[50.0, np.zeros(13)], np.zeros(14))
    with pytest.raises(ValueError):
        run_with_checkpoints(FakeJob(aberrations=ab), str(tmp_path), 4)
    moved = FakeJob()
    moved.job = moved.job.replace(probe_xy=moved.job.probe_xy + 0.1)
    with pytest.raises(ValueError):
        run_with_checkpoints(moved, str(tmp_path), 4)
