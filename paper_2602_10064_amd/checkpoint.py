"""Frame-granular checkpoints of a job's exit waves (Methods 2.1 "Workflow
Architecture": exit waves are cached per frame so that an interrupted run
restarts without recomputing finished frames).

The job runs in chunks of frames.  After each chunk its exit waves go to one
.npy file in the checkpoint directory; a later run of the same job restores
the chunks whose files exist (numpy.load without pickles) and computes only
the rest, then runs the time stage.  The directory belongs to one job: its
manifest records the exit-store shape, the chunk size and a digest of every
input that decides the exit waves, and a mismatch is an error.
"""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np


def job_digest(job) -> str:
    """SHA-256 of every input that decides a job's exit waves: the cell, grids,
    slices, beam, frame spacing, positions, species, form-factor coefficients,
    probes, binning rule and probe aberrations.  `job` is a TacawJob (its
    description `.job` and current `.aberrations`)."""
    d = job.job
    h = hashlib.sha256()

    def arr(x, dtype):
        a = np.ascontiguousarray(x, dtype=dtype)
        h.update(repr(a.shape).encode())
        h.update(a.tobytes())

    arr(d.cell, np.float64)
    h.update(repr((int(d.nx), int(d.ny), int(d.n_slices), int(d.pot_nx), int(d.pot_ny),
                   float(d.voltage_V), float(d.aperture_mrad), float(d.dt_fs),
                   bool(getattr(d, "slice_by_instant_z", False)))).encode())
    arr(d.positions, np.float64)
    arr(d.atom_species, np.int32)
    arr(d.species_Z, np.int32)
    arr(d.gauss_a, np.float64)
    arr(d.gauss_b, np.float64)
    arr(d.probe_xy if d.aperture_mrad > 0 else np.zeros((0, 2)), np.float64)
    ab = getattr(job, "aberrations", None)
    if ab is None:
        h.update(b"no aberrations")
    else:
        arr(ab[0], np.float64)
        arr(ab[1], np.float64)
    return h.hexdigest()


def run_with_checkpoints(job, directory: str, chunk_frames: int, stream=None) -> int:
    """Run a TacawJob chunk by chunk with per-chunk exit-wave files; returns the
    number of chunks computed (the others were restored)."""
    if chunk_frames < 1:
        raise ValueError("chunk_frames must be positive")
    os.makedirs(directory, exist_ok=True)
    shape = [int(job.n_probes), int(job.n_frames), int(job.ny), int(job.nx)]
    manifest = {"exit_store": shape, "chunk_frames": int(chunk_frames), "job_sha256": job_digest(job)}
    mpath = os.path.join(directory, "manifest.json")
    if os.path.exists(mpath):
        with open(mpath) as f:
            if json.load(f) != manifest:
                raise ValueError(f"checkpoint directory {directory} belongs to another job or chunking")
    else:
        with open(mpath, "w") as f:
            json.dump(manifest, f)
    computed = 0
    for f0 in range(0, job.n_frames, chunk_frames):
        f1 = min(f0 + chunk_frames, job.n_frames)
        path = os.path.join(directory, f"frames_{f0:06d}_{f1:06d}.npy")
        if os.path.exists(path):
            waves = np.load(path, allow_pickle=False)
            job.put_exit_frames(f0, waves)
            continue
        job.run_frames(f0, f1, stream)
        waves = job.exit_frames(f0, f1)
        tmp = path[:-4] + ".partial.npy"
        np.save(tmp, waves)
        os.replace(tmp, path)       # a chunk file is either whole or absent
        computed += 1
    job.finish(stream)
    return computed
