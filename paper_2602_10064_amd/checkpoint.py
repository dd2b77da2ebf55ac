"""Frame-granular checkpoints of a job's exit waves (Methods 2.1 "Workflow
Architecture": exit waves are cached per frame so that an interrupted run
restarts without recomputing finished frames).

The job runs in chunks of frames.  After each chunk its exit waves go to one
.npy file in the checkpoint directory; a later run of the same job restores
the chunks whose files exist (numpy.load without pickles) and computes only
the rest, then runs the time stage.  The directory belongs to one job: its
manifest records the exit-store shape and the chunk size, and a mismatch is an
error.
"""
from __future__ import annotations

import json
import os

import numpy as np


def run_with_checkpoints(job, directory: str, chunk_frames: int, stream=None) -> int:
    """Run a TacawJob chunk by chunk with per-chunk exit-wave files; returns the
    number of chunks computed (the others were restored)."""
    if chunk_frames < 1:
        raise ValueError("chunk_frames must be positive")
    os.makedirs(directory, exist_ok=True)
    shape = [int(job.n_probes), int(job.n_frames), int(job.ny), int(job.nx)]
    manifest = {"exit_store": shape, "chunk_frames": int(chunk_frames)}
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
