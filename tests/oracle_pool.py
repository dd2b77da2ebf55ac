"""Runs the oracle frame by frame in a process pool (test helper).

Workers are spawned (not forked) so they never inherit a GPU context, and each
uses a single BLAS thread."""
import multiprocessing as mp
import os

import numpy as np


def _init():
    os.environ["OMP_NUM_THREADS"] = "1"
    os.environ["OPENBLAS_NUM_THREADS"] = "1"


def _one(args):
    job, f, probes = args
    from oracle import tacaw_oracle
    return tacaw_oracle.exit_waves(job, frames=[f], probes=probes)


def exit_waves_parallel(job, frames=None, probes=None, workers=None):
    frames = list(range(job.n_frames)) if frames is None else list(frames)
    workers = workers or min(len(frames), max(1, min(16, len(os.sched_getaffinity(0)))))
    if workers <= 1 or len(frames) == 1:
        from oracle import tacaw_oracle
        return tacaw_oracle.exit_waves(job, frames=frames, probes=probes)
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers, initializer=_init) as pool:
        parts = pool.map(_one, [(job, f, probes) for f in frames])
    return np.concatenate(parts, axis=1)
