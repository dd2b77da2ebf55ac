"""Frame ranges, checkpoint/restart and trajectory averaging through the C ABI
(needs an MI355X): Methods 2.1 "Workflow Architecture" (per-frame exit waves,
restart after interruption) and "Molecular Dynamics" with the Supplement's
"Trajectory averaging"."""
import numpy as np
import pytest

from paper_2602_10064_amd import workloads as w

pytestmark = pytest.mark.gpu

SPEC_TOL = 1e-3


@pytest.fixture(scope="module")
def tacaw():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2602_10064_amd import tacaw as t
    t.lib()
    return t


@pytest.fixture(scope="module")
def ctx(tacaw):
    c = tacaw.Context(0)
    yield c
    c.close()


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def probe_job(seed, n_frames=12):
    return w.random_small_job(seed, nx=48, ny=32, n_slices=3, n_frames=n_frames, n_atoms=7, aperture_mrad=25.0,
                              n_probes=2, cell=(7.0, 5.0, 4.0))


def test_frame_ranges_match_the_full_run(tacaw, ctx):
    job = probe_job(91)
    print("[gpu] frame ranges", flush=True)
    with tacaw.TacawJob(ctx, job) as j:
        j.run()
        ex, spec = j.exit_waves(), j.spectrum()
        j.finish()                      # a whole-job run leaves every frame present
        assert np.array_equal(j.spectrum(), spec)
    with tacaw.TacawJob(ctx, job, use_graph=True) as j:
        j.run()
        j.finish()                      # so does a graph replay
        assert np.array_equal(j.spectrum(), spec)
    with tacaw.TacawJob(ctx, job) as j:
        tacaw.run_batch([j])
        j.finish()                      # and the batched executor
        assert np.array_equal(j.spectrum(), spec)
    with tacaw.TacawJob(ctx, job) as j:
        for f0, f1 in [(0, 5), (5, 9), (9, 12)]:
            j.run_frames(f0, f1)
        j.finish()
        assert np.array_equal(j.exit_waves(), ex)
        assert np.array_equal(j.spectrum(), spec)
        assert np.array_equal(j.exit_frames(3, 7), ex[:, 3:7])


def test_checkpoint_restart(tacaw, ctx, tmp_path):
    from paper_2602_10064_amd.checkpoint import run_with_checkpoints
    job = probe_job(92, n_frames=10)
    print("[gpu] checkpoint restart", flush=True)
    with tacaw.TacawJob(ctx, job) as j:
        j.run()
        spec = j.spectrum()
    with tacaw.TacawJob(ctx, job) as j:
        assert run_with_checkpoints(j, str(tmp_path), 4) == 3
        assert np.array_equal(j.spectrum(), spec)
    (tmp_path / "frames_000004_000008.npy").unlink()       # lost with an interrupted run
    with tacaw.TacawJob(ctx, job) as j:
        assert run_with_checkpoints(j, str(tmp_path), 4) == 1
        assert np.array_equal(j.spectrum(), spec)


def test_frame_range_errors(tacaw, ctx):
    job = probe_job(93, n_frames=6)
    with tacaw.TacawJob(ctx, job) as j:
        for f0, f1 in [(-1, 2), (3, 3), (4, 7)]:
            with pytest.raises(tacaw.TacawError):
                j.run_frames(f0, f1)
        j.run_frames(0, 3)
        with pytest.raises(tacaw.TacawError):
            j.finish()                                   # frames 3-5 missing
        with pytest.raises(tacaw.TacawError):
            j.exit_frames(2, 4)                          # frame 3 not computed
        with pytest.raises(ValueError):
            j.put_exit_frames(3, np.zeros((1, 3, 32, 48), np.complex64))
        j.put_exit_frames(3, np.zeros((2, 3, 32, 48), np.complex64))
        j.finish()


def test_average_of_trajectories(tacaw, ctx, oracle):
    jobs = [probe_job(s, n_frames=8) for s in (94, 95, 96)]
    print("[gpu] trajectory average", flush=True)
    handles = [tacaw.TacawJob(ctx, jb) for jb in jobs]
    try:
        for h in handles:
            h.run()
        own = [h.spectrum() for h in handles]
        avg = tacaw.average_spectra(handles)
    finally:
        for h in handles:
            h.destroy()
    assert avg.dtype == np.float32
    assert np.array_equal(avg, oracle.average_spectra(own).astype(np.float32))
    ref = oracle.average_spectra(oracle.tacaw_spectrum(oracle.exit_waves(jb)) for jb in jobs)
    assert rel(avg, ref) <= SPEC_TOL
    with tacaw.TacawJob(ctx, probe_job(97, n_frames=6)) as other:
        other.run()
        with tacaw.TacawJob(ctx, jobs[0]) as first:
            first.run()
            with pytest.raises(tacaw.TacawError):
                tacaw.average_spectra([first, other])   # 4 bins against 3


def test_segment_average_batched(tacaw, ctx, oracle):
    # three 8-frame segments of one 24-frame trajectory, run by the batched
    # executor and averaged on the device
    job = probe_job(98, n_frames=24)
    segs = w.frame_segments(job, 3)
    print("[gpu] segment average", flush=True)
    handles = [tacaw.TacawJob(ctx, s) for s in segs]
    try:
        tacaw.run_batch(handles)
        avg = tacaw.average_spectra(handles)
    finally:
        for h in handles:
            h.destroy()
    ref = oracle.segment_average_spectrum(oracle.exit_waves(job), 3)
    assert avg.shape == ref.shape
    assert rel(avg, ref) <= SPEC_TOL
