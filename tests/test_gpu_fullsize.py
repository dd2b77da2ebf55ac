"""Full-size and degenerate cases of the HIP path, through the C ABI (needs an
MI355X).

The 512x512 grid, 32 slices, 1024 frames job runs in the launch configuration
the bench times; the oracle checks it on sampled frames (exit waves, computed
one frame at a time) and the time stage on sampled k-points (an FP64 mean,
subtraction and FFT of the GPU's own exit-wave series at those k).
"""
import numpy as np
import pytest

from paper_2602_10064_amd import workloads as w
from tests.oracle_pool import exit_waves_parallel
from tests.parity import (EXIT_TOL, SPEC_TOL, check_parity, per_frame_rel_l2, rel_l2,
                          spectrum_element_ratio)

pytestmark = pytest.mark.gpu


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


def test_c2_full_size_sampled(tacaw, ctx, oracle):
    import torch
    job = w.c2_plain()                     # 1024 frames
    print(f"[gpu] c2 full: {job.nx}x{job.ny}, {job.n_slices} slices, {job.n_frames} frames", flush=True)
    with tacaw.TacawJob(ctx, job, keep_exit_waves=True) as j:
        j.run()
        exd = torch.empty(j.exit_shape, dtype=torch.complex64, device="cuda")
        j.exit_waves(out=exd)
        spec = j.spectrum()
    frames = [0, 517, 1023]
    got = exd[0, frames].cpu().numpy()
    ref = exit_waves_parallel(job, frames=frames)[0]
    e1 = rel_l2(got, ref)
    e_frame = float(per_frame_rel_l2(got[None], ref[None]).max())
    # time stage on 2048 sampled k-points: the oracle's transform of the GPU's
    # own exit-wave series at those k (all 1024 frames)
    rng = np.random.default_rng(7)
    idx = np.sort(rng.choice(job.nx * job.ny, size=2048, replace=False))
    series = exd[0].reshape(job.n_frames, -1)[:, torch.as_tensor(idx, device="cuda")].cpu().numpy()
    series = series.astype(np.complex128)[None, :, None, :]          # [1, F, 1, 2048]
    ref_spec = oracle.tacaw_spectrum(series)
    got_spec = spec[0].reshape(job.n_frames // 2, -1)[:, idx][None, :, None, :]
    e2 = rel_l2(got_spec, ref_spec)
    ratio = spectrum_element_ratio(got_spec, ref_spec, series, series)
    print(f"[gpu] c2 full: sampled exit relL2 {e1:.3e} (worst frame {e_frame:.3e}), sampled spectrum "
          f"relL2 {e2:.3e}, element bound ratio {ratio:.3f}", flush=True)
    assert e1 <= EXIT_TOL and e_frame <= EXIT_TOL
    assert e2 <= SPEC_TOL
    assert ratio <= 1.0
    # unitary propagation: every captured wave keeps unit norm
    norms = (exd[0].abs() ** 2).sum(dim=(1, 2)).double().cpu().numpy()
    assert np.max(np.abs(norms - 1.0)) < 1e-4
    del exd


def check(tacaw, ctx, oracle, job):
    with tacaw.TacawJob(ctx, job) as j:
        j.run()
        ex, spec = j.exit_waves(), j.spectrum()
    ref_ex = oracle.exit_waves(job)
    ref_spec = oracle.tacaw_spectrum(ref_ex, two_sided=job.two_sided)
    if np.linalg.norm(ref_spec) > 1e-20:
        check_parity(ex, spec, ref_ex, ref_spec, job.two_sided, job.name)
    else:                       # nothing inelastic: both sides hold rounding only
        assert rel_l2(ex, ref_ex) <= EXIT_TOL
        assert per_frame_rel_l2(ex, ref_ex).max() <= EXIT_TOL
        assert spec.max() < 1e-20
    return ex, spec


def test_no_atoms(tacaw, ctx, oracle):
    # empty trajectory: the plane wave propagates freely, nothing scatters
    job = w.random_small_job(51, nx=32, ny=32, n_frames=6, n_atoms=0)
    ex, spec = check(tacaw, ctx, oracle, job)
    assert spec.max() < 1e-20


def test_one_slice_two_frames(tacaw, ctx, oracle):
    # the smallest frame count and a single slice (first and last slice at
    # once); two-sided, since the one-sided output of 2 frames is the DC bin
    check(tacaw, ctx, oracle, w.random_small_job(52, nx=64, ny=64, n_slices=1, n_frames=2, n_atoms=5,
                                                 two_sided=True))


def test_single_probe_one_frame_batch(tacaw, ctx, oracle, monkeypatch):
    # one probe, frame batches of one frame (3 frames, 3 batches)
    monkeypatch.setenv("TACAW_FB", "1")
    check(tacaw, ctx, oracle, w.random_small_job(53, nx=32, ny=48, n_slices=2, n_frames=3, n_atoms=4,
                                                 aperture_mrad=20.0, n_probes=1, cell=(8.0, 9.0, 3.0)))


def test_largest_time_transform(tacaw, ctx, oracle):
    # 2048 frames: the largest time transform the time stage holds in LDS
    job = w.random_small_job(54, nx=16, ny=16, n_slices=2, n_frames=2048, n_atoms=3, cell=(3.0, 3.0, 2.0))
    check(tacaw, ctx, oracle, job)
