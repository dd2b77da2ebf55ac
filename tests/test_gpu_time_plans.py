"""Every compiled time-stage plan and the spectrum-image shape, through the C
ABI, against the FP64 oracle (needs an MI355X).

The time stage (FP64 frame mean, FP64 subtraction, length-F transform, |.|^2;
Methods 2.1 "Workflow Architecture", Supplement "Sampling Considerations") has
one compile-time plan per frame count in {16, 32, 48, 64, 96, 128, 160, 192,
256, 320, 384, 512, 640, 768, 1024, 2048}, each with its own radix sequence,
k-points per workgroup and LDS stride, and a runtime-radix kernel for every
other 2*3*5-smooth count.  Each plan runs here on a small grid with one slice,
so the oracle covers every frame.
"""
import numpy as np
import pytest

from paper_2602_10064_amd import workloads as w
from tests.oracle_pool import exit_waves_parallel
from tests.parity import check_parity, per_frame_rel_l2, rel_l2, spectrum_element_ratio, EXIT_TOL, SPEC_TOL

pytestmark = pytest.mark.gpu

COMPILED = [32, 48, 96, 128, 160, 192, 256, 320, 384, 512, 640, 768]
# runtime-radix frame counts from the uneven mix (2*3*5-smooth, not compiled)
RUNTIME = [135, 250, 729, 1000]


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


def run_and_check(tacaw, ctx, oracle, job):
    print(f"[gpu] {job.name}: grid {job.nx}x{job.ny} slices {job.n_slices} frames {job.n_frames} "
          f"probes {job.n_probes} two-sided {job.two_sided}", flush=True)
    with tacaw.TacawJob(ctx, job) as j:
        j.run()
        ex, spec = j.exit_waves(), j.spectrum()
    ref_ex = oracle.exit_waves(job)
    ref_spec = oracle.tacaw_spectrum(ref_ex, two_sided=job.two_sided)
    check_parity(ex, spec, ref_ex, ref_spec, job.two_sided, job.name)
    # the DC bin holds rounding only (FP64 mean subtraction)
    assert spec[:, 0].max() <= 1e-6 * spec.max()


@pytest.mark.parametrize("n_frames", COMPILED + RUNTIME)
def test_time_plan_plane_wave(tacaw, ctx, oracle, n_frames):
    job = w.random_small_job(300 + n_frames % 97, nx=16, ny=16, n_slices=1, n_frames=n_frames, n_atoms=4,
                             cell=(3.0, 3.0, 2.0))
    run_and_check(tacaw, ctx, oracle, job.replace(name=f"time_plan_F{n_frames}"))


@pytest.mark.parametrize("n_frames", [48, 256, 640])
def test_time_plan_probes_two_sided(tacaw, ctx, oracle, n_frames):
    # several probes (one column set per probe), windows cut from a larger
    # potential grid, every bin kept
    job = w.random_small_job(400 + n_frames % 89, nx=32, ny=16, n_slices=1, n_frames=n_frames, n_atoms=6,
                             aperture_mrad=40.0, n_probes=3, cell=(6.0, 4.0, 2.0), voltage_V=60e3,
                             pot_grid=(48, 32), two_sided=True)
    run_and_check(tacaw, ctx, oracle, job.replace(name=f"time_plan_probes_F{n_frames}"))


def test_c3_geometry_256_frames(tacaw, ctx, oracle):
    """The spectrum-image job's geometry (38 400 atoms, 1000x866 potential grid,
    256^2 windows, 20 slices, 30 mrad at 60 kV) with 8 of its probes and all 256
    frames: exit waves of 2 probes x 2 frames against the oracle; the whole
    F = 256 spectrum of every probe against the oracle's transform of the GPU's
    own exit waves."""
    import torch
    full = w.c3_probe(n_frames=256)
    pick = np.array([0, 37, 150, 333, 517, 700, 891, 1023])       # spread over the 32x32 scan
    job = full.replace(probe_xy=full.probe_xy[pick], name="c3_geometry_F256")
    print(f"[gpu] {job.name}: {job.n_probes} probes x {job.n_frames} frames, windows {job.nx}x{job.ny} of "
          f"{job.pot_nx}x{job.pot_ny}", flush=True)
    with tacaw.TacawJob(ctx, job) as j:
        j.run()
        exd = torch.empty(j.exit_shape, dtype=torch.complex64, device="cuda")
        j.exit_waves(out=exd)
        spec = j.spectrum()
    frames, probes = [0, 255], [0, 7]
    got = exd[probes][:, frames].cpu().numpy()
    ref = exit_waves_parallel(job, frames=frames, probes=probes)
    e1 = rel_l2(got, ref)
    e_frame = float(per_frame_rel_l2(got, ref).max())
    print(f"[gpu] {job.name}: sampled exit relL2 {e1:.3e} (worst frame {e_frame:.3e})", flush=True)
    assert e1 <= EXIT_TOL and e_frame <= EXIT_TOL
    worst_l2, worst_ratio = 0.0, 0.0
    for p in range(job.n_probes):
        series = exd[p:p + 1].cpu().numpy().astype(np.complex128)
        ref_spec = oracle.tacaw_spectrum(series)
        worst_l2 = max(worst_l2, rel_l2(spec[p:p + 1], ref_spec))
        worst_ratio = max(worst_ratio, spectrum_element_ratio(spec[p:p + 1], ref_spec, series, series))
    print(f"[gpu] {job.name}: spectrum of the GPU's exit waves, worst probe relL2 {worst_l2:.3e}, "
          f"element bound ratio {worst_ratio:.3f}", flush=True)
    assert worst_l2 <= SPEC_TOL
    assert worst_ratio <= 1.0
    del exd
