"""Waves resident in LDS (square 64 and 128 grids) against the FP64 oracle and
against the two-pass form, through the C ABI (needs an MI355X).

The resident kernel is the default on these grids; TACAW_RESIDENT=0 forces
the row and column passes.  It runs the same FFT stages, twiddles,
transmission and propagator products as the passes; only the exchanges go
through the resident wave instead of per-line scratch, so the two forms give
bitwise the same exit waves.  Cases: one slice
group and several (the wave leaves LDS between groups), ragged frame
batches, plane waves and probes cut from a larger, wrapped potential grid,
the batched executor with jobs of two grid sizes.
"""
import numpy as np
import pytest

from paper_2602_10064_amd import workloads as w
from tests.oracle_pool import exit_waves_parallel
from tests.parity import check_parity, rel_l2

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


def run(tacaw, ctx, job):
    print(f"[gpu] {job.name}: grid {job.nx}x{job.ny} pot {job.pot_nx}x{job.pot_ny} slices {job.n_slices} "
          f"frames {job.n_frames} probes {job.n_probes}", flush=True)
    with tacaw.TacawJob(ctx, job) as j:
        j.run()
        return j.exit_waves(), j.spectrum()


CASES = {
    "c1_tiny": lambda: w.c1_tiny(n_frames=24),
    "128_plane": lambda: w.random_small_job(81, nx=128, ny=128, n_slices=7, n_frames=12, cell=(16.0, 16.0, 9.0),
                                            n_atoms=40),
    "64_probes_window": lambda: w.random_small_job(82, nx=64, ny=64, n_slices=5, n_frames=8, cell=(11.0, 9.0, 6.0),
                                                   n_atoms=30, aperture_mrad=28.0, n_probes=3, voltage_V=60e3,
                                                   pot_grid=(96, 80)),
    "128_probes_window": lambda: w.random_small_job(83, nx=128, ny=128, n_slices=4, n_frames=6,
                                                    cell=(20.0, 18.0, 5.0), n_atoms=50, aperture_mrad=25.0,
                                                    n_probes=2, pot_grid=(160, 144), two_sided=True),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("groups", ["all", "3"])
def test_resident_against_oracle_and_passes(tacaw, ctx, oracle, monkeypatch, name, groups):
    job = CASES[name]()
    monkeypatch.setenv("TACAW_FB", "5")                # ragged frame batches
    if groups != "all":
        monkeypatch.setenv("TACAW_SPLAT_GROUP", groups)   # the wave leaves LDS between slice groups
    monkeypatch.setenv("TACAW_RESIDENT", "1")
    ex, spec = run(tacaw, ctx, job)
    ref_ex = exit_waves_parallel(job)
    ref_spec = oracle.tacaw_spectrum(ref_ex, two_sided=job.two_sided)
    check_parity(ex, spec, ref_ex, ref_spec, job.two_sided, job.name + " resident")
    monkeypatch.setenv("TACAW_RESIDENT", "0")
    ex2, spec2 = run(tacaw, ctx, job)
    bitwise = np.array_equal(ex.view(np.uint32), ex2.view(np.uint32))
    d = rel_l2(ex, ex2)
    print(f"[gpu] {job.name}: resident vs passes bitwise {bitwise}, relL2 {d:.3e}", flush=True)
    assert bitwise, f"relL2 {d:.3e}"


def test_resident_batched(tacaw, ctx, monkeypatch):
    """The batched executor with resident lanes: jobs of 64^2 and 128^2 with
    different slice and frame counts, equal to each job's own resident run."""
    monkeypatch.setenv("TACAW_RESIDENT", "1")
    frames = [6, 8, 10, 12, 16]
    jobs = [w.random_small_job(90 + i, nx=n, ny=n, n_slices=3 + i, n_frames=frames[i], cell=(n / 8.0, n / 8.0, 5.0),
                               n_atoms=20 + i) for i, n in enumerate([64, 128, 64, 128, 64])]
    ref = [run(tacaw, ctx, j)[1] for j in jobs]
    handles = [tacaw.TacawJob(ctx, j) for j in jobs]
    try:
        tacaw.run_batch(handles)
        for h, r in zip(handles, ref):
            assert np.array_equal(h.spectrum().view(np.uint32), r.view(np.uint32)), h.job.name
    finally:
        for h in handles:
            h.destroy()
