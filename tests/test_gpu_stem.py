"""Aberrated probes and ADF/HAADF detector sums on the device ("Beyond
Vibrational Spectroscopy"; Methods 2.1 HAADFData), through the C ABI (needs an
MI355X).  Exit waves and spectra of aberrated probes are held to the path's
tolerances; the detector reductions of the GPU's own exit waves agree with the
oracle's reductions of them to FP64 rounding."""
import math

import numpy as np
import pytest

from paper_2602_10064_amd import workloads as w

pytestmark = pytest.mark.gpu

EXIT_TOL = 1e-4
SPEC_TOL = 1e-3
FP64_TOL = 1e-12


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
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def aberrations(seed):
    # defocus, two-fold astigmatism, coma, three-fold, Cs and C5 of typical sizes
    rng = np.random.default_rng(seed)
    c = np.zeros(14)
    c[0] = rng.uniform(-80, 80)        # C10
    c[1] = rng.uniform(0, 20)          # C12
    c[2] = rng.uniform(0, 500)         # C21
    c[3] = rng.uniform(0, 500)         # C23
    c[4] = rng.uniform(-2e5, 2e5)      # C30
    c[10] = rng.uniform(0, 5e7)        # C50
    return np.stack([c, rng.uniform(0, 2 * math.pi, 14)])


def test_aberrated_probes(tacaw, ctx, oracle):
    job = w.random_small_job(81, nx=64, ny=48, n_slices=3, n_frames=8, n_atoms=8, aperture_mrad=25.0,
                             n_probes=3, cell=(8.0, 7.0, 4.0))
    job.aberrations = aberrations(81)
    print(f"[gpu] aberrated probes {job.nx}x{job.ny} P={job.n_probes}", flush=True)
    with tacaw.TacawJob(ctx, job) as j:
        j.run()
        ex, spec = j.exit_waves(), j.spectrum()
    ref_ex = oracle.exit_waves(job)
    assert rel(ex, ref_ex) <= EXIT_TOL
    assert rel(spec, oracle.tacaw_spectrum(ref_ex)) <= SPEC_TOL
    # the aberrations do change the result
    plain = job.aberrations
    job.aberrations = None
    assert rel(oracle.exit_waves(job, frames=[0]), ref_ex[:, :1]) > 1e-2
    job.aberrations = plain


def test_aberrated_windowed_probes(tacaw, ctx, oracle):
    job = w.random_small_job(82, nx=64, ny=64, n_slices=2, n_frames=6, n_atoms=10, aperture_mrad=20.0,
                             n_probes=2, cell=(12.0, 10.0, 3.0), pot_grid=(96, 80))
    job.aberrations = aberrations(82)
    print(f"[gpu] aberrated windowed probes {job.nx}x{job.ny} of {job.pot_nx}x{job.pot_ny}", flush=True)
    with tacaw.TacawJob(ctx, job) as j:
        j.run()
        ex = j.exit_waves()
    assert rel(ex, oracle.exit_waves(job)) <= EXIT_TOL


def test_set_aberrations_between_runs(tacaw, ctx, oracle):
    # a job that already holds its probes rebuilds them; clearing restores them
    job = w.random_small_job(83, nx=32, ny=32, n_slices=2, n_frames=4, n_atoms=5, aperture_mrad=25.0,
                             n_probes=2, cell=(6.0, 6.0, 3.0))
    ab = aberrations(83)
    with tacaw.TacawJob(ctx, job) as j:
        j.run()
        ex0 = j.exit_waves()
        j.set_aberrations(ab[0], ab[1])
        j.run()
        ex1 = j.exit_waves()
        j.set_aberrations(None)
        j.run()
        ex2 = j.exit_waves()
    ref0 = oracle.exit_waves(job)
    job.aberrations = ab
    ref1 = oracle.exit_waves(job)
    assert rel(ex0, ref0) <= EXIT_TOL
    assert rel(ex1, ref1) <= EXIT_TOL
    assert np.array_equal(ex2, ex0)


def test_mean_diffraction_and_adf(tacaw, ctx, oracle):
    job = w.random_small_job(84, nx=48, ny=64, n_slices=3, n_frames=10, n_atoms=40, aperture_mrad=22.0,
                             n_probes=4, cell=(7.0, 9.0, 4.0), n_species=3)
    job.aberrations = aberrations(84)
    dx, dy = job.cell[0] / job.nx, job.cell[1] / job.ny
    kx, ky = np.fft.fftfreq(job.nx, dx), np.fft.fftfreq(job.ny, dy)
    lam = oracle.wavelength_A(job.voltage_V)
    bands = [(0.0, 22.0), (31.7, 77.3), (52.1, 1e9), (0.0, 1e9)]
    with tacaw.TacawJob(ctx, job) as j:
        j.run()
        ex = j.exit_waves()
        md = j.mean_diffraction()
        adf = [j.adf(a, b) for a, b in bands]
    own = oracle.mean_diffraction(ex)
    assert md.shape == (job.n_probes, job.ny, job.nx)
    assert rel(md, own) <= FP64_TOL
    ref_md = oracle.mean_diffraction(oracle.exit_waves(job))
    assert rel(md, ref_md) <= 2 * EXIT_TOL
    for (a, b), got in zip(bands, adf):
        assert rel(got, oracle.adf(own, kx, ky, lam, a, b)) <= FP64_TOL
        assert rel(got, oracle.adf(ref_md, kx, ky, lam, a, b)) <= SPEC_TOL
    # a detector over every node collects the unit norm of each probe
    assert np.max(np.abs(adf[-1] - 1.0)) < 1e-5


def test_stem_errors(tacaw, ctx):
    plane = w.random_small_job(85, nx=32, ny=32, n_slices=1, n_frames=4, n_atoms=2)
    with tacaw.TacawJob(ctx, plane) as j:
        with pytest.raises(tacaw.TacawError):
            j.set_aberrations(np.ones(14))            # no probe to aberrate
        with pytest.raises(tacaw.TacawError):
            j.adf(0.0, 10.0)                          # not run yet
        j.run()
        with pytest.raises(tacaw.TacawError):
            j.adf(10.0, 10.0)                         # empty annulus
        assert j.adf(0.0, 1e9).shape == (1,)
    probe = w.random_small_job(86, nx=32, ny=32, n_slices=1, n_frames=4, n_atoms=2, aperture_mrad=20.0)
    with tacaw.TacawJob(ctx, probe) as j:
        bad = np.zeros(14)
        bad[4] = np.inf
        with pytest.raises(tacaw.TacawError):
            j.set_aberrations(bad)
    with tacaw.TacawJob(ctx, probe, keep_exit_waves=False) as j:
        j.run()
        with pytest.raises(tacaw.TacawError):
            j.mean_diffraction()                      # exit waves not kept


def test_graph_replay_picks_up_new_aberrations(tacaw, ctx):
    # a captured job rebuilds its probes in place when aberrations change, so
    # later replays use them; each replay equals the eager run of the same
    # state, with eager work between replays
    import torch
    job = w.random_small_job(87, nx=32, ny=32, n_slices=2, n_frames=6, n_atoms=5, aperture_mrad=25.0,
                             n_probes=2, cell=(6.0, 6.0, 3.0))
    ab = aberrations(87)
    with tacaw.TacawJob(ctx, job) as e:
        e.run()
        ref0 = e.spectrum()
        e.set_aberrations(ab[0], ab[1])
        e.run()
        ref1 = e.spectrum()
    assert not np.array_equal(ref0, ref1)
    with tacaw.TacawJob(ctx, job, use_graph=True) as g:
        for rep in range(2):
            g.run()
            torch.cuda.synchronize()
            assert np.array_equal(g.spectrum().view(np.uint32), ref0.view(np.uint32)), rep
            torch.randn(1 << 18, device="cuda").sum().item()
        g.set_aberrations(ab[0], ab[1])
        for rep in range(2):
            g.run()
            torch.cuda.synchronize()
            assert np.array_equal(g.spectrum().view(np.uint32), ref1.view(np.uint32)), rep
            torch.randn(1 << 18, device="cuda").sum().item()
