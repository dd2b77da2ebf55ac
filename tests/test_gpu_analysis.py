"""Spectrum analysis on the device (spectral diffraction, spectrum image,
dispersion; Methods 2.1 "Data Structure Design", Supplement MWE) through the
C ABI (needs an MI355X).

The device reductions run in FP64 over the job's float32 spectrum; the oracle's
reductions of that same spectrum agree to FP64 rounding, and applied to the
oracle's own spectrum they agree to the spectrum tolerance.
"""
import numpy as np
import pytest

from paper_2602_10064_amd import workloads as w

pytestmark = pytest.mark.gpu

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


def axes(job):
    dx = job.cell[0] / (job.pot_nx or job.nx)
    dy = job.cell[1] / (job.pot_ny or job.ny)
    return dx, dy, np.fft.fftfreq(job.nx, dx), np.fft.fftfreq(job.ny, dy)


def check_job(tacaw, ctx, oracle, job, f_list, k_bounds, end_to_end=True):
    dx, dy, kx, ky = axes(job)
    with tacaw.TacawJob(ctx, job) as j:
        j.run()
        spec = j.spectrum()
        got = {}
        for f in f_list:
            got[f] = (j.spectral_diffraction(f),
                      [j.spectrum_image(f, a, b) for a, b in k_bounds])
        # a path through grid nodes, between nodes and past the Nyquist wrap
        t = np.linspace(0.0, 1.0, 23)
        px = t * 0.9 * kx.max() * 2.0 - 0.3 * kx.max()
        py = -t * 0.7 * ky.max() * 1.5
        disp = j.dispersion(px, py)
    s64 = spec.astype(np.float64)
    ref_spec = oracle.tacaw_spectrum(oracle.exit_waves(job), two_sided=job.two_sided) if end_to_end else None
    for f in f_list:
        m = oracle.frequency_bin(f, job.n_frames, job.dt_fs, job.two_sided)
        sd, si = got[f]
        assert sd.shape == (job.ny, job.nx)
        assert rel(sd, oracle.spectral_diffraction(s64, m)) <= FP64_TOL
        for (a, b), s in zip(k_bounds, si):
            assert s.shape == (job.n_probes,)
            assert rel(s, oracle.spectrum_image(s64, m, kx, ky, a, b)) <= FP64_TOL
            if ref_spec is not None and np.linalg.norm(ref_spec[:, m]) > 1e-20:
                assert rel(s, oracle.spectrum_image(ref_spec, m, kx, ky, a, b)) <= SPEC_TOL
        if ref_spec is not None and np.linalg.norm(ref_spec[:, m]) > 1e-20:
            assert rel(sd, oracle.spectral_diffraction(ref_spec, m)) <= SPEC_TOL
    ref_disp = oracle.dispersion(s64, px, py, job.nx * dx, job.ny * dy)
    assert disp.shape == (len(px), spec.shape[1])
    assert rel(disp, ref_disp) <= FP64_TOL
    return spec


def test_plane_wave_job(tacaw, ctx, oracle):
    job = w.random_small_job(61, nx=64, ny=48, n_slices=3, n_frames=20, n_atoms=8, cell=(9.0, 7.0, 4.0))
    print(f"[gpu] analysis plane wave {job.nx}x{job.ny} F={job.n_frames}", flush=True)
    fmax = 0.5 / (job.dt_fs * 1e-3)
    check_job(tacaw, ctx, oracle, job, [0.0, 0.37 * fmax, 0.9 * fmax],
              [(0.0, 0.0), (0.41, 1.73), (1.1, 0.0)])


def test_probe_scan_two_sided(tacaw, ctx, oracle):
    job = w.random_small_job(62, nx=48, ny=64, n_slices=2, n_frames=12, n_atoms=6, aperture_mrad=25.0,
                             n_probes=5, cell=(7.0, 8.0, 3.0), two_sided=True)
    print(f"[gpu] analysis probes {job.n_probes} two-sided F={job.n_frames}", flush=True)
    fmax = 0.5 / (job.dt_fs * 1e-3)
    check_job(tacaw, ctx, oracle, job, [-0.6 * fmax, 0.0, 0.3 * fmax], [(0.0, 0.0), (0.2, 0.9)])


def test_windowed_probes(tacaw, ctx, oracle):
    # probes see 64^2 windows of a 96x80 potential grid: the analysis axes
    # follow the window grid
    job = w.random_small_job(63, nx=64, ny=64, n_slices=2, n_frames=8, n_atoms=10, aperture_mrad=20.0,
                             n_probes=3, cell=(12.0, 10.0, 3.0), pot_grid=(96, 80))
    print(f"[gpu] analysis windowed {job.nx}x{job.ny} of {job.pot_nx}x{job.pot_ny}", flush=True)
    check_job(tacaw, ctx, oracle, job, [10.0, 40.0], [(0.0, 0.0), (0.3, 1.2)])


def test_frequency_out_of_range_and_before_run(tacaw, ctx):
    job = w.random_small_job(64, nx=32, ny=32, n_slices=1, n_frames=8, n_atoms=3)
    fmax = 0.5 / (job.dt_fs * 1e-3)           # one-sided keeps bins below fmax
    with tacaw.TacawJob(ctx, job) as j:
        with pytest.raises(tacaw.TacawError):
            j.spectral_diffraction(1.0)        # no spectrum yet
        j.run()
        df = 1.0 / (job.n_frames * job.dt_fs * 1e-3)
        last = (job.n_frames // 2 - 1) * df
        j.spectral_diffraction(last + 0.49 * df)   # within half a bin of the last kept bin
        with pytest.raises(tacaw.TacawError):
            j.spectral_diffraction(last + 0.51 * df)
        with pytest.raises(tacaw.TacawError):
            j.spectrum_image(-0.6 * df)
        with pytest.raises(tacaw.TacawError):
            j.spectrum_image(0.0, 1.0, 0.5)        # outer bound below the inner one
        with pytest.raises(tacaw.TacawError):
            j.dispersion([np.nan], [0.0])
        assert fmax > last
