"""HIP path vs the FP64 oracle, through the C ABI (needs an MI355X).

Tolerances (complex64 GPU path vs FP64 oracle): relative L2 error <= 1e-4 on
exit waves psi(k, t), over the whole array and for every (probe, frame) wave,
and <= 1e-3 on I(k, w), plus the per-element spectrum bound of tests/parity.py.
"""
import os

import numpy as np
import pytest

from paper_2602_10064_amd import workloads as w
from tests.oracle_pool import exit_waves_parallel
from tests.parity import EXIT_TOL, SPEC_TOL, check_parity, rel_l2

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


def run_gpu(tacaw, ctx, job):
    print(f"[gpu] {job.name}: grid {job.nx}x{job.ny} pot {job.pot_nx}x{job.pot_ny} slices "
          f"{job.n_slices} frames {job.n_frames} probes {job.n_probes} atoms {job.n_atoms}", flush=True)
    with tacaw.TacawJob(ctx, job) as j:
        j.run()
        return j.exit_waves(), j.spectrum(), j.slices()


def check_job(tacaw, ctx, oracle, job, exit_tol=EXIT_TOL, spec_tol=SPEC_TOL):
    ex, spec, sl = run_gpu(tacaw, ctx, job)
    ref_sl = oracle.slice_index(job.positions, job.cell[2], job.n_slices)
    assert np.array_equal(sl, ref_sl)
    ref_ex = exit_waves_parallel(job)
    ref_spec = oracle.tacaw_spectrum(ref_ex, two_sided=job.two_sided)
    check_parity(ex, spec, ref_ex, ref_spec, job.two_sided, job.name, exit_tol, spec_tol)
    return ex, spec, ref_ex, ref_spec


def test_c1_tiny_full(tacaw, ctx, oracle):
    job = w.c1_tiny()
    ex, spec, _, _ = check_job(tacaw, ctx, oracle, job)
    # FP64 mean subtraction: the DC bin holds rounding only
    assert spec[:, 0].max() <= 1e-6 * spec.max()
    # unitary propagation in FP32
    norms = np.sum(np.abs(ex.astype(np.complex128)) ** 2, axis=(2, 3))
    assert np.max(np.abs(norms - 1.0)) < 1e-5


SMALL = [
    dict(seed=11, nx=16, ny=16, n_slices=3, n_frames=8, cell=(3.2, 3.2, 3.0)),
    dict(seed=12, nx=32, ny=48, n_slices=4, n_frames=12, cell=(5.0, 7.5, 4.0)),
    dict(seed=13, nx=96, ny=64, n_slices=5, n_frames=10, cell=(12.0, 8.0, 6.0), n_atoms=12),
    dict(seed=14, nx=160, ny=128, n_slices=2, n_frames=6, cell=(18.0, 15.0, 3.0), n_atoms=10),
    dict(seed=15, nx=384, ny=192, n_slices=2, n_frames=4, cell=(40.0, 22.0, 3.0), n_atoms=20),
    dict(seed=16, nx=64, ny=64, n_slices=3, n_frames=8, cell=(8.0, 8.0, 4.0), aperture_mrad=30.0,
         n_probes=3, voltage_V=60e3),
    dict(seed=17, nx=32, ny=32, n_slices=3, n_frames=8, cell=(10.0, 9.0, 4.0), aperture_mrad=25.0,
         n_probes=4, voltage_V=100e3, pot_grid=(100, 90)),
    dict(seed=18, nx=48, ny=32, n_slices=2, n_frames=15, cell=(9.5, 8.1, 4.0), aperture_mrad=30.0,
         n_probes=2, voltage_V=200e3, pot_grid=(95, 81), two_sided=True),
    dict(seed=19, nx=640, ny=16, n_slices=2, n_frames=4, cell=(64.0, 2.0, 3.0), n_atoms=8),
    # 512 rows under a narrower grid: the default six-step column kernel
    dict(seed=20, nx=96, ny=512, n_slices=2, n_frames=5, cell=(12.0, 64.0, 3.0), n_atoms=16),
    # register FFT kernels for 128 and 256 (rows and columns, mixed shapes)
    dict(seed=31, nx=128, ny=128, n_slices=3, n_frames=6, cell=(14.0, 14.0, 4.0), n_atoms=16),
    dict(seed=32, nx=256, ny=256, n_slices=2, n_frames=4, cell=(26.0, 26.0, 3.0), n_atoms=24),
    dict(seed=33, nx=256, ny=128, n_slices=2, n_frames=6, cell=(27.0, 13.0, 3.0), n_atoms=12),
    dict(seed=34, nx=128, ny=256, n_slices=3, n_frames=5, cell=(13.0, 26.0, 4.0), n_atoms=12,
         aperture_mrad=30.0, n_probes=2, voltage_V=100e3),
    dict(seed=35, nx=128, ny=128, n_slices=2, n_frames=6, cell=(30.0, 27.0, 4.0), aperture_mrad=25.0,
         n_probes=3, voltage_V=60e3, pot_grid=(300, 270), two_sided=True),
    # 12- and 16-value register kernels: 384, 768 and the serving mix's 1024
    dict(seed=36, nx=1024, ny=1024, n_slices=2, n_frames=4, cell=(110.0, 110.0, 3.0), n_atoms=40),
    dict(seed=37, nx=384, ny=384, n_slices=3, n_frames=5, cell=(40.0, 40.0, 4.0), n_atoms=25),
    dict(seed=38, nx=768, ny=384, n_slices=2, n_frames=4, cell=(80.0, 40.0, 3.0), n_atoms=30),
    dict(seed=39, nx=384, ny=768, n_slices=2, n_frames=4, cell=(40.0, 80.0, 3.0), n_atoms=30,
         aperture_mrad=30.0, n_probes=2, voltage_V=100e3),
]


@pytest.mark.parametrize("kw", SMALL, ids=[f"s{k['seed']}_{k['nx']}x{k['ny']}" for k in SMALL])
def test_small_jobs(tacaw, ctx, oracle, kw):
    job = w.random_small_job(**kw)
    check_job(tacaw, ctx, oracle, job)


def test_c2_shape_reduced_frames_ragged_batches(tacaw, ctx, oracle, monkeypatch):
    # full 512^2 grid, 32 slices, 9216 atoms; 16 frames in batches of 5 (5+5+5+1)
    monkeypatch.setenv("TACAW_FB", "5")
    job = w.c2_plain(n_frames=16)
    check_job(tacaw, ctx, oracle, job)


def test_splat_all_slices_mode_matches(tacaw, ctx, monkeypatch):
    # potentials of all slices of a batch at once give bitwise the same result
    job = w.c1_tiny(n_frames=16)
    _, a, _ = run_gpu(tacaw, ctx, job)
    monkeypatch.setenv("TACAW_SPLAT_ALL", "1")
    monkeypatch.setenv("TACAW_FB", "3")
    _, b, _ = run_gpu(tacaw, ctx, job)
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


def test_determinism_bitwise(tacaw, ctx):
    job = w.c1_tiny(n_frames=32)
    ex1, sp1, _ = run_gpu(tacaw, ctx, job)
    ex2, sp2, _ = run_gpu(tacaw, ctx, job)
    assert np.array_equal(ex1.view(np.uint32), ex2.view(np.uint32))
    assert np.array_equal(sp1.view(np.uint32), sp2.view(np.uint32))


def test_static_trajectory_gives_zero_spectrum(tacaw, ctx):
    job = w.random_small_job(21, nx=32, ny=32, n_frames=8, cell=(5.0, 5.0, 3.0))
    job.positions[:] = job.positions[0:1]
    _, spec, _ = run_gpu(tacaw, ctx, job)
    assert spec.max() < 1e-20


def test_circular_frame_shift_invariance(tacaw, ctx):
    job = w.c1_tiny(n_frames=32)
    _, a, _ = run_gpu(tacaw, ctx, job)
    _, b, _ = run_gpu(tacaw, ctx, job.replace(positions=np.roll(job.positions, 5, axis=0)))
    assert rel_l2(b, a) < 1e-4


def test_device_destination_and_stream(tacaw, ctx):
    import torch
    job = w.c1_tiny(n_frames=16)
    with tacaw.TacawJob(ctx, job) as j:
        s = torch.cuda.Stream()
        j.run(stream=s)
        host = j.spectrum()
        dev = torch.empty(j.spectrum_shape, dtype=torch.float32, device="cuda")
        j.spectrum(out=dev)
        assert np.array_equal(dev.cpu().numpy(), host)
        exd = torch.empty(j.exit_shape, dtype=torch.complex64, device="cuda")
        j.exit_waves(out=exd)
        assert np.array_equal(exd.cpu().numpy(), j.exit_waves())


def test_errors_do_not_poison_context(tacaw, ctx):
    job = w.random_small_job(22, nx=16, ny=16, n_frames=8)
    with pytest.raises(tacaw.TacawError):
        tacaw.TacawJob(ctx, job.replace(atom_species=np.full(job.n_atoms, 7, np.int32)))
    with tacaw.TacawJob(ctx, job) as j:
        with pytest.raises(tacaw.TacawError) as e:
            j.spectrum()
        assert e.value.status == 5          # not run yet
        j.run()
        assert np.isfinite(j.spectrum()).all()


@pytest.mark.parametrize("col_variant", ["default", "7"])
def test_c3_shape_reduced_probes_frames(tacaw, ctx, oracle, monkeypatch, col_variant):
    # full c3 geometry (38400 atoms, 1000x866 potential grid, 256^2 windows,
    # 20 slices, 30 mrad at 60 kV) with a 3x3 scan and 4 frames
    if col_variant != "default":
        monkeypatch.setenv("TACAW_COL_VARIANT", col_variant)
    job = w.c3_probe(n_frames=4, n_scan=3)
    check_job(tacaw, ctx, oracle, job)


@pytest.mark.parametrize("n", [64, 128])
def test_deep_row_kernel_matches(tacaw, ctx, monkeypatch, n):
    # two rows in flight per wavefront: the same per-row arithmetic, so the
    # same values to FP32 rounding (ragged grid stride over 9 frames)
    monkeypatch.setenv("TACAW_RESIDENT", "0")   # the row and column passes, not the LDS-resident kernel
    job = w.random_small_job(41, nx=n, ny=n, n_slices=3, n_frames=9, cell=(n / 9.0, n / 9.0, 4.0))
    _, a, _ = run_gpu(tacaw, ctx, job)
    monkeypatch.setenv("TACAW_ROW_VARIANT", "3")
    _, b, _ = run_gpu(tacaw, ctx, job)
    assert rel_l2(b, a) < 1e-6


def test_fft_variants_agree(tacaw, ctx, monkeypatch):
    # the LDS Stockham kernels with one or two rows per workgroup run the same
    # arithmetic per row (bitwise equal); the register kernels agree with them
    # to FP32 rounding
    monkeypatch.setenv("TACAW_RESIDENT", "0")   # the row and column passes, not the LDS-resident kernel
    job = w.c1_tiny(n_frames=16)
    _, reg, _ = run_gpu(tacaw, ctx, job)          # default: register kernels for 64
    monkeypatch.setenv("TACAW_COL_VARIANT", "0")
    monkeypatch.setenv("TACAW_ROW_VARIANT", "0")
    _, v0, _ = run_gpu(tacaw, ctx, job)
    monkeypatch.setenv("TACAW_ROW_VARIANT", "1")
    _, v1, _ = run_gpu(tacaw, ctx, job)
    assert np.array_equal(v0.view(np.uint32), v1.view(np.uint32))
    assert rel_l2(reg, v0) < 1e-5


@pytest.mark.parametrize("variant", ["2", "3"])
def test_c2_shape_register_row_kernel(tacaw, ctx, oracle, monkeypatch, variant):
    # register row kernels with one (2) or two (3) rows in flight per wavefront
    monkeypatch.setenv("TACAW_ROW_VARIANT", variant)
    monkeypatch.setenv("TACAW_FB", "3")
    job = w.c2_plain(n_frames=8)
    check_job(tacaw, ctx, oracle, job)


@pytest.mark.parametrize("fb", ["5", "64"])
def test_overlapped_potentials_bitwise(tacaw, ctx, monkeypatch, fb):
    # potentials built one slice ahead on a side stream give bitwise the same
    # result as building each right before its row pass (ragged batches too)
    monkeypatch.setenv("TACAW_FB", fb)
    monkeypatch.setenv("TACAW_OVERLAP", "1")
    job = w.c1_tiny(n_frames=24)
    ex_a, sp_a, _ = run_gpu(tacaw, ctx, job)
    monkeypatch.setenv("TACAW_OVERLAP", "0")
    ex_b, sp_b, _ = run_gpu(tacaw, ctx, job)
    assert np.array_equal(ex_a.view(np.uint32), ex_b.view(np.uint32))
    assert np.array_equal(sp_a.view(np.uint32), sp_b.view(np.uint32))


def test_overlapped_potentials_graph_replay(tacaw, ctx, monkeypatch):
    # the side stream's launches are captured with the job's graph; replays
    # with eager work in between match the eager run
    import torch
    monkeypatch.setenv("TACAW_FB", "6")
    monkeypatch.setenv("TACAW_OVERLAP", "1")
    job = w.c1_tiny(n_frames=20)
    _, ref, _ = run_gpu(tacaw, ctx, job)
    with tacaw.TacawJob(ctx, job, use_graph=True) as j:
        for i in range(3):
            j.run()
            torch.cuda.synchronize()
            got = j.spectrum()
            assert np.array_equal(got.view(np.uint32), ref.view(np.uint32)), f"replay {i}"
            x = torch.randn(1 << 20, device="cuda")
            (x * 2).sum().item()


@pytest.mark.parametrize("variant", ["2", "3", "4", "5", "6"])
def test_c2_shape_register_column_kernels(tacaw, ctx, oracle, monkeypatch, variant):
    # register column pass on 8-column tiles (2), 16-column tiles (3),
    # 8-column tiles with two LDS buffers (4), the six-step kernel on
    # 8-column tiles (5) and on 16-column tiles (6)
    monkeypatch.setenv("TACAW_COL_VARIANT", variant)
    monkeypatch.setenv("TACAW_FB", "3")
    job = w.c2_plain(n_frames=5)
    check_job(tacaw, ctx, oracle, job)


@pytest.mark.parametrize("variant", ["2", "5", "6"])
def test_512_rows_narrow_grid(tacaw, ctx, oracle, monkeypatch, variant):
    # 512 rows and 64 columns: the six-step column kernel (default at 512 rows)
    # and the register kernel, probes included, ragged frame batches
    monkeypatch.setenv("TACAW_COL_VARIANT", variant)
    monkeypatch.setenv("TACAW_FB", "4")
    job = w.random_small_job(47, nx=64, ny=512, n_slices=3, n_frames=10, cell=(8.0, 64.0, 4.0), n_atoms=20,
                             aperture_mrad=25.0, n_probes=2)
    check_job(tacaw, ctx, oracle, job)


@pytest.mark.parametrize("variant", ["2", "3", "4", "7"])
def test_256_rows_column_kernels(tacaw, ctx, oracle, monkeypatch, variant):
    # 256 rows: the register column kernel on 8-column tiles (2), 16-column
    # tiles (3) and 8-column tiles with two LDS buffers (4), and the six-step
    # kernel on 16-column tiles (7); probes in windows of a larger potential
    # grid, ragged frame batches
    monkeypatch.setenv("TACAW_COL_VARIANT", variant)
    monkeypatch.setenv("TACAW_FB", "3")
    job = w.random_small_job(48, nx=48, ny=256, n_slices=3, n_frames=10, cell=(6.0, 32.0, 4.0), n_atoms=24,
                             aperture_mrad=25.0, n_probes=3, pot_grid=(64, 320))
    check_job(tacaw, ctx, oracle, job)


@pytest.mark.parametrize("variant", ["2", "8"])
def test_384_rows_column_kernels(tacaw, ctx, oracle, monkeypatch, variant):
    # 384 rows: the 12-value register column kernel (2) and the six-step
    # kernel 384 = 6 x 64 on 8-column tiles (8, whose second layout has six
    # wavefronts); probes in windows of a larger potential grid, ragged frame
    # batches, 48 columns (six tiles)
    monkeypatch.setenv("TACAW_COL_VARIANT", variant)
    monkeypatch.setenv("TACAW_FB", "3")
    job = w.random_small_job(49, nx=48, ny=384, n_slices=3, n_frames=10, cell=(6.0, 48.0, 4.0), n_atoms=24,
                             aperture_mrad=25.0, n_probes=2, pot_grid=(64, 448))
    check_job(tacaw, ctx, oracle, job)


@pytest.mark.parametrize("variant", ["2", "4"])
def test_384_wide_row_kernels(tacaw, ctx, oracle, monkeypatch, variant):
    # 384-wide rows: the 12-value register row kernel (2) and the six-step
    # row kernel 384 = 6 x 64 (4: first-slice rows from the incident probe
    # through the forward steps, later rows through the conjugate steps, the
    # transmission at scrambled positions and back); probes in windows of a
    # larger potential grid (wrapped potential rows), ragged frame batches
    monkeypatch.setenv("TACAW_ROW_VARIANT", variant)
    monkeypatch.setenv("TACAW_FB", "3")
    job = w.random_small_job(51, nx=384, ny=48, n_slices=3, n_frames=10, cell=(48.0, 6.0, 4.0), n_atoms=24,
                             aperture_mrad=25.0, n_probes=2, pot_grid=(448, 64))
    check_job(tacaw, ctx, oracle, job)


def test_384_square_six_step(tacaw, ctx, oracle, monkeypatch):
    # the six-step row and column kernels on a 384^2 plane-wave job with
    # several column tiles per frame and a last slice (exit waves stored from
    # the second layout)
    monkeypatch.setenv("TACAW_COL_VARIANT", "8")
    monkeypatch.setenv("TACAW_ROW_VARIANT", "4")
    monkeypatch.setenv("TACAW_FB", "2")
    job = w.random_small_job(50, nx=384, ny=384, n_slices=3, n_frames=5, cell=(40.0, 40.0, 4.0), n_atoms=25)
    check_job(tacaw, ctx, oracle, job)


def test_splat_rounds_of_16(tacaw, ctx, oracle, monkeypatch):
    # potentials built in rounds of 16 (atom, term) pairs: same values as
    # rounds of 32 up to the order of the FP32 sums, parity with the oracle
    job = w.c1_tiny(n_frames=16)
    _, a, _ = run_gpu(tacaw, ctx, job)
    monkeypatch.setenv("TACAW_SPLAT_ROUND", "16")
    check_job(tacaw, ctx, oracle, job)
    _, b, _ = run_gpu(tacaw, ctx, job)
    assert rel_l2(b, a) < 1e-5


def test_splat_slice_groups_bitwise(tacaw, ctx, monkeypatch):
    # potentials of several slices per launch (8 slices in groups of 3: 3+3+2)
    job = w.c1_tiny(n_frames=16)
    _, a, _ = run_gpu(tacaw, ctx, job)
    monkeypatch.setenv("TACAW_SPLAT_GROUP", "3")
    monkeypatch.setenv("TACAW_FB", "6")
    _, b, _ = run_gpu(tacaw, ctx, job)
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


@pytest.mark.parametrize("probes", [0, 2], ids=["plane", "probes"])
def test_per_frame_slice_binning(tacaw, ctx, oracle, probes):
    # atoms oscillating across slice boundaries, binned frame by frame
    # (TACAW_SLICE_BY_INSTANT_Z), against the oracle's per-frame binning
    import dataclasses
    job = w.random_small_job(48, nx=48, ny=32, n_slices=4, n_frames=12, n_atoms=10, cell=(7.0, 5.0, 4.0),
                             aperture_mrad=25.0 if probes else 0.0, n_probes=max(probes, 1))
    rng = np.random.default_rng(48)
    pos = job.positions.copy()
    t = np.arange(job.n_frames)[:, None]
    pos[:, :, 2] = rng.integers(1, 4, size=job.n_atoms)[None, :] + 0.3 * np.sin(
        2 * np.pi * t / job.n_frames + rng.uniform(0, 6, job.n_atoms)[None, :])
    job = dataclasses.replace(job, positions=pos, slice_by_instant_z=True)
    with tacaw.TacawJob(ctx, job) as j:
        j.run()
        ex, spec = j.exit_waves(), j.spectrum()
    ref_ex = oracle.exit_waves(job)
    check_parity(ex, spec, ref_ex, oracle.tacaw_spectrum(ref_ex), label="per-frame binning")
    # the frame-mean binning gives a different result on this trajectory
    mean = oracle.exit_waves(dataclasses.replace(job, slice_by_instant_z=False), frames=[0, 5])
    assert rel_l2(ex[:, [0, 5]], mean) > 2 * EXIT_TOL


def test_integer_pixel_translation_leaves_spectrum(tacaw, ctx):
    # moving every atom by whole pixels translates each potential exactly on the
    # periodic grid; the exit wave gains a frame-independent phase in k, which
    # the mean subtraction and |.|^2 remove, so I(k, w) is unchanged (up to the
    # rounding of the shifted positions)
    import dataclasses
    job = w.random_small_job(49, nx=64, ny=48, n_slices=3, n_frames=16, n_atoms=12, cell=(8.0, 6.0, 4.0))
    dx, dy = job.cell[0] / job.nx, job.cell[1] / job.ny
    pos = job.positions.copy()
    pos[:, :, 0] = np.mod(pos[:, :, 0] + 13 * dx, job.cell[0])
    pos[:, :, 1] = np.mod(pos[:, :, 1] + 29 * dy, job.cell[1])
    moved = dataclasses.replace(job, positions=pos)
    _, a, _ = run_gpu(tacaw, ctx, job)
    _, b, _ = run_gpu(tacaw, ctx, moved)
    assert rel_l2(b, a) < 1e-4
