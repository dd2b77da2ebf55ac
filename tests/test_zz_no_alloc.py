"""The allocation-free spectrum image against tacaw_spectrum_image, through
the C ABI (needs an MI355X).

Both entry points run the same reduction kernel over the same resident
spectrum, so results must be equal bit for bit: two calls in a row, the
second on a smaller job (fewer probes, smaller grid), to host and to device
destinations, plus the error paths (no run yet, more probes than the fixed
scratch holds)."""
import numpy as np
import pytest

from paper_2602_10064_amd import workloads as w

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


def _check_pair(tacaw, j, job, f_THz, k_in, k_out):
    import torch
    ref = j.spectrum_image(f_THz, k_in, k_out)
    got = j.spectrum_image_noalloc(f_THz, k_in, k_out)
    assert got.shape == ref.shape == (job.n_probes,)
    assert np.array_equal(got, ref), (got, ref)
    dev = torch.full((job.n_probes,), -1.0, dtype=torch.float64, device="cuda")
    j.spectrum_image_noalloc(f_THz, k_in, k_out, out=dev)
    torch.cuda.synchronize()
    assert np.array_equal(dev.cpu().numpy(), ref)
    return ref


def test_noalloc_spectrum_image_matches_two_calls(tacaw, ctx):
    big = w.random_small_job(71, nx=48, ny=32, n_slices=2, n_frames=16, n_atoms=6, aperture_mrad=40.0,
                             n_probes=7, cell=(6.0, 4.0, 3.0), voltage_V=100e3)
    small = w.random_small_job(72, nx=16, ny=16, n_slices=1, n_frames=8, n_atoms=4, aperture_mrad=40.0,
                               n_probes=3, cell=(4.0, 4.0, 2.0), voltage_V=100e3)
    print(f"[gpu] noalloc: {big.n_probes} probes {big.nx}x{big.ny}, then {small.n_probes} probes "
          f"{small.nx}x{small.ny}", flush=True)
    with tacaw.TacawJob(ctx, big) as jb, tacaw.TacawJob(ctx, small) as js:
        jb.run()
        js.run()
        f_big = 2.0 / (big.n_frames * big.dt_fs * 1e-3)     # bin 2
        r1 = _check_pair(tacaw, jb, big, f_big, 0.2, 1.5)
        f_small = 1.0 / (small.n_frames * small.dt_fs * 1e-3)
        r2 = _check_pair(tacaw, js, small, f_small, 0.0, 0.0)
        assert np.all(r1 > 0) and np.all(r2 > 0)
        # and back to the larger job: the shared array holds the small job's sums
        _check_pair(tacaw, jb, big, f_big, 0.0, 0.9)


def test_noalloc_errors(tacaw, ctx):
    job = w.random_small_job(73, nx=16, ny=16, n_slices=1, n_frames=8, n_atoms=3, aperture_mrad=40.0,
                             n_probes=2, cell=(4.0, 4.0, 2.0))
    with tacaw.TacawJob(ctx, job) as j:
        with pytest.raises(tacaw.TacawError) as e:
            j.spectrum_image_noalloc(10.0)
        assert e.value.status == 5          # ENOTREADY: not run yet
    many = w.random_small_job(74, nx=16, ny=16, n_slices=1, n_frames=8, n_atoms=3, aperture_mrad=40.0,
                              n_probes=65537, cell=(6.0, 6.0, 2.0))
    print(f"[gpu] noalloc: {many.n_probes} probes (beyond the fixed scratch)", flush=True)
    with tacaw.TacawJob(ctx, many) as j:
        j.run()
        with pytest.raises(tacaw.TacawError) as e:
            j.spectrum_image_noalloc(0.0)
        assert e.value.status == 1          # EINVAL
        assert "65536" in str(e.value)
        assert j.spectrum_image(0.0).shape == (65537,)
