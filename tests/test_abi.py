"""The C-ABI library loads, exports every symbol include/tacaw.h declares, and
its host-only logic (validation, footprint, axes) behaves.  No GPU needed:
nothing here launches a kernel."""
import os
import re

import numpy as np
import pytest

from paper_2602_10064_amd import workloads as w

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tacaw.h")


def _tacaw():
    from paper_2602_10064_amd import tacaw
    if not os.path.exists(tacaw.LIB_PATH):
        pytest.skip("libtacaw.so not built (run __graft_entry__.build())")
    return tacaw


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tacaw_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["tacaw_ctx_create", "tacaw_job_create", "tacaw_run", "tacaw_submit", "tacaw_poll",
                 "tacaw_wait", "tacaw_cancel", "tacaw_get_spectrum", "tacaw_get_exit_waves",
                 "tacaw_axes", "tacaw_job_destroy", "tacaw_last_error", "tacaw_job_footprint"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    t = _tacaw()
    L = t.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
    assert set(t.EXPORTED) == set(declared_functions())
    assert "gfx950" in t.version()


def test_axes_match_oracle(oracle):
    t = _tacaw()
    for job in (w.c1_tiny(n_frames=64), w.random_small_job(3, nx=48, ny=32, n_frames=12),
                w.random_small_job(4, nx=32, ny=32, n_frames=10, two_sided=True)):
        kx, ky, f = t.axes(job)
        lx, ly, _, pnx, pny, dx, dy = oracle.job_geometry(job)
        assert np.array_equal(kx, oracle.k_axis(job.nx, dx))
        assert np.array_equal(ky, oracle.k_axis(job.ny, dy))
        assert np.allclose(f, oracle.freq_axis_THz(job.n_frames, job.dt_fs, job.two_sided),
                           rtol=1e-15, atol=1e-12)


def test_validation_errors():
    t = _tacaw()
    base = w.random_small_job(1, nx=16, ny=16, n_frames=8)
    assert t.footprint(base) > 0
    bad = [
        base.replace(nx=14),                                  # prime factor 7
        base.replace(n_slices=0),
        base.replace(voltage_V=-1.0),
        base.replace(dt_fs=0.0),
        base.replace(positions=base.positions[:7]),           # 7 frames
        base.replace(aperture_mrad=30.0, probe_xy=np.zeros((0, 2))),
        base.replace(aperture_mrad=900.0, probe_xy=np.zeros((1, 2))),   # aperture beyond Nyquist
        base.replace(pot_nx=32, pot_ny=32),                  # window with a plane wave
        base.replace(gauss_b=-base.gauss_b),
    ]
    for j in bad:
        with pytest.raises(t.TacawError) as e:
            t.footprint(j)
        assert e.value.status == 1, (j, e.value)
    with pytest.raises(t.TacawError) as e:
        t.footprint(base.replace(nx=25 * 81))                 # smooth, but no kernel for it
    assert e.value.status == 7


def test_footprint_scales_with_frames_and_probes():
    t = _tacaw()
    a = t.footprint(w.random_small_job(1, nx=32, ny=32, n_frames=8))
    b = t.footprint(w.random_small_job(1, nx=32, ny=32, n_frames=16))
    assert b > a
    c2 = w.c2_plain(n_frames=2).replace(positions=np.zeros((1024, 1, 3)), atom_species=np.zeros(1, np.int32))
    # exit waves (2 GiB) + one-sided spectrum (512 MiB) dominate the c2 footprint
    assert t.footprint(c2) > (2 << 30) + (512 << 20)


def test_per_frame_binning_footprint_and_limit():
    t = _tacaw()
    base = w.random_small_job(2, nx=16, ny=16, n_frames=8, n_atoms=12)
    inst = base.replace(slice_by_instant_z=True)
    # the per-frame slice table adds 2 bytes per frame and atom
    assert t.footprint(inst) == t.footprint(base) + 2 * base.n_frames * base.n_atoms
    with pytest.raises(t.TacawError) as e:
        t.footprint(inst.replace(n_slices=40000))            # 16-bit slice indices
    assert e.value.status == 1


def test_kspace_route_validation_and_footprint():
    # the paper's reciprocal-space potential route: coefficient checks, the
    # potential grid must have FFT plans, and the slice-pair structure factors
    # add to the footprint
    t = _tacaw()
    base = w.with_kirkland(w.random_small_job(5, nx=32, ny=32, n_frames=8, n_slices=4), seed=1)
    real = base.replace(kirkland=None)
    assert t.footprint(base) > t.footprint(real)
    assert t.footprint(base.replace(gauss_a=None, gauss_b=None)) == t.footprint(base)
    for col in (3, 4, 5):                                    # b must be > 0
        k = base.kirkland.copy()
        k[0, col] = 0.0
        with pytest.raises(t.TacawError) as e:
            t.footprint(base.replace(kirkland=k))
        assert e.value.status == 1
    k = base.kirkland.copy()
    k[1, 10] = -0.5                                          # d must be >= 0
    with pytest.raises(t.TacawError) as e:
        t.footprint(base.replace(kirkland=k))
    assert e.value.status == 1
    k = base.kirkland.copy()
    k[0, 0] = np.nan
    with pytest.raises(t.TacawError) as e:
        t.footprint(base.replace(kirkland=k))
    assert e.value.status == 1
    # a window on a potential grid without FFT plans (1000 x 866) is refused
    win = base.replace(aperture_mrad=30.0, probe_xy=np.array([[3.0, 3.0]]), pot_nx=1000, pot_ny=866,
                       cell=np.array([100.0, 86.6, 4.0]))
    with pytest.raises(t.TacawError) as e:
        t.footprint(win)
    assert e.value.status == 7
    assert t.footprint(win.replace(kirkland=None)) > 0
