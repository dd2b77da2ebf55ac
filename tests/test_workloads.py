"""Checks of the seeded input generators (CPU only)."""
import numpy as np

from paper_2602_10064_amd import workloads as w


def test_c1_shape_and_rms():
    j = w.c1_tiny()
    assert j.positions.shape == (64, 64, 3)
    assert np.allclose(j.cell, [10.86, 10.86, 10.86])
    lat, _ = w.diamond_cubic(5.43, (2, 2, 2), z_shift=10.86 / 16)
    u = j.positions - lat[None]
    u[:, :, :2] = (u[:, :, :2] + 5.43) % 10.86 - 5.43     # undo the xy wrap
    assert np.allclose(np.sqrt(np.mean(u * u, axis=(0, 1))), 0.08, rtol=1e-12)


def test_c2_species_split_and_counts():
    j = w.c2_plain(n_frames=2)
    assert j.n_atoms == 9216
    assert np.bincount(j.atom_species).tolist() == [4608, 4608]
    assert j.nx == j.ny == 512 and j.n_slices == 32


def test_seed_determinism():
    a = w.c1_tiny(n_frames=4)
    b = w.c1_tiny(n_frames=4)
    assert np.array_equal(a.positions, b.positions)
    assert np.array_equal(a.gauss_a, b.gauss_a)


def test_gaussian_coefficient_ranges():
    a, b = w.gaussian_coefficients(7, [3, 14, 40])
    assert a.shape == (3, 5) and np.all((a >= 0.1) & (a <= 2.0))
    assert np.all((b >= 0.1) & (b <= 10.0))


def test_c3_geometry():
    j = w.c3_probe(n_frames=2)
    assert j.n_atoms == 38400
    assert np.allclose(j.cell[:2], [100.0, 20 * 2.5 * np.sqrt(3)])
    assert j.n_probes == 1024 and j.pot_nx == 1000 and j.pot_ny == 866


def test_c4_jobs_are_smooth_and_snapped():
    for jj in range(6):
        j = w.c4_job(jj, frames_range=(128, 160))
        assert j.nx in (128, 256, 384, 512)
        f = j.n_frames
        for p in (2, 3, 5):
            while f % p == 0:
                f //= p
        assert f == 1
        dz = j.cell[2] / j.n_slices
        zbar = j.positions[:, :, 2].mean(axis=0)
        frac = zbar / dz - np.floor(zbar / dz)
        assert np.min(np.abs(frac - 0.5)) < 0.5 and np.min(frac) > 0.05 and np.max(frac) < 0.95
