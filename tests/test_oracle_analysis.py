"""Pins of the oracle's spectrum analysis (dispersion, spectral diffraction,
spectrum image; Methods 2.1 "Data Structure Design", Supplement MWE) against
hand-computed values and brute-force counts."""
import numpy as np

from oracle import tacaw_oracle as o


def test_frequency_bin_mwe():
    # the MWE's 200 frames at 10 fs: bins of 0.5 THz, 15 THz is bin 30
    assert o.frequency_bin(15.0, 200, 10.0) == 30
    assert o.frequency_bin(15.2, 200, 10.0) == 30
    assert o.frequency_bin(15.3, 200, 10.0) == 31
    assert o.frequency_bin(0.0, 200, 10.0) == 0
    # two-sided: -3 THz is fftfreq index 200 - 6
    assert o.frequency_bin(-3.0, 200, 10.0, two_sided=True) == 194
    # one-sided: above the last kept bin (49.5 THz) the last bin is nearest
    assert o.frequency_bin(60.0, 200, 10.0) == 99


def test_spectral_diffraction_sums_probes():
    rng = np.random.default_rng(0)
    spec = rng.random((3, 5, 4, 6)).astype(np.float32)
    d = o.spectral_diffraction(spec, 2)
    assert d.shape == (4, 6)
    assert np.allclose(d, spec[0, 2] + spec[1, 2] + spec[2, 2])


def test_spectrum_image_annulus_counts_nodes():
    # a flat spectrum: each probe's value is the number of nodes in the annulus
    nx, ny, d = 16, 12, 0.2
    kx, ky = o.k_axis(nx, d), o.k_axis(ny, d)
    spec = np.ones((2, 3, ny, nx), np.float32)
    k_in, k_out = 0.5, 1.6
    count = 0
    for iy in range(ny):
        for ix in range(nx):
            k = np.hypot(kx[ix], ky[iy])
            count += k_in <= k < k_out
    s = o.spectrum_image(spec, 1, kx, ky, k_in, k_out)
    assert np.array_equal(s, [count, count])
    # no bounds: every node
    assert np.array_equal(o.spectrum_image(spec, 0, kx, ky), [nx * ny, nx * ny])


def test_two_reductions_agree():
    # the total over k of a spectral diffraction pattern equals the total over
    # probes of the full-k spectrum image
    rng = np.random.default_rng(1)
    spec = rng.random((4, 6, 8, 10)).astype(np.float32)
    kx, ky = o.k_axis(10, 0.3), o.k_axis(8, 0.3)
    for m in range(6):
        assert np.isclose(o.spectral_diffraction(spec, m).sum(), o.spectrum_image(spec, m, kx, ky).sum())


def test_dispersion_nearest_nodes():
    rng = np.random.default_rng(2)
    nx, ny, lx, ly = 10, 8, 5.0, 4.0
    spec = rng.random((2, 7, ny, nx)).astype(np.float32)
    # exact grid points, a negative frequency (wraps to the last index), a
    # point just below half way to the next node; points past half way up
    # (2.6 nodes -> 3) and down (-2.4 nodes -> -2), where rounding and
    # truncation differ; a tie half way (2.5 nodes) goes to the upper node
    kx = np.array([0.0, 3 / lx, -1 / lx, 2.49 / lx, 2.6 / lx, -2.4 / lx, 2.5 / lx, 0.0])
    ky = np.array([0.0, 1 / ly, 0.0, -2 / ly, -2.4 / ly, 2.6 / ly, 0.0, 1.5 / ly])
    d = o.dispersion(spec, kx, ky, lx, ly)
    want = [(0, 0), (1, 3), (0, nx - 1), (ny - 2, 2), (ny - 2, 3), (3, nx - 2), (0, 3), (2, 0)]
    for i, (iy, ix) in enumerate(want):
        assert np.allclose(d[i], spec[0, :, iy, ix] + spec[1, :, iy, ix])
