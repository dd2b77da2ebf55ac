"""Pins of the oracle's conventional-STEM additions: aberrated probes and
ADF/HAADF detector integration ("Beyond Vibrational Spectroscopy"; Methods 2.1
HAADFData).  Each aberration term is checked against a closed form that does
not go through the general polar sum, or against the Fresnel propagator."""
import math

import numpy as np

from oracle import tacaw_oracle as o
from paper_2602_10064_amd import workloads as w

LAM = o.wavelength_A(100e3)


def coeffs(**kw):
    """(C_nm, phi_nm) arrays from keywords such as C10=..., phi12=..."""
    c, a = np.zeros(14), np.zeros(14)
    for i, (n, m) in enumerate(o.ABERRATIONS):
        c[i] = kw.get(f"C{n}{m}", 0.0)
        a[i] = kw.get(f"phi{n}{m}", 0.0)
    return c, a


def grid(nx=48, ny=40, dx=0.11, dy=0.13):
    return nx, ny, dx, dy, o.k_axis(nx, dx), o.k_axis(ny, dy)


def test_defocus_is_fresnel_propagation():
    # C10 = z: the probe is the focused probe propagated over z in vacuum
    nx, ny, dx, dy, kx, ky = grid()
    z = 37.5
    focused = o.probe_wave(nx, ny, dx, dy, LAM, 0.03, 2.1, 1.7)
    moved = np.fft.ifft2(o.propagator(nx, ny, dx, dy, LAM, z) * np.fft.fft2(focused, norm="ortho"), norm="ortho")
    got = o.probe_wave(nx, ny, dx, dy, LAM, 0.03, 2.1, 1.7, coeffs(C10=z))
    assert np.allclose(got, moved, atol=1e-13)


def test_spherical_and_defocus_textbook_form():
    # chi = pi lambda k^2 (Cs lambda^2 k^2 / 2 - df) with df = -C10
    nx, ny, dx, dy, kx, ky = grid()
    cs, c10 = 1.2e7, -850.0
    chi = o.aberration_chi(kx, ky, LAM, *coeffs(C10=c10, C30=cs))
    k2 = kx[None, :] ** 2 + ky[:, None] ** 2
    ref = math.pi * LAM * k2 * (0.5 * cs * LAM ** 2 * k2 + c10)
    assert np.allclose(chi, ref, rtol=1e-12, atol=1e-9)
    # fifth order: chi = pi C5 lambda^5 k^6 / 3
    chi5 = o.aberration_chi(kx, ky, LAM, *coeffs(C50=3.0e9))
    assert np.allclose(chi5, math.pi * 3.0e9 * LAM ** 5 * k2 ** 3 / 3.0, rtol=1e-12, atol=1e-9)


def test_two_fold_astigmatism_closed_forms():
    nx, ny, dx, dy, kx, ky = grid()
    c12 = 55.0
    # phi12 = 0: pi lambda C12 (kx^2 - ky^2); pi/4: pi lambda C12 (2 kx ky)
    chi0 = o.aberration_chi(kx, ky, LAM, *coeffs(C12=c12))
    chi45 = o.aberration_chi(kx, ky, LAM, *coeffs(C12=c12, phi12=math.pi / 4))
    kxx, kyy = np.meshgrid(kx, ky)
    assert np.allclose(chi0, math.pi * LAM * c12 * (kxx ** 2 - kyy ** 2), atol=1e-10)
    assert np.allclose(chi45, math.pi * LAM * c12 * 2 * kxx * kyy, atol=1e-10)
    # as a probe: separable x and y Fresnel factors of opposite sign
    a = 0.03
    got = o.probe_wave(nx, ny, dx, dy, LAM, a, 1.0, 2.0, coeffs(C12=c12))
    kk = np.sqrt(kxx ** 2 + kyy ** 2)
    spec = (LAM * kk <= a) * np.exp(-2j * math.pi * (kxx * 1.0 + kyy * 2.0))
    spec = spec * np.exp(-1j * math.pi * LAM * c12 * kxx ** 2) * np.exp(1j * math.pi * LAM * c12 * kyy ** 2)
    ref = np.fft.ifft2(spec, norm="ortho")
    ref /= np.linalg.norm(ref)
    assert np.allclose(got, ref, atol=1e-13)


def test_coma_closed_form():
    # C21 along x: chi = (2 pi / 3) lambda^2 C21 |k|^2 kx
    nx, ny, dx, dy, kx, ky = grid()
    chi = o.aberration_chi(kx, ky, LAM, *coeffs(C21=4.0e3))
    kxx, kyy = np.meshgrid(kx, ky)
    assert np.allclose(chi, 2 * math.pi / 3 * LAM ** 2 * 4.0e3 * (kxx ** 2 + kyy ** 2) * kxx, atol=1e-10)


def test_m_fold_rotation_symmetry():
    # rotating k by t and every phi_nm by t leaves chi unchanged; phi_nm + 2 pi / m too
    rng = np.random.default_rng(3)
    c = rng.uniform(-1, 1, 14) * np.array([1e2, 1e2, 1e3, 1e3, 1e5, 1e5, 1e5, 1e6, 1e6, 1e6, 1e8, 1e8, 1e8, 1e8])
    a = rng.uniform(0, 2 * math.pi, 14)
    ms = np.array([m for _, m in o.ABERRATIONS])
    for kx0, ky0 in [(0.31, -0.12), (-0.05, 0.47), (0.6, 0.6)]:
        base = o.aberration_chi(np.array([kx0]), np.array([ky0]), LAM, c, a)[0, 0]
        t = 0.73
        rx, ry = kx0 * math.cos(t) - ky0 * math.sin(t), kx0 * math.sin(t) + ky0 * math.cos(t)
        assert np.isclose(o.aberration_chi(np.array([rx]), np.array([ry]), LAM, c, a + t)[0, 0], base,
                          rtol=1e-10, atol=1e-9)
        shifted = a + np.where(ms > 0, 2 * math.pi / np.maximum(ms, 1), 0.0)
        assert np.isclose(o.aberration_chi(np.array([kx0]), np.array([ky0]), LAM, c, shifted)[0, 0], base,
                          rtol=1e-10, atol=1e-9)


def test_aberrations_change_only_the_phase():
    # |psi(k)| of an aberrated probe is the flat aperture disc
    nx, ny, dx, dy, kx, ky = grid()
    a = 0.025
    p = o.probe_wave(nx, ny, dx, dy, LAM, a, 3.0, 1.0, coeffs(C10=-120.0, C30=2e6, C23=800.0, phi23=0.4))
    mag = np.abs(np.fft.fft2(p, norm="ortho"))
    kk = np.sqrt(kx[None, :] ** 2 + ky[:, None] ** 2)
    ap = LAM * kk <= a
    assert np.allclose(mag, ap / math.sqrt(ap.sum()), atol=1e-13)


def test_mean_diffraction_by_hand():
    ex = np.zeros((1, 2, 2, 2), np.complex128)
    ex[0, 0] = [[1.0, 1j], [0.0, 0.5]]
    ex[0, 1] = [[0.0, 1.0], [2.0, 0.5j]]
    assert np.allclose(o.mean_diffraction(ex)[0], [[0.5, 1.0], [2.0, 0.25]])


def test_adf_of_a_probe_through_vacuum():
    # no atoms: |psi(k)|^2 = A(k) / count, so a detector reads its share of
    # aperture nodes, counted by brute force
    job = w.random_small_job(70, nx=32, ny=24, n_slices=2, n_frames=2, n_atoms=0, aperture_mrad=25.0,
                             n_probes=2, cell=(5.0, 4.0, 3.0))
    ex = o.exit_waves(job)
    dx, dy = job.cell[0] / job.nx, job.cell[1] / job.ny
    kx, ky = o.k_axis(job.nx, dx), o.k_axis(job.ny, dy)
    lam = o.wavelength_A(job.voltage_V)
    d = o.mean_diffraction(ex)
    inside = total = 0
    for iy in range(job.ny):
        for ix in range(job.nx):
            th = 1e3 * lam * math.hypot(kx[ix], ky[iy])
            total += th <= 25.0
            inside += 10.0 <= th < 20.0
    assert np.allclose(o.adf(d, kx, ky, lam, 10.0, 20.0), inside / total, atol=1e-12)
    assert np.allclose(o.adf(d, kx, ky, lam, 0.0, 1e9), 1.0, atol=1e-12)
    assert np.allclose(o.adf(d, kx, ky, lam, 25.1, 1e9), 0.0, atol=1e-12)


def test_adf_full_detector_is_unitary():
    # with atoms, a detector covering every node collects the whole unit norm
    job = w.random_small_job(71, nx=32, ny=32, n_slices=3, n_frames=3, n_atoms=6, aperture_mrad=20.0,
                             n_probes=2)
    ex = o.exit_waves(job)
    dx = job.cell[0] / job.nx
    kx = o.k_axis(job.nx, dx)
    lam = o.wavelength_A(job.voltage_V)
    full = o.adf(o.mean_diffraction(ex), kx, kx, lam, 0.0, 1e9)
    assert np.allclose(full, 1.0, atol=1e-12)
    # and the annuli partition it
    parts = sum(o.adf(o.mean_diffraction(ex), kx, kx, lam, a, b) for a, b in [(0, 20), (20, 60), (60, 1e9)])
    assert np.allclose(parts, full, atol=1e-14)
