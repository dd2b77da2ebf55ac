"""Pins for the oracle's reciprocal-space potential (CPU only).

Methods 2.2, "Atomic Scattering Potentials": the paper builds each slice's
projected potential from the structure-factor sum V(k) = sum_j f_Z(k)
exp(-2 pi i k.r_j) with the 3 Lorentzian + 3 Gaussian form factor
f(q) = sum_i a_i/(q^2 + b_i) + c_i exp(-d_i q^2), followed by an inverse FFT.
The oracle evaluates it at the grid's own frequencies (band-limited).  These
tests pin it against things other than its own formula:

* the Gaussian part alone equals the (separately pinned) real-space route
  when the Gaussians are wide enough for neither aliasing nor band limit to
  matter;
* the Lorentzian part equals the band of the closed-form projected
  Lorentzian 2 pi a K0(2 pi sqrt(b) r), summed over periodic images and
  sampled on finer grids (Richardson-extrapolated);
* the cell mean is the forward-scattering amplitude sum_j f_Z(0) C / A;
* an explicit cosine sum over atoms and frequencies on a small rectangular
  grid (brute force, including the Nyquist reading).
"""
import math

import numpy as np
import pytest
from scipy.special import k0


def _kirk(a=(0, 0, 0), b=(1, 1, 1), c=(0, 0, 0), d=(1, 1, 1)):
    return np.array(list(a) + list(b) + list(c) + list(d), dtype=np.float64)


@pytest.mark.parametrize("seed", [0, 1])
def test_gaussian_part_equals_realspace_route(oracle, seed):
    # Lorentzian amplitudes zero; Gaussians with d >= 1.2 A^2 on a grid with
    # k_Nyquist ~ 6 / A: exp(-d k^2) < 1e-18 beyond the band, so the band-limited
    # sum equals the point samples of the real-space Gaussian projection
    rng = np.random.default_rng(seed)
    lx, ly, nx, ny = 5.3, 4.1, 64, 50
    xy = rng.uniform(0, 1, (4, 2)) * [lx, ly]
    xy[0] = [0.02, ly - 0.01]
    species = np.array([0, 1, 1, 0])
    kirk = np.zeros((2, 12))
    ga = np.zeros((2, 5))
    gb = np.ones((2, 5))
    for s in range(2):
        c = rng.uniform(0.05, 0.3, 3)
        d = rng.uniform(1.2, 4.0, 3)
        kirk[s] = _kirk(c=c, d=d)
        ga[s, :3], gb[s, :3] = c, d          # two unused real-space terms of amplitude 0
    v_k = oracle.kspace_potential(xy, species, kirk, lx, ly, nx, ny)
    v_r = oracle.projected_potential(xy, species, ga, gb, lx, ly, nx, ny)
    assert np.max(np.abs(v_k - v_r)) < 1e-11 * np.max(np.abs(v_r))


def _lorentzian_band_from_k0(lx, ly, nx, ny, a, b, xj, yj, m_fine, cpref):
    """Band-limited potential of one Lorentzian term from its closed-form
    projection C a 2 pi K0(2 pi sqrt(b) r) (all images within 3 cells),
    sampled on a grid m_fine times finer with the atom centred in a fine cell,
    transformed, cut to the coarse band and transformed back."""
    fx, fy = nx * m_fine, ny * m_fine
    ox = (xj % (lx / fx)) - 0.5 * lx / fx
    oy = (yj % (ly / fy)) - 0.5 * ly / fy
    gx = np.arange(fx) * lx / fx + ox
    gy = np.arange(fy) * ly / fy + oy
    v = np.zeros((fy, fx))
    for m in range(-3, 4):
        for n in range(-3, 4):
            dx = gx[None, :] - xj - m * lx
            dy = gy[:, None] - yj - n * ly
            v += k0(2 * math.pi * math.sqrt(b) * np.sqrt(dx * dx + dy * dy))
    v *= cpref * a * 2 * math.pi
    # Fourier coefficients of the samples, referred back to the unshifted origin
    kfx = np.fft.fftfreq(fx, lx / fx)
    kfy = np.fft.fftfreq(fy, ly / fy)
    ck = np.fft.fft2(v) / (fx * fy) * np.exp(-2j * math.pi * (kfx[None, :] * ox + kfy[:, None] * oy))
    ix = np.round(np.fft.fftfreq(nx, 1.0 / nx)).astype(int) % fx
    iy = np.round(np.fft.fftfreq(ny, 1.0 / ny)).astype(int) % fy
    band = ck[np.ix_(iy, ix)]
    return (np.fft.ifft2(band) * nx * ny).real


@pytest.mark.parametrize("a,b,xj,yj", [(0.37, 1.3, 1.2345, 2.71), (0.8, 0.6, 4.02, 0.33)])
def test_lorentzian_part_equals_k0_projection(oracle, a, b, xj, yj):
    lx, ly, nx, ny = 5.0, 4.0, 40, 32
    cpref = oracle.potential_prefactor()
    kirk = np.array([_kirk(a=(a, 0, 0), b=(b, 1, 1))])
    v = oracle.kspace_potential(np.array([[xj, yj]]), np.array([0]), kirk, lx, ly, nx, ny)
    # the fine-sampling alias error falls as 1/m^2: extrapolate from m = 8, 16
    v8 = _lorentzian_band_from_k0(lx, ly, nx, ny, a, b, xj, yj, 8, cpref)
    v16 = _lorentzian_band_from_k0(lx, ly, nx, ny, a, b, xj, yj, 16, cpref)
    ref = (4 * v16 - v8) / 3
    assert np.max(np.abs(v - ref)) < 2e-5 * np.max(np.abs(ref))
    # and the unextrapolated m = 16 band is already close (guards the extrapolation)
    assert np.max(np.abs(v - v16)) < 2e-3 * np.max(np.abs(ref))


def test_mean_is_forward_scattering(oracle):
    rng = np.random.default_rng(7)
    lx, ly, nx, ny = 6.0, 7.5, 30, 36
    xy = rng.uniform(0, 1, (5, 2)) * [lx, ly]
    species = np.array([0, 1, 1, 0, 1])
    kirk = np.array([_kirk(a=rng.uniform(0.05, 1, 3), b=rng.uniform(0.5, 50, 3),
                           c=rng.uniform(0.005, 0.2, 3), d=rng.uniform(0.1, 4, 3)) for _ in range(2)])
    v = oracle.kspace_potential(xy, species, kirk, lx, ly, nx, ny)
    f0 = [sum(kirk[s, i] / kirk[s, 3 + i] + kirk[s, 6 + i] for i in range(3)) for s in range(2)]
    expect = oracle.potential_prefactor() / (lx * ly) * sum(f0[s] for s in species)
    assert v.mean() == pytest.approx(expect, rel=1e-13)


def test_brute_force_cosine_sum(oracle):
    # V(r) = (C/A) sum over the 6 x 10 grid frequencies and atoms of
    # f(|k|) cos(2 pi k.(r - r_j)); an even grid's Nyquist frequency enters
    # once, at -N/2 / L (numpy fftfreq), which the cosine makes real
    lx, ly, nx, ny = 2.7, 4.4, 6, 10
    xy = np.array([[0.31, 3.9], [2.05, 1.17]])
    species = np.array([1, 0])
    kirk = np.array([_kirk(a=(0.3, 0.1, 0.05), b=(2.0, 9.0, 30.0), c=(0.02, 0.1, 0.05), d=(0.4, 1.1, 3.0)),
                     _kirk(a=(0.6, 0.2, 0.01), b=(1.0, 5.0, 20.0), c=(0.15, 0.01, 0.07), d=(0.2, 2.0, 0.7))])
    v = oracle.kspace_potential(xy, species, kirk, lx, ly, nx, ny)
    cpref = oracle.potential_prefactor()
    ref = np.zeros((ny, nx))
    for py in range(ny):
        for px in range(nx):
            x, y = px * lx / nx, py * ly / ny
            acc = 0.0
            for my in range(ny):
                ky = (my if my < (ny + 1) // 2 else my - ny) / ly
                for mx in range(nx):
                    kx = (mx if mx < (nx + 1) // 2 else mx - nx) / lx
                    q2 = kx * kx + ky * ky
                    for j in range(2):
                        p = kirk[species[j]]
                        f = sum(p[i] / (q2 + p[3 + i]) + p[6 + i] * math.exp(-p[9 + i] * q2)
                                for i in range(3))
                        acc += f * math.cos(2 * math.pi * (kx * (x - xy[j, 0]) + ky * (y - xy[j, 1])))
            ref[py, px] = cpref / (lx * ly) * acc
    assert np.max(np.abs(v - ref)) < 1e-12 * np.max(np.abs(ref))


def test_frame_potentials_take_the_kspace_route(oracle):
    rng = np.random.default_rng(11)
    pos = rng.uniform(0, 5, (5, 3))
    slice_of = np.array([0, 2, 2, 1, 0])
    sp = np.array([0, 1, 0, 1, 1])
    kirk = np.array([_kirk(a=(0.2, 0.1, 0.3), b=(1, 4, 9), c=(0.1, 0.02, 0.05), d=(0.5, 1.0, 2.0)),
                     _kirk(a=(0.4, 0.05, 0.1), b=(2, 6, 12), c=(0.03, 0.1, 0.01), d=(0.3, 1.5, 3.0))])
    pots = oracle.frame_potentials(pos, sp, slice_of, None, None, 5.0, 5.0, 16, 20, 4, kirk)
    assert np.all(pots[3] == 0)
    one = oracle.kspace_potential(pos[[1, 2], :2], sp[[1, 2]], kirk, 5.0, 5.0, 16, 20)
    assert np.array_equal(pots[2], one)
