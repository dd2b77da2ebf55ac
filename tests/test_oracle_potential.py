"""Pins for the oracle's projected potential (CPU only).

The main pin is the paper's own route (Methods 2.2, Atomic Scattering
Potentials): V(k) = sum_j f_Z(k) exp(-2 pi i k.r_j) followed by an inverse FFT.
Point-sampling the real-space potential on the grid equals the inverse DFT of
the structure factor with all reciprocal-lattice aliases folded in (Poisson
summation), so the two independent codes must agree to rounding.
"""
import math

import numpy as np
import pytest


def _reciprocal_route(xy, species, ga, gb, lx, ly, nx, ny, cpref, n_alias=6):
    kx = np.fft.fftfreq(nx, lx / nx)
    ky = np.fft.fftfreq(ny, ly / ny)
    vk = np.zeros((ny, nx), dtype=np.complex128)
    for mx in range(-n_alias, n_alias + 1):
        for my in range(-n_alias, n_alias + 1):
            qx = kx[None, :] + mx * nx / lx
            qy = ky[:, None] + my * ny / ly
            q2 = qx * qx + qy * qy
            for j in range(len(xy)):
                s = species[j]
                f = cpref * np.sum(ga[s][:, None, None] * np.exp(-gb[s][:, None, None] * q2[None]),
                                   axis=0)
                vk += f * np.exp(-2j * math.pi * (qx * xy[j, 0] + qy * xy[j, 1]))
    # V(r_p) = (1/A) sum_k Vk exp(+2 pi i k r_p); numpy ifft2 carries 1/(nx ny)
    return np.fft.ifft2(vk) * (nx * ny) / (lx * ly)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_realspace_splat_equals_structure_factor_route(oracle, seed):
    rng = np.random.default_rng(seed)
    lx, ly, nx, ny = 7.3, 6.1, 48, 40                  # non-square, dx ~ 0.15 A
    xy = rng.uniform(0, 1, (3, 2)) * [lx, ly]
    xy[0] = [0.01, ly - 0.02]                          # atom near the cell corner
    species = np.array([0, 1, 1])
    ga = rng.uniform(0.1, 2.0, (2, 5))
    gb = rng.uniform(0.3, 10.0, (2, 5))
    v = oracle.projected_potential(xy, species, ga, gb, lx, ly, nx, ny)
    ref = _reciprocal_route(xy, species, ga, gb, lx, ly, nx, ny, oracle.potential_prefactor())
    assert np.max(np.abs(ref.imag)) < 1e-9 * np.max(np.abs(v))
    assert np.max(np.abs(v - ref.real)) < 1e-10 * np.max(np.abs(v))


def test_narrow_gaussian_aliasing_matches_too(oracle):
    # b = 0.1 A^2 is narrower than a pixel: the point samples alias; the reciprocal
    # route with folded aliases reproduces that exactly.
    lx = ly = 4.0
    nx = ny = 24
    xy = np.array([[1.234, 2.71]])
    ga = np.array([[1.0, 0.5, 0.3, 0.2, 0.1]])
    gb = np.array([[0.1, 0.2, 0.5, 1.0, 4.0]])
    v = oracle.projected_potential(xy, np.array([0]), ga, gb, lx, ly, nx, ny)
    ref = _reciprocal_route(xy, [0], ga, gb, lx, ly, nx, ny, oracle.potential_prefactor(),
                            n_alias=8)
    assert np.max(np.abs(v - ref.real)) < 1e-10 * np.max(np.abs(v))


def test_direct_2d_image_sum_small_cell(oracle):
    # literal definition: explicit double loop over images and the radial form
    lx, ly, nx, ny = 3.0, 2.5, 12, 10
    xy = np.array([[0.3, 2.4], [2.2, 1.0]])
    sp = np.array([0, 0])
    ga = np.array([[0.7, 0.4, 1.1, 0.2, 0.9]])
    gb = np.array([[0.5, 1.5, 3.0, 6.0, 9.5]])
    v = oracle.projected_potential(xy, sp, ga, gb, lx, ly, nx, ny)
    cpref = oracle.potential_prefactor()
    ref = np.zeros((ny, nx))
    for py in range(ny):
        for px in range(nx):
            x, y = px * lx / nx, py * ly / ny
            acc = 0.0
            for j in range(2):
                for m in range(-12, 13):
                    for n in range(-12, 13):
                        r2 = (x - xy[j, 0] - m * lx) ** 2 + (y - xy[j, 1] - n * ly) ** 2
                        for i in range(5):
                            acc += cpref * ga[0, i] * math.pi / gb[0, i] * math.exp(
                                -math.pi ** 2 * r2 / gb[0, i])
            ref[py, px] = acc
    assert np.max(np.abs(v - ref)) < 1e-12 * np.max(np.abs(ref))


def test_integral_equals_forward_scattering(oracle):
    # int v d^2r = C sum_i a_i  (f(q=0)); wide Gaussians on a fine grid -> no aliasing
    lx = ly = 12.0
    nx = ny = 96
    ga = np.array([[0.3, 0.6, 0.9, 1.2, 1.5]])
    gb = np.array([[2.0, 3.0, 4.0, 6.0, 9.0]])
    v = oracle.projected_potential(np.array([[5.1, 3.3]]), np.array([0]), ga, gb, lx, ly,
                                   nx, ny)
    integral = v.sum() * (lx / nx) * (ly / ny)
    assert integral == pytest.approx(oracle.potential_prefactor() * ga.sum(), rel=1e-12)


def test_frame_potentials_respect_slices(oracle):
    rng = np.random.default_rng(3)
    pos = rng.uniform(0, 5, (4, 3))
    slice_of = np.array([0, 2, 2, 1])
    ga = np.ones((1, 5))
    gb = np.full((1, 5), 2.0)
    pots = oracle.frame_potentials(pos, np.zeros(4, int), slice_of, ga, gb, 5.0, 5.0, 16, 16, 4)
    assert np.all(pots[3] == 0)
    one = oracle.projected_potential(pos[[1, 2], :2], np.zeros(2, int), ga, gb, 5.0, 5.0, 16, 16)
    assert np.allclose(pots[2], one, rtol=0, atol=1e-13)
