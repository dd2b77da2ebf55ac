"""Pins for the oracle's constants, axes and slice binning (CPU only).

Each check compares the oracle with something other than itself: an
independently written closed form, a limit, the paper's printed worked
numbers (tests/golden/mwe_sampling.json), or integer counts fixed by the
lattice geometry.
"""
import json
import math
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("volt", [20e3, 60e3, 100e3, 200e3, 300e3])
def test_sigma_matches_kirkland_closed_form(oracle, volt):
    # sigma = (2 pi / (lambda E)) (m0 c^2 + eE) / (2 m0 c^2 + eE), with energies in eV
    mc2_eV = 510998.95000
    lam = oracle.wavelength_A(volt)
    alt = 2 * math.pi / (lam * volt) * (mc2_eV + volt) / (2 * mc2_eV + volt)
    assert oracle.sigma_rad_per_VA(volt) == pytest.approx(alt, rel=1e-12)


@pytest.mark.parametrize("volt", [60e3, 100e3, 200e3])
def test_wavelength_relativistic_momentum(oracle, volt):
    # pc = sqrt(E_k^2 + 2 E_k m c^2); lambda = hc / pc, hc = 12398.419843320026 eV A
    mc2_eV = 510998.95000
    pc = math.sqrt(volt * volt + 2.0 * volt * mc2_eV)
    assert oracle.wavelength_A(volt) == pytest.approx(12398.419843320026 / pc, rel=1e-10)


def test_wavelength_nonrelativistic_limit(oracle):
    # lambda -> h / sqrt(2 m e E) = 12.2643 / sqrt(E[V]) A for E << m c^2
    for volt in (0.1, 1.0, 10.0):
        assert oracle.wavelength_A(volt) == pytest.approx(12.26426 / math.sqrt(volt), rel=1e-5)


def test_potential_prefactor_is_2pi_hbar2_over_m(oracle):
    # a0 * e^2/(4 pi eps0) = hbar^2 / m_e; expressed in eV A^2 via hbar c and m c^2
    hbar_c_eVA = 1973.2698044604
    mc2_eV = 510998.95000
    assert oracle.potential_prefactor() == pytest.approx(
        2 * math.pi * hbar_c_eVA ** 2 / mc2_eV, rel=1e-9)


def test_mwe_sampling_numbers(oracle):
    g = json.load(open(os.path.join(GOLDEN, "mwe_sampling.json")))
    for case in g["cases"]:
        if "df_THz" in case:
            f = oracle.freq_axis_THz(case["n_frames"], case["dt_fs"])
            assert f[1] - f[0] == pytest.approx(case["df_THz"], rel=1e-12)
        if "fmax_THz" in case:
            f2 = oracle.freq_axis_THz(case["n_frames"], case["dt_fs"], two_sided=True)
            assert np.max(np.abs(f2)) == pytest.approx(case["fmax_THz"], rel=1e-12)
        if "dk_inv_A" in case:
            n = 1086
            k = oracle.k_axis(n, case["L_A"] / n)
            assert k[1] == pytest.approx(case["dk_inv_A"], rel=case["rel_tol"])
        if "kmax_inv_A" in case:
            k = oracle.k_axis(1000, case["sampling_A"])
            assert np.max(np.abs(k)) == pytest.approx(case["kmax_inv_A"], rel=1e-12)
        if "frames" in case:
            assert case["production_steps"] // case["save_interval"] == case["frames"]
            assert case["md_dt_fs"] * case["save_interval"] == case["frame_dt_fs"]


def test_one_sided_axis_drops_negative_half(oracle):
    f = oracle.freq_axis_THz(64, 5.0)
    assert len(f) == 32 and f[0] == 0.0
    assert f[1] == pytest.approx(3.125)            # 1 / (64 * 5 fs)
    assert f[-1] == pytest.approx(31 * 3.125)


def test_k_axis_layout(oracle):
    k = oracle.k_axis(8, 0.5)                        # L = 4 A -> dk = 0.25
    assert np.allclose(k, [0, .25, .5, .75, -1.0, -.75, -.5, -.25])


def test_slice_binning_counts(oracle):
    from paper_2602_10064_amd import workloads as w
    j1 = w.c1_tiny(n_frames=8)
    s1 = oracle.slice_index(j1.positions, j1.cell[2], j1.n_slices)
    assert np.array_equal(np.bincount(s1, minlength=8), np.full(8, 8))
    j2 = w.c2_plain(n_frames=2)
    s2 = oracle.slice_index(j2.positions, j2.cell[2], j2.n_slices)
    assert np.array_equal(np.bincount(s2, minlength=32), np.full(32, 288))


def test_slice_binning_half_open_wrap_and_clamp(oracle):
    lz, ns = 10.0, 4                                  # dz = 2.5
    z = np.array([0.0, 2.5, 2.4999999, 9.9999, 10.0, -0.1, 12.6, 7.5])
    pos = np.zeros((3, len(z), 3))
    pos[:, :, 2] = z[None, :]
    s = oracle.slice_index(pos, lz, ns)
    assert list(s) == [0, 1, 0, 3, 0, 3, 1, 3]
    # binning follows the frame mean, not instantaneous z
    pos2 = np.zeros((2, 1, 3))
    pos2[:, 0, 2] = [2.4, 2.8]                         # mean 2.6 -> slice 1
    assert oracle.slice_index(pos2, lz, ns)[0] == 1
