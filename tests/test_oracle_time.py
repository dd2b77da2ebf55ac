"""Pins for the oracle's TACAW time transform (CPU only): Wiener-Khinchin
equality with the autocorrelation route that names the method, explicit DFT
loops, a single tone, Parseval, circular frame shifts and the static limit."""
import cmath
import math

import numpy as np
import pytest


def _rand_exit(rng, p=2, f=12, ny=3, nx=4):
    return rng.standard_normal((p, f, ny, nx)) + 1j * rng.standard_normal((p, f, ny, nx))


@pytest.mark.parametrize("n_f", [8, 12, 15])
def test_wiener_khinchin(oracle, n_f):
    ex = _rand_exit(np.random.default_rng(n_f), f=n_f)
    a = oracle.tacaw_spectrum(ex, two_sided=True)
    b = oracle.autocorrelation_spectrum(ex, two_sided=True)
    assert np.max(np.abs(a - b)) < 1e-13 * np.max(a)


@pytest.mark.parametrize("n_f", [8, 12])
def test_bruteforce_dft(oracle, n_f):
    ex = _rand_exit(np.random.default_rng(100 + n_f), p=1, f=n_f, ny=2, nx=2)
    got = oracle.tacaw_spectrum(ex, two_sided=True)
    for y in range(2):
        for x in range(2):
            col = [ex[0, f, y, x] for f in range(n_f)]
            mean = sum(col) / n_f
            for m in range(n_f):
                acc = 0j
                for f in range(n_f):
                    acc += (col[f] - mean) * cmath.exp(-2j * math.pi * m * f / n_f)
                assert got[0, m, y, x] == pytest.approx(abs(acc / n_f) ** 2, rel=1e-12, abs=1e-15)


def test_single_tone(oracle):
    n_f, m0, eps = 64, 5, 0.01
    f = np.arange(n_f)
    col = 0.7 - 0.2j + eps * np.exp(2j * math.pi * m0 * f / n_f)
    ex = col[None, :, None, None]
    spec = oracle.tacaw_spectrum(ex)
    assert spec.shape == (1, 32, 1, 1)
    assert spec[0, m0, 0, 0] == pytest.approx(eps * eps, rel=1e-12)
    others = np.delete(spec[0, :, 0, 0], m0)
    assert np.max(others) < 1e-28


def test_parseval_and_dc(oracle):
    ex = _rand_exit(np.random.default_rng(7), f=16)
    spec = oracle.tacaw_spectrum(ex, two_sided=True)
    d = ex - ex.mean(axis=1, keepdims=True)
    assert np.allclose(spec.sum(axis=1), np.mean(np.abs(d) ** 2, axis=1), rtol=1e-12)
    assert np.max(spec[:, 0]) < 1e-28


def test_circular_frame_shift_invariance(oracle):
    ex = _rand_exit(np.random.default_rng(8), f=20)
    a = oracle.tacaw_spectrum(ex)
    b = oracle.tacaw_spectrum(np.roll(ex, 7, axis=1))
    assert np.max(np.abs(a - b)) < 1e-14 * np.max(a)


def test_static_trajectory_gives_zero(oracle):
    from paper_2602_10064_amd import workloads as w
    job = w.random_small_job(2, n_frames=6)
    job.positions[:] = job.positions[0:1]
    ex, spec = oracle.run_job(job)
    assert np.max(np.abs(ex - ex[:, :1])) == 0.0
    assert np.max(spec) < 1e-30          # only the rounding of the mean remains


def test_c1_oracle_run_sanity(oracle):
    from paper_2602_10064_amd import workloads as w
    job = w.c1_tiny(n_frames=16)
    ex, spec = oracle.run_job(job)
    assert ex.shape == (1, 16, 64, 64) and spec.shape == (1, 8, 64, 64)
    assert np.max(np.abs(np.sum(np.abs(ex) ** 2, axis=(2, 3)) - 1)) < 1e-13
    assert np.max(spec[:, 0]) < 1e-25 * np.max(spec)
    assert np.max(spec[:, 1:]) > 0
