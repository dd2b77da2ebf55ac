"""Pins of the oracle's trajectory and segment averaging (Methods 2.1
"Molecular Dynamics"; Supplement "Trajectory averaging")."""
import math

import numpy as np

from oracle import tacaw_oracle as o
from paper_2602_10064_amd import workloads as w


def tone(n_p, n_f, ny, nx, amp, q, offset):
    t = np.arange(n_f)
    wave = offset + amp * np.exp(2j * math.pi * q * t / n_f)
    return np.broadcast_to(wave[None, :, None, None], (n_p, n_f, ny, nx)).astype(np.complex128)


def test_segments_of_a_pure_tone():
    # a tone with q cycles over F frames has q / S cycles per segment: every
    # segment's spectrum is |amp|^2 at bin q / S and zero elsewhere, and so is
    # the average
    n_f, s, q, amp = 48, 4, 8, 0.3 - 0.2j
    ex = tone(2, n_f, 3, 5, amp, q, 1.7 + 0.4j)
    avg = o.segment_average_spectrum(ex, s)
    assert avg.shape == (2, n_f // s // 2, 3, 5)
    ref = np.zeros_like(avg)
    ref[:, q // s] = abs(amp) ** 2
    assert np.allclose(avg, ref, atol=1e-15)


def test_one_segment_is_the_plain_spectrum():
    rng = np.random.default_rng(5)
    ex = rng.standard_normal((1, 12, 4, 4)) + 1j * rng.standard_normal((1, 12, 4, 4))
    assert np.array_equal(o.segment_average_spectrum(ex, 1), o.tacaw_spectrum(ex))


def test_average_is_linear_and_segments_tile_the_trajectory():
    rng = np.random.default_rng(6)
    ex = rng.standard_normal((2, 20, 3, 3)) + 1j * rng.standard_normal((2, 20, 3, 3))
    # by hand: the mean of the two halves' spectra
    a = o.tacaw_spectrum(ex[:, :10])
    b = o.tacaw_spectrum(ex[:, 10:])
    assert np.allclose(o.segment_average_spectrum(ex, 2), 0.5 * (a + b), rtol=1e-15, atol=0)
    # Parseval per segment: sum over bins (two-sided) = mean |dpsi|^2
    two = o.segment_average_spectrum(ex, 2, two_sided=True)
    d0 = ex[:, :10] - ex[:, :10].mean(axis=1, keepdims=True)
    d1 = ex[:, 10:] - ex[:, 10:].mean(axis=1, keepdims=True)
    parseval = 0.5 * ((np.abs(d0) ** 2).mean(axis=1) + (np.abs(d1) ** 2).mean(axis=1))
    assert np.allclose(two.sum(axis=1), parseval, rtol=1e-12)


def test_frame_segments_split_the_trajectory():
    job = w.random_small_job(90, n_frames=13, n_atoms=4)
    segs = w.frame_segments(job, 3)
    assert [s.n_frames for s in segs] == [4, 4, 4]
    assert np.array_equal(np.concatenate([s.positions for s in segs]), job.positions[:12])
