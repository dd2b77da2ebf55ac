"""Parity metrics of the GPU tests: the complex64 HIP path against the FP64
oracle (Methods 2.1 time transform; Methods 2.2 multislice).

* Exit waves: relative L2 error <= 1e-4 over the whole array, and also for
  every single (probe, frame) wave.
* Spectrum: relative L2 error <= 1e-3 over the whole array, and a bound on
  every element.  The element bound follows from the arithmetic of the time
  stage.  With e_f(k) the exit-wave error of frame f at k, the mean
  subtraction is an orthogonal projection over frames and the 1/F-normalised
  DFT satisfies Parseval, sum_m |d psi~_m|^2 = (1/F) sum_f |d dpsi_f|^2, so
  every bin's amplitude error is at most E(k) = sqrt(mean_f |e_f(k)|^2).  The
  FP32 time stage adds at most a few eps * log2(F) of the column's rms
  inelastic amplitude S(k); 1e-5 S(k) covers F up to 2048 with margin.  With
  E' = E + 1e-5 S, |I - I_ref| = ||a + d|^2 - |a|^2| <= 2 |a| E' + E'^2 with
  |a| = sqrt(I_ref).  Unlike a bound relative to each bin's maximum, this one
  also holds in bins that hold nothing but rounding.
"""
import numpy as np

EXIT_TOL = 1e-4
SPEC_TOL = 1e-3
TIME_STAGE_REL = 1e-5


def rel_l2(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def per_frame_rel_l2(ex, ref) -> np.ndarray:
    """[P, F] relative L2 error of every (probe, frame) wave."""
    d = np.asarray(ex, np.complex128) - ref
    return np.sqrt(np.sum(np.abs(d) ** 2, axis=(2, 3)) / np.sum(np.abs(ref) ** 2, axis=(2, 3)))


def spectrum_element_bound(ref_spec, ex, ref_ex, two_sided=False) -> np.ndarray:
    """Per-element bound on |I - I_ref| (see the module docstring).

    ex, ref_ex: [P, F, ny, nx] exit waves behind the two spectra (ex may be
    ref_ex itself when both spectra come from the same exit waves)."""
    ref_ex = np.asarray(ref_ex, np.complex128)
    e = np.asarray(ex, np.complex128) - ref_ex
    err = np.sqrt(np.mean(np.abs(e) ** 2, axis=1))[:, None]
    d = ref_ex - ref_ex.mean(axis=1, keepdims=True)
    rms = np.sqrt(np.mean(np.abs(d) ** 2, axis=1))[:, None]
    e_tot = err + TIME_STAGE_REL * rms
    return 2.0 * np.sqrt(np.asarray(ref_spec, np.float64)) * e_tot + e_tot ** 2


def spectrum_element_ratio(spec, ref_spec, ex, ref_ex, two_sided=False) -> float:
    """max over elements of |I - I_ref| / bound (must be <= 1)."""
    bound = spectrum_element_bound(ref_spec, ex, ref_ex, two_sided)
    diff = np.abs(np.asarray(spec, np.float64) - ref_spec)
    # elements where both the bound and the difference are exactly 0 pass
    tiny = np.finfo(np.float64).tiny
    return float(np.max(diff / np.maximum(bound, tiny)))


def check_parity(ex, spec, ref_ex, ref_spec, two_sided=False, label="", exit_tol=EXIT_TOL,
                 spec_tol=SPEC_TOL):
    """Assert every metric above; returns them for printing."""
    e1 = rel_l2(ex, ref_ex)
    e_frame = float(per_frame_rel_l2(ex, ref_ex).max())
    e2 = rel_l2(spec, ref_spec)
    ratio = spectrum_element_ratio(spec, ref_spec, ex, ref_ex, two_sided)
    print(f"[gpu] {label}: exit relL2 {e1:.3e} (worst frame {e_frame:.3e})  spectrum relL2 {e2:.3e}"
          f"  element bound ratio {ratio:.3f}", flush=True)
    assert e1 <= exit_tol
    assert e_frame <= exit_tol
    assert e2 <= spec_tol
    assert ratio <= 1.0
    return e1, e_frame, e2, ratio
