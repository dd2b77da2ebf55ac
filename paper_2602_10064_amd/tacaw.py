"""ctypes binding of libtacaw (C ABI in include/tacaw.h).

Argument marshalling only: every step of the hot path runs in the library's
HIP kernels.  If ``libtacaw.so`` has not been built, loading fails loudly;
there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libtacaw.so")

TACAW_OK = 0
STATUS_NAMES = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EDEVICE", 4: "EBUSY", 5: "ENOTREADY",
                6: "ECANCELLED", 7: "EUNSUPPORTED"}
TWO_SIDED = 1
KEEP_EXIT_WAVES = 2
DEFER_ALLOC = 4
USE_GRAPH = 8
SLICE_BY_INSTANT_Z = 16

K_SPLAT, K_ROW, K_COL, K_TIME, K_OTHER = range(5)
KERNEL_CLASSES = {"splat": K_SPLAT, "row": K_ROW, "col": K_COL, "time": K_TIME, "other": K_OTHER}


class TacawError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class JobDesc(ctypes.Structure):
    _fields_ = [
        ("cell", ctypes.c_double * 3),
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("n_slices", ctypes.c_int32),
        ("voltage_V", ctypes.c_double),
        ("aperture_mrad", ctypes.c_double),
        ("n_probes", ctypes.c_int32),
        ("probe_xy", ctypes.POINTER(ctypes.c_double)),
        ("pot_nx", ctypes.c_int32), ("pot_ny", ctypes.c_int32),
        ("dt_fs", ctypes.c_double),
        ("n_frames", ctypes.c_int32),
        ("n_atoms", ctypes.c_int32),
        ("n_species", ctypes.c_int32),
        ("species_Z", ctypes.POINTER(ctypes.c_int32)),
        ("gauss_a", ctypes.POINTER(ctypes.c_double)),
        ("gauss_b", ctypes.POINTER(ctypes.c_double)),
        ("flags", ctypes.c_uint32),
        ("kspace_coef", ctypes.POINTER(ctypes.c_double)),
    ]


_lib = None

EXPORTED = [
    "tacaw_ctx_create", "tacaw_ctx_destroy", "tacaw_job_footprint", "tacaw_job_create", "tacaw_run",
    "tacaw_submit", "tacaw_poll", "tacaw_wait", "tacaw_cancel", "tacaw_get_spectrum",
    "tacaw_get_exit_waves", "tacaw_axes", "tacaw_job_slices", "tacaw_job_destroy", "tacaw_last_error",
    "tacaw_timing_enable", "tacaw_timing_select", "tacaw_timing_get", "tacaw_version", "tacaw_job_latency",
    "tacaw_run_batch", "tacaw_autotune", "tacaw_job_plan",
    "tacaw_spectral_diffraction", "tacaw_spectrum_image", "tacaw_spectrum_image_noalloc", "tacaw_dispersion",
    "tacaw_job_set_aberrations", "tacaw_mean_diffraction", "tacaw_adf",
    "tacaw_run_frames", "tacaw_finish", "tacaw_get_exit_frames", "tacaw_put_exit_frames",
    "tacaw_average_spectra", "tacaw_batch_capture", "tacaw_batch_launch", "tacaw_batch_destroy",
    "tacaw_serve_stats",
]


def lib() -> ctypes.CDLL:
    """Load libtacaw.so (built in-tree by paper_2602_10064_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2602_10064_amd.build`"
                           " (the HIP library is the only implementation)")
    L = ctypes.CDLL(LIB_PATH)
    vp, sz, i32, dp = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_double
    P = ctypes.POINTER
    sig = {
        "tacaw_ctx_create": [ctypes.c_int, sz, P(vp)],
        "tacaw_ctx_destroy": [vp],
        "tacaw_job_footprint": [P(JobDesc), P(sz)],
        "tacaw_job_create": [vp, P(JobDesc), P(i32), P(dp), P(vp)],
        "tacaw_run": [vp, vp],
        "tacaw_submit": [vp, vp],
        "tacaw_poll": [vp, P(ctypes.c_int)],
        "tacaw_wait": [vp],
        "tacaw_cancel": [vp],
        "tacaw_get_spectrum": [vp, vp, sz, ctypes.c_int],
        "tacaw_get_exit_waves": [vp, vp, sz, ctypes.c_int],
        "tacaw_axes": [P(JobDesc), P(dp), P(dp), P(dp)],
        "tacaw_job_slices": [vp, P(i32), sz],
        "tacaw_job_destroy": [vp],
        "tacaw_timing_enable": [vp, ctypes.c_int],
        "tacaw_timing_select": [vp, ctypes.c_uint, ctypes.c_int],
        "tacaw_timing_get": [vp, ctypes.c_int, P(dp), P(ctypes.c_int64)],
        "tacaw_job_latency": [vp, P(dp), P(dp)],
        "tacaw_serve_stats": [vp, P(ctypes.c_int64), P(ctypes.c_int64)],
        "tacaw_run_batch": [P(vp), ctypes.c_int, vp],
        "tacaw_autotune": [vp, vp, P(ctypes.c_int), P(ctypes.c_int)],
        "tacaw_job_plan": [vp, P(i32), P(i32)],
        "tacaw_spectral_diffraction": [vp, dp, vp, sz, ctypes.c_int],
        "tacaw_spectrum_image": [vp, dp, dp, dp, vp, sz, ctypes.c_int],
        "tacaw_spectrum_image_noalloc": [vp, dp, dp, dp, vp, sz, ctypes.c_int],
        "tacaw_dispersion": [vp, P(dp), P(dp), i32, vp, sz, ctypes.c_int],
        "tacaw_job_set_aberrations": [vp, P(dp), P(dp)],
        "tacaw_mean_diffraction": [vp, vp, sz, ctypes.c_int],
        "tacaw_adf": [vp, dp, dp, vp, sz, ctypes.c_int],
        "tacaw_run_frames": [vp, i32, i32, vp],
        "tacaw_finish": [vp, vp],
        "tacaw_get_exit_frames": [vp, i32, i32, vp, sz, ctypes.c_int],
        "tacaw_put_exit_frames": [vp, i32, i32, vp, sz, ctypes.c_int],
        "tacaw_average_spectra": [P(vp), i32, vp, sz, ctypes.c_int],
        "tacaw_batch_capture": [P(vp), i32, P(vp)],
        "tacaw_batch_launch": [vp, vp],
        "tacaw_batch_destroy": [vp],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    L.tacaw_last_error.restype = ctypes.c_char_p
    L.tacaw_last_error.argtypes = []
    L.tacaw_version.restype = ctypes.c_char_p
    L.tacaw_version.argtypes = []
    _lib = L
    return L


def _check(status: int):
    if status != TACAW_OK:
        raise TacawError(status, lib().tacaw_last_error().decode(errors="replace"))


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


class _DescHolder:
    """A JobDesc plus the numpy arrays its pointers refer to (kept alive)."""

    def __init__(self, job, keep_exit_waves: Optional[bool] = None):
        self.species_Z = np.ascontiguousarray(job.species_Z, dtype=np.int32)
        self.gauss_a = None if job.gauss_a is None else np.ascontiguousarray(job.gauss_a, dtype=np.float64)
        self.gauss_b = None if job.gauss_b is None else np.ascontiguousarray(job.gauss_b, dtype=np.float64)
        self.probe_xy = np.ascontiguousarray(job.probe_xy, dtype=np.float64).reshape(-1, 2)
        if self.probe_xy.size == 0:
            self.probe_xy = np.zeros((1, 2))
        d = JobDesc()
        d.cell[:] = [float(v) for v in job.cell]
        d.nx, d.ny, d.n_slices = int(job.nx), int(job.ny), int(job.n_slices)
        d.voltage_V = float(job.voltage_V)
        d.aperture_mrad = float(job.aperture_mrad)
        d.n_probes = int(job.probe_xy.shape[0]) if job.aperture_mrad > 0 else 1
        d.probe_xy = _ptr(self.probe_xy, ctypes.c_double)
        d.pot_nx, d.pot_ny = int(job.pot_nx), int(job.pot_ny)
        d.dt_fs = float(job.dt_fs)
        d.n_frames = int(job.positions.shape[0])
        d.n_atoms = int(job.positions.shape[1])
        d.n_species = int(len(self.species_Z))
        d.species_Z = _ptr(self.species_Z, ctypes.c_int32)
        if self.gauss_a is not None and self.gauss_b is not None:
            d.gauss_a = _ptr(self.gauss_a, ctypes.c_double)
            d.gauss_b = _ptr(self.gauss_b, ctypes.c_double)
        keep = job.keep_exit_waves if keep_exit_waves is None else keep_exit_waves
        d.flags = (TWO_SIDED if job.two_sided else 0) | (KEEP_EXIT_WAVES if keep else 0)
        if getattr(job, "slice_by_instant_z", False):
            d.flags |= SLICE_BY_INSTANT_Z
        kirk = getattr(job, "kirkland", None)
        if kirk is not None:        # the paper's reciprocal-space potential route
            self.kspace_coef = np.ascontiguousarray(kirk, dtype=np.float64).reshape(len(self.species_Z), 12)
            d.kspace_coef = _ptr(self.kspace_coef, ctypes.c_double)
        self.desc = d


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)      # torch.cuda.Stream


class Context:
    """tacaw_ctx: a device, a memory budget, timing and the serving loop."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        h = ctypes.c_void_p()
        _check(lib().tacaw_ctx_create(int(device), int(hbm_budget_bytes), ctypes.byref(h)))
        self.handle = h
        self.device = device

    def close(self):
        if self.handle:
            _check(lib().tacaw_ctx_destroy(self.handle))
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def timing_enable(self, on: bool = True):
        _check(lib().tacaw_timing_enable(self.handle, 1 if on else 0))

    def timing_select(self, classes=None, every: int = 1):
        """Time only these kernel classes (names or numbers; None: all), one
        launch in `every` of each."""
        if classes is None:
            mask = 0xFFFFFFFF
        else:
            mask = 0
            for k in classes:
                mask |= 1 << (KERNEL_CLASSES[k] if isinstance(k, str) else int(k))
        _check(lib().tacaw_timing_select(self.handle, ctypes.c_uint(mask), int(every)))

    def timing_get(self, kernel_class) -> tuple:
        cls = KERNEL_CLASSES[kernel_class] if isinstance(kernel_class, str) else int(kernel_class)
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        _check(lib().tacaw_timing_get(self.handle, cls, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def submit(self, job: "TacawJob"):
        _check(lib().tacaw_submit(self.handle, job.handle))

    def serve_stats(self) -> tuple:
        """(pass launches of the serving loop that served several jobs, served
        jobs that shared at least one launch with another job)."""
        a, b = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().tacaw_serve_stats(self.handle, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value


class TacawJob:
    """tacaw_job created from a workloads.Job (inputs copied by the library)."""

    def __init__(self, ctx: Context, job, keep_exit_waves: Optional[bool] = None,
                 defer_alloc: bool = False, use_graph: bool = False):
        self.ctx = ctx
        self.job = job
        self._d = _DescHolder(job, keep_exit_waves)
        if defer_alloc:
            self._d.desc.flags |= DEFER_ALLOC
        if use_graph:
            self._d.desc.flags |= USE_GRAPH
        sp = np.ascontiguousarray(job.atom_species, dtype=np.int32)
        pos = np.ascontiguousarray(job.positions, dtype=np.float64)
        h = ctypes.c_void_p()
        _check(lib().tacaw_job_create(ctx.handle, ctypes.byref(self._d.desc), _ptr(sp, ctypes.c_int32),
                                      _ptr(pos, ctypes.c_double), ctypes.byref(h)))
        self.handle = h
        self.n_probes = self._d.desc.n_probes
        self.n_frames = self._d.desc.n_frames
        self.n_bins = self.n_frames if job.two_sided else self.n_frames // 2
        self.nx, self.ny = job.nx, job.ny
        self.aberrations = None
        ab = getattr(job, "aberrations", None)
        if ab is not None:
            self.set_aberrations(ab[0], ab[1])

    # plain per-job form
    def run(self, stream=None):
        _check(lib().tacaw_run(self.handle, _stream_handle(stream)))

    # serving form
    def poll(self) -> bool:
        d = ctypes.c_int()
        _check(lib().tacaw_poll(self.handle, ctypes.byref(d)))
        return bool(d.value)

    def wait(self):
        _check(lib().tacaw_wait(self.handle))

    def cancel(self):
        _check(lib().tacaw_cancel(self.handle))

    def submit(self):
        _check(lib().tacaw_submit(self.ctx.handle, self.handle))

    def autotune(self, stream=None) -> tuple:
        """Pick the faster row/column tile variants for this grid size."""
        r = ctypes.c_int()
        c = ctypes.c_int()
        _check(lib().tacaw_autotune(self.handle, _stream_handle(stream), ctypes.byref(r), ctypes.byref(c)))
        return r.value, c.value

    def latency_ms(self) -> tuple:
        """(queued_ms, total_ms) of a job that finished in the serving loop."""
        q = ctypes.c_double()
        t = ctypes.c_double()
        _check(lib().tacaw_job_latency(self.handle, ctypes.byref(q), ctypes.byref(t)))
        return q.value, t.value

    @property
    def spectrum_shape(self):
        return (self.n_probes, self.n_bins, self.ny, self.nx)

    @property
    def exit_shape(self):
        return (self.n_probes, self.n_frames, self.ny, self.nx)

    def spectrum(self, out=None):
        """I[p][m][ky][kx] float32 into a new numpy array, or into `out` (numpy or
        a CUDA torch tensor)."""
        n = int(np.prod(self.spectrum_shape))
        if out is None:
            out = np.empty(self.spectrum_shape, dtype=np.float32)
        if isinstance(out, np.ndarray):
            assert out.dtype == np.float32 and out.flags.c_contiguous and out.size == n
            _check(lib().tacaw_get_spectrum(self.handle, out.ctypes.data, n, 0))
        else:
            assert out.is_cuda and out.is_contiguous() and out.numel() == n
            _check(lib().tacaw_get_spectrum(self.handle, out.data_ptr(), n, 1))
        return out

    def exit_waves(self, out=None):
        """psi[p][f][ky][kx] complex64 into a new numpy array or into `out`."""
        n = int(np.prod(self.exit_shape))
        if out is None:
            out = np.empty(self.exit_shape, dtype=np.complex64)
        if isinstance(out, np.ndarray):
            assert out.dtype == np.complex64 and out.flags.c_contiguous and out.size == n
            _check(lib().tacaw_get_exit_waves(self.handle, out.ctypes.data, n, 0))
        else:
            assert out.is_cuda and out.is_contiguous() and out.numel() == n
            _check(lib().tacaw_get_exit_waves(self.handle, out.data_ptr(), n, 1))
        return out

    def slices(self) -> np.ndarray:
        n = int(self._d.desc.n_atoms)
        out = np.empty(n, dtype=np.int32)
        _check(lib().tacaw_job_slices(self.handle, _ptr(out, ctypes.c_int32), n))
        return out

    def spectral_diffraction(self, f_THz: float) -> np.ndarray:
        """Sum over probes of I at the kept frequency bin nearest f_THz: [ny, nx] float64."""
        out = np.empty((self.ny, self.nx), dtype=np.float64)
        _check(lib().tacaw_spectral_diffraction(self.handle, float(f_THz), out.ctypes.data, out.size, 0))
        return out

    def spectrum_image(self, f_THz: float, k_inner: float = 0.0, k_outer: float = 0.0) -> np.ndarray:
        """Per probe: sum of I at the bin nearest f_THz over k_inner <= |k| < k_outer."""
        out = np.empty(self.n_probes, dtype=np.float64)
        _check(lib().tacaw_spectrum_image(self.handle, float(f_THz), float(k_inner), float(k_outer),
                                          out.ctypes.data, out.size, 0))
        return out

    def spectrum_image_noalloc(self, f_THz: float, k_inner: float = 0.0, k_outer: float = 0.0,
                               out=None) -> np.ndarray:
        """spectrum_image through the allocation-free entry point; `out` may be
        a float64 torch tensor on the job's device (one value per probe)."""
        if out is not None:
            _check(lib().tacaw_spectrum_image_noalloc(self.handle, float(f_THz), float(k_inner),
                                                      float(k_outer), out.data_ptr(), out.numel(), 1))
            return out
        res = np.empty(self.n_probes, dtype=np.float64)
        _check(lib().tacaw_spectrum_image_noalloc(self.handle, float(f_THz), float(k_inner), float(k_outer),
                                                  res.ctypes.data, res.size, 0))
        return res

    def dispersion(self, kx, ky) -> np.ndarray:
        """Sum over probes of I at the grid nodes nearest (kx[i], ky[i]): [n_points, M] float64."""
        kx = np.ascontiguousarray(kx, dtype=np.float64)
        ky = np.ascontiguousarray(ky, dtype=np.float64)
        if kx.shape != ky.shape or kx.ndim != 1:
            raise ValueError("kx and ky must be 1-D arrays of one length")
        out = np.empty((kx.size, self.spectrum_shape[1]), dtype=np.float64)
        _check(lib().tacaw_dispersion(self.handle, _ptr(kx, ctypes.c_double), _ptr(ky, ctypes.c_double),
                                      int(kx.size), out.ctypes.data, out.size, 0))
        return out

    # frame ranges and checkpoints
    def run_frames(self, f_begin: int, f_end: int, stream=None) -> None:
        """Exit waves of frames [f_begin, f_end) only; the spectrum waits for finish()."""
        _check(lib().tacaw_run_frames(self.handle, int(f_begin), int(f_end), _stream_handle(stream)))

    def finish(self, stream=None) -> None:
        """Time stage over the complete exit store."""
        _check(lib().tacaw_finish(self.handle, _stream_handle(stream)))

    def exit_frames(self, f_begin: int, f_end: int) -> np.ndarray:
        """Frames [f_begin, f_end) of the exit store: [P, frames, ny, nx] complex64."""
        out = np.empty((self.n_probes, f_end - f_begin, self.ny, self.nx), dtype=np.complex64)
        _check(lib().tacaw_get_exit_frames(self.handle, int(f_begin), int(f_end), out.ctypes.data, out.size, 0))
        return out

    def put_exit_frames(self, f_begin: int, waves: np.ndarray) -> None:
        """Restore frames [f_begin, f_begin + waves.shape[1]) of the exit store."""
        w = np.ascontiguousarray(waves, dtype=np.complex64)
        if w.ndim != 4 or w.shape[0] != self.n_probes or w.shape[2:] != (self.ny, self.nx):
            raise ValueError(f"need [{self.n_probes}, frames, {self.ny}, {self.nx}] exit waves")
        _check(lib().tacaw_put_exit_frames(self.handle, int(f_begin), int(f_begin + w.shape[1]), w.ctypes.data,
                                           w.size, 0))

    def set_aberrations(self, c_angstrom=None, phi_rad=None) -> None:
        """Probe aberrations: 14 polar coefficients C_nm [A] and angles [rad]
        for (n, m) = 10, 12, 21, 23, 30, 32, 34, 41, 43, 45, 50, 52, 54, 56."""
        if c_angstrom is None:
            _check(lib().tacaw_job_set_aberrations(self.handle, None, None))
            self.aberrations = None
            return
        c = np.ascontiguousarray(c_angstrom, dtype=np.float64).reshape(-1)
        a = np.zeros(14) if phi_rad is None else np.ascontiguousarray(phi_rad, dtype=np.float64).reshape(-1)
        if c.size != 14 or a.size != 14:
            raise ValueError("need 14 aberration coefficients and 14 angles")
        _check(lib().tacaw_job_set_aberrations(self.handle, _ptr(c, ctypes.c_double), _ptr(a, ctypes.c_double)))
        self.aberrations = (c.copy(), a.copy())

    def mean_diffraction(self) -> np.ndarray:
        """Frame-averaged diffraction pattern of every probe: [P, ny, nx] float64."""
        out = np.empty((self.n_probes, self.ny, self.nx), dtype=np.float64)
        _check(lib().tacaw_mean_diffraction(self.handle, out.ctypes.data, out.size, 0))
        return out

    def adf(self, inner_mrad: float, outer_mrad: float) -> np.ndarray:
        """Annular detector signal per probe over inner <= angle < outer (mrad)."""
        out = np.empty(self.n_probes, dtype=np.float64)
        _check(lib().tacaw_adf(self.handle, float(inner_mrad), float(outer_mrad), out.ctypes.data, out.size, 0))
        return out

    def plan(self) -> tuple:
        """(frames per batch, slices per potential launch) chosen by the planner."""
        fb, g = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().tacaw_job_plan(self.handle, ctypes.byref(fb), ctypes.byref(g)))
        return fb.value, g.value

    def destroy(self):
        if self.handle:
            _check(lib().tacaw_job_destroy(self.handle))
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.destroy()


def run_batch(jobs, stream=None):
    """tacaw_run_batch over a list of TacawJob of one context."""
    arr = (ctypes.c_void_p * len(jobs))(*[j.handle.value for j in jobs])
    _check(lib().tacaw_run_batch(arr, len(jobs), _stream_handle(stream)))


class Batch:
    """tacaw_batch: the batched launch sequence of a list of TacawJob,
    captured once as a HIP graph and replayed with launch()."""

    def __init__(self, jobs):
        self.jobs = list(jobs)
        arr = (ctypes.c_void_p * len(self.jobs))(*[j.handle.value for j in self.jobs])
        h = ctypes.c_void_p()
        _check(lib().tacaw_batch_capture(arr, len(self.jobs), ctypes.byref(h)))
        self.handle = h

    def launch(self, stream=None):
        _check(lib().tacaw_batch_launch(self.handle, _stream_handle(stream)))

    def destroy(self):
        if self.handle:
            _check(lib().tacaw_batch_destroy(self.handle))
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.destroy()


def footprint(job) -> int:
    d = _DescHolder(job)
    b = ctypes.c_size_t()
    _check(lib().tacaw_job_footprint(ctypes.byref(d.desc), ctypes.byref(b)))
    return b.value


def axes(job):
    """(kx[nx], ky[ny], f_THz[M]) as the library reports them."""
    d = _DescHolder(job)
    m = job.n_frames if job.two_sided else job.n_frames // 2
    kx = np.empty(job.nx)
    ky = np.empty(job.ny)
    f = np.empty(m)
    _check(lib().tacaw_axes(ctypes.byref(d.desc), _ptr(kx, ctypes.c_double), _ptr(ky, ctypes.c_double),
                            _ptr(f, ctypes.c_double)))
    return kx, ky, f


def version() -> str:
    return lib().tacaw_version().decode()


def average_spectra(jobs) -> np.ndarray:
    """(1/J) sum_j I_j over jobs with spectra of one shape, on the device: float32."""
    jobs = list(jobs)
    if not jobs:
        raise ValueError("need at least one job")
    arr = (ctypes.c_void_p * len(jobs))(*[j.handle.value for j in jobs])
    out = np.empty(jobs[0].spectrum_shape, dtype=np.float32)
    _check(lib().tacaw_average_spectra(arr, len(jobs), out.ctypes.data, out.size, 0))
    return out
