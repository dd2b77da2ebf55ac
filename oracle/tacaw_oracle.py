"""FP64 CPU oracle for the TACAW hot path.

TEST INFRASTRUCTURE ONLY.  This module is the plain, slow reference that the
HIP path is checked against.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import or call it; the product path never
does, and it shares no code with the HIP library (it imports only numpy).

What it computes (paper: PySlice, arXiv 2602.10064):
  * Methods 2.2 "Multislice Propagation": transmission t = exp(i sigma V) per
    slice, Fresnel propagator P(k) = exp(-i pi lambda dz |k|^2) applied in
    reciprocal space between slices, with a relativistic interaction parameter.
  * Methods 2.2 "Atomic Scattering Potentials": per-slice projected potential
    assembled from per-species form factors over the atoms inside the slice's
    z-bounds.  The paper's tabulated Kirkland coefficients are not available;
    a 5-term Gaussian form factor f(q) = C sum_i a_i exp(-b_i q^2) stands in
    (reading R1 below), evaluated in real space.  The paper's own route, its
    3 Lorentzian + 3 Gaussian form summed as a structure factor in reciprocal
    space and inverse-transformed, is kspace_potential (reading R-kspace),
    used when a job carries per-species coefficients of that form.
  * Methods 2.1 "Workflow Architecture": psi~(k, w) = F_t[psi(k,t) - <psi(k,t)>_t]
    and I(k, w) = |psi~(k, w)|^2.
  * Supplement "Sampling Considerations": dk = 1/L, df = 1/(N dt), f_max = 1/(2 dt).

Readings taken where the paper is silent, garbled or inconsistent:
  R-sigma   The interaction parameter is printed as sigma = 2 pi m_e lambda / h^2,
            which drops the electron charge; we use sigma = 2 pi gamma m0 e lambda / h^2.
  R1        Potential prefactor C = 2 pi a0 e (= 47.88 V A^2): the a_i are electron
            form-factor amplitudes in A, so v(r) = C sum_i a_i (pi/b_i) exp(-pi^2 r^2/b_i)
            is the 2D Fourier transform of C sum_i a_i exp(-b_i q^2), in V*A.
  R-images  Every periodic image whose FP64 contribution is non-zero is summed
            (no cutoff).
  R-kspace  The paper's own route (optional, with per-species coefficients of
            its 3 Lorentzian + 3 Gaussian form): V(k) = sum_j f(k) exp(-2 pi i
            k.r_j) at the potential grid's own fftfreq frequencies (one period,
            so the potential is band-limited), inverse FFT, times C/A; the real
            part is kept.  Only the unpaired Nyquist frequencies of even grids
            make the sum complex, so keeping the real part is the same as taking
            each Nyquist term as the mean of its +k and -k images.
  R-bin     An atom belongs to slice floor((zbar mod Lz)/dz) (clamped), zbar being
            its FP64 mean z over all frames; slices are half-open [k dz, (k+1) dz).
            Optionally (slice_by_instant_z) each frame bins by its own z, the
            literal reading of "atoms within the slice z-bounds".
  R-order   The printed product P_{N-1} t_N ... P_0 t_1 has garbled indices; we
            transmit then propagate in every slice, so N propagators, one after the
            last slice, and the exit wave is taken in reciprocal space after it.
  R-fft     FFTs are numpy's (forward kernel exp(-2 pi i k.r), matching the
            exp(-2 pi i k.r_j) phase of the structure-factor sum), 2D transforms
            with norm="ortho", so a plane wave of unit norm stays of unit norm.
  R-probe   Plane wave psi0 = 1/sqrt(Nx Ny).  A convergent probe is a hard
            aperture A(k) = 1 for lambda |k| <= alpha (edge inclusive), times
            exp(-i chi(k)) when aberrations are given (R-aberr), times
            exp(-2 pi i k.r_p), inverse-transformed and normalised to unit norm.  Windowed probes use a window of the wave
            grid cropped (periodic wrap) from the full-cell potential, with origin
            pixel floor(r_p/dx) - N/2; the probe sits at r_p relative to it.
  R-aberr   "Beyond Vibrational Spectroscopy" names the standard aberration
            function (defocus, astigmatism, coma, spherical and higher orders)
            applied at probe formation.  We take the polar-coefficient form
            chi(k) = (2 pi / lambda) sum_nm C_nm alpha^(n+1) / (n+1)
            cos(m (phi - phi_nm)), alpha = lambda |k|, phi = atan2(ky, kx),
            over the 14 coefficients of orders 1..5 listed in ABERRATIONS,
            and the probe factor exp(-i chi).  C10 = z is then the same as
            propagating the focused probe over z with the Fresnel propagator.
  R-adf     ADF/HAADF (HAADFData in Methods 2.1 and "Beyond Vibrational
            Spectroscopy"): the frame-averaged diffraction pattern
            D[p](k) = (1/F) sum_f |psi(p, f, k)|^2 (frozen-phonon average of the
            exit-wave intensities), summed over the detector annulus
            inner <= lambda |k| < outer (angles in mrad, small-angle).
  R-time    Arithmetic mean over all frames per (probe, k); no window; forward
            numpy sign with 1/F normalisation; I_m for m = 0..F/2-1 (one-sided),
            or all F bins when two-sided output is asked for.
"""
from __future__ import annotations

import math

import numpy as np

# CODATA 2018 constants (SI)
_H = 6.62607015e-34          # Planck constant [J s]
_ME = 9.1093837015e-31       # electron rest mass [kg]
_QE = 1.602176634e-19        # elementary charge [C]
_C = 299792458.0             # speed of light [m/s]
_A0 = 0.529177210903         # Bohr radius [A]
_E2_4PIEPS0 = 14.399645478425668  # e^2/(4 pi eps0) [eV A], i.e. "e" as V*A


# ---------------------------------------------------------------------------
# Constants (Methods 2.2, Multislice Propagation)
# ---------------------------------------------------------------------------
def wavelength_A(voltage_V: float) -> float:
    """Relativistic electron wavelength lambda = h / sqrt(2 m0 e E (1 + eE/(2 m0 c^2))) [A]."""
    e_j = _QE * voltage_V
    p = math.sqrt(2.0 * _ME * e_j * (1.0 + e_j / (2.0 * _ME * _C * _C)))
    return _H / p * 1e10


def sigma_rad_per_VA(voltage_V: float) -> float:
    """Interaction parameter sigma = 2 pi gamma m0 e lambda / h^2 [rad / (V A)] (reading R-sigma)."""
    gamma = 1.0 + _QE * voltage_V / (_ME * _C * _C)
    lam_m = wavelength_A(voltage_V) * 1e-10
    return 2.0 * math.pi * gamma * _ME * _QE * lam_m / (_H * _H) * 1e-10


def potential_prefactor() -> float:
    """C = 2 pi a0 e [V A^2] (reading R1)."""
    return 2.0 * math.pi * _A0 * _E2_4PIEPS0


# ---------------------------------------------------------------------------
# Grids and axes (Supplement, Sampling Considerations)
# ---------------------------------------------------------------------------
def k_axis(n: int, d: float) -> np.ndarray:
    """Spatial frequencies in cycles/A, unshifted (DC first); spacing 1/(n d)."""
    return np.fft.fftfreq(n, d)


def freq_axis_THz(n_frames: int, dt_fs: float, two_sided: bool = False) -> np.ndarray:
    """f_m = m / (F dt); one-sided keeps m = 0..F/2-1, two-sided all F in fftfreq order."""
    dt_ps = dt_fs * 1e-3
    f = np.fft.fftfreq(n_frames, dt_ps)
    return f if two_sided else f[: n_frames // 2]


# ---------------------------------------------------------------------------
# Slice binning (Methods 2.2: "atoms within the slice z-bounds"; reading R-bin)
# ---------------------------------------------------------------------------
def slice_index(positions: np.ndarray, lz: float, n_slices: int, instant: bool = False) -> np.ndarray:
    """Slice of every atom: [A] from the FP64 frame-mean z (reading R-bin), or
    [F, A] from each frame's own z when instant (the literal per-frame reading)."""
    z = positions[:, :, 2] if instant else positions[:, :, 2].mean(axis=0)
    dz = lz / n_slices
    s = np.floor(np.mod(z, lz) / dz).astype(np.int64)
    return np.clip(s, 0, n_slices - 1)


# ---------------------------------------------------------------------------
# Projected potential (Methods 2.2 Atomic Scattering Potentials; readings R1, R-images)
# ---------------------------------------------------------------------------
def _periodic_gaussian_1d(grid_x: np.ndarray, x0: float, length: float, c: float) -> np.ndarray:
    """sum over images m of exp(-c (x - x0 - m L)^2), all images with non-zero FP64 value."""
    reach = math.sqrt(800.0 / c)                 # exp(-800) underflows to 0 in FP64
    m_lo = int(math.floor((grid_x.min() - x0 - reach) / length)) - 1
    m_hi = int(math.ceil((grid_x.max() - x0 + reach) / length)) + 1
    out = np.zeros_like(grid_x)
    for m in range(m_lo, m_hi + 1):
        d = grid_x - x0 - m * length
        out += np.exp(-c * d * d)
    return out


def projected_potential(xy: np.ndarray, species: np.ndarray, gauss_a: np.ndarray,
                        gauss_b: np.ndarray, lx: float, ly: float, nx: int, ny: int) -> np.ndarray:
    """V(r_p) = sum_j sum_images v_{Z_j}(r_p - r_j - image) at r_p = (p_x Lx/Nx, p_y Ly/Ny).

    v_Z(r) = C sum_i a_i (pi/b_i) exp(-pi^2 |r|^2 / b_i).  Each isotropic 2D
    Gaussian is the product of two 1D Gaussians and the rectangular lattice of
    images factorises the same way, so
        sum_images exp(-c |r - r_j - (m Lx, n Ly)|^2)
          = [sum_m exp(-c (x - x_j - m Lx)^2)] [sum_n exp(-c (y - y_j - n Ly)^2)].
    Returns V[ny, nx] in V*A (float64).
    The sum over (atom, term) of weight * outer(profile_y, profile_x) is
    evaluated as one matrix product.
    """
    cpref = potential_prefactor()
    gx = np.arange(nx) * (lx / nx)
    gy = np.arange(ny) * (ly / ny)
    n_terms = gauss_a.shape[1]
    k = xy.shape[0] * n_terms
    prof_x = np.zeros((k, nx))
    prof_y = np.zeros((k, ny))
    weight = np.zeros(k)
    for j in range(xy.shape[0]):
        s = int(species[j])
        for i in range(n_terms):
            a_i, b_i = gauss_a[s, i], gauss_b[s, i]
            c = math.pi ** 2 / b_i
            r = j * n_terms + i
            prof_x[r] = _periodic_gaussian_1d(gx, xy[j, 0], lx, c)
            prof_y[r] = _periodic_gaussian_1d(gy, xy[j, 1], ly, c)
            weight[r] = cpref * a_i * math.pi / b_i
    return (prof_y * weight[:, None]).T @ prof_x


def kirkland_form_factor(q2: np.ndarray, p) -> np.ndarray:
    """The paper's parameterised form factor (Methods 2.2, Atomic Scattering
    Potentials): f(q) = sum_{i=1..3} [a_i / (q^2 + b_i) + c_i exp(-d_i q^2)],
    q in cycles/A.  p = (a1, a2, a3, b1, b2, b3, c1, c2, c3, d1, d2, d3) with
    a in 1/A, b in 1/A^2, c in A, d in A^2, so f is in A."""
    p = np.asarray(p, dtype=np.float64)
    out = np.zeros_like(q2, dtype=np.float64)
    for i in range(3):
        out += p[i] / (q2 + p[3 + i]) + p[6 + i] * np.exp(-p[9 + i] * q2)
    return out


def kspace_potential(xy: np.ndarray, species: np.ndarray, kirkland: np.ndarray,
                     lx: float, ly: float, nx: int, ny: int) -> np.ndarray:
    """The paper's reciprocal-space route (Methods 2.2, Atomic Scattering
    Potentials; reading R-kspace): the structure-factor sum
        V(k) = sum_j f_{Z_j}(|k|) exp(-2 pi i k.r_j)
    over the slice's atoms at the grid's own frequencies k (numpy fftfreq of
    the potential grid, one period: band-limited), then an inverse FFT:
        V(r_p) = Re (C/A) sum_k V(k) exp(+2 pi i k.r_p),
    C = 2 pi a0 e (reading R1), A = Lx Ly.  Returns V[ny, nx] in V*A.
    kirkland: [S, 12] coefficients per species (kirkland_form_factor order)."""
    kx = k_axis(nx, lx / nx)
    ky = k_axis(ny, ly / ny)
    q2 = ky[:, None] ** 2 + kx[None, :] ** 2
    vk = np.zeros((ny, nx), dtype=np.complex128)
    for s in np.unique(species):
        # structure factor of the species: sum_j exp(-2 pi i ky y_j) exp(-2 pi i kx x_j)
        sf = np.zeros((ny, nx), dtype=np.complex128)
        for j in np.nonzero(species == s)[0]:
            sf += np.outer(np.exp(-2j * math.pi * ky * xy[j, 1]), np.exp(-2j * math.pi * kx * xy[j, 0]))
        vk += kirkland_form_factor(q2, kirkland[int(s)]) * sf
    # numpy's ifft2 carries 1/(nx ny): (C/A) sum_k = C/(dx dy) ifft2
    return (potential_prefactor() * nx * ny / (lx * ly) * np.fft.ifft2(vk)).real


def frame_potentials(positions_f: np.ndarray, atom_species: np.ndarray, slice_of: np.ndarray,
                     gauss_a: np.ndarray, gauss_b: np.ndarray, lx: float, ly: float,
                     nx: int, ny: int, n_slices: int, kirkland=None) -> np.ndarray:
    """Projected potential of every slice for one frame: [n_slices, ny, nx].
    With kirkland ([S, 12]) the paper's reciprocal-space route is used instead
    of the real-space Gaussian sum."""
    out = np.zeros((n_slices, ny, nx))
    for s in range(n_slices):
        sel = np.nonzero(slice_of == s)[0]
        if len(sel):
            if kirkland is not None:
                out[s] = kspace_potential(positions_f[sel, :2], atom_species[sel], kirkland,
                                          lx, ly, nx, ny)
            else:
                out[s] = projected_potential(positions_f[sel, :2], atom_species[sel], gauss_a,
                                             gauss_b, lx, ly, nx, ny)
    return out


# ---------------------------------------------------------------------------
# Multislice (Methods 2.2 Multislice Propagation; readings R-order, R-fft)
# ---------------------------------------------------------------------------
def transmission(v: np.ndarray, sigma: float) -> np.ndarray:
    """t(r) = exp(i sigma V(r))."""
    return np.exp(1j * sigma * v)


def propagator(nx: int, ny: int, dx: float, dy: float, lam: float, dz: float) -> np.ndarray:
    """P(k) = exp(-i pi lambda dz |k|^2) on the unshifted [ky, kx] grid."""
    kx = k_axis(nx, dx)
    ky = k_axis(ny, dy)
    k2 = ky[:, None] ** 2 + kx[None, :] ** 2
    return np.exp(-1j * math.pi * lam * dz * k2)


def multislice(psi0: np.ndarray, potentials: np.ndarray, sigma: float,
               prop: np.ndarray) -> np.ndarray:
    """Transmit then propagate through every slice; return the exit wave in
    reciprocal space (after the last propagator, without a final inverse FFT)."""
    psi = psi0.astype(np.complex128)
    n = potentials.shape[0]
    psik = None
    for s in range(n):
        psi = psi * transmission(potentials[s], sigma)
        psik = np.fft.fft2(psi, norm="ortho") * prop
        if s < n - 1:
            psi = np.fft.ifft2(psik, norm="ortho")
    if psik is None:       # no slices: the exit wave is the incident wave
        psik = np.fft.fft2(psi, norm="ortho")
    return psik


# ---------------------------------------------------------------------------
# Illumination (Supplement MWE: aperture=0 parallel beam, aperture=30 mrad probe; R-probe)
# ---------------------------------------------------------------------------
def plane_wave(nx: int, ny: int) -> np.ndarray:
    return np.full((ny, nx), 1.0 / math.sqrt(nx * ny), dtype=np.complex128)


# (n, m) of the polar aberration coefficients C_nm, orders 1..5 (reading R-aberr):
# defocus C10, two-fold astigmatism C12, coma C21, three-fold C23, spherical C30,
# star C32, four-fold C34, C41, C43, C45, fifth-order spherical C50, C52, C54, C56
ABERRATIONS = [(1, 0), (1, 2), (2, 1), (2, 3), (3, 0), (3, 2), (3, 4),
               (4, 1), (4, 3), (4, 5), (5, 0), (5, 2), (5, 4), (5, 6)]


def aberration_chi(kx: np.ndarray, ky: np.ndarray, lam: float, c_A, phi_rad) -> np.ndarray:
    """chi(k) [rad] on the [ky, kx] grid: (2 pi / lambda) sum C_nm alpha^(n+1)/(n+1)
    cos(m (phi - phi_nm)), alpha = lambda |k|, phi = atan2(ky, kx)."""
    kxx, kyy = np.meshgrid(kx, ky)
    alpha = lam * np.sqrt(kxx ** 2 + kyy ** 2)
    phi = np.arctan2(kyy, kxx)
    chi = np.zeros_like(alpha)
    for (n, m), c, a in zip(ABERRATIONS, c_A, phi_rad):
        chi += c * alpha ** (n + 1) / (n + 1) * np.cos(m * (phi - a))
    return 2.0 * math.pi / lam * chi


def probe_wave(nx: int, ny: int, dx: float, dy: float, lam: float, alpha_rad: float,
               rx: float, ry: float, aberrations=None) -> np.ndarray:
    """Hard-aperture probe centred at (rx, ry) on an nx*ny grid of pixel (dx, dy);
    aberrations: None or (C_nm [A], phi_nm [rad]), 14 each in ABERRATIONS order."""
    kx = k_axis(nx, dx)
    ky = k_axis(ny, dy)
    kk = np.sqrt(ky[:, None] ** 2 + kx[None, :] ** 2)
    aperture = (lam * kk <= alpha_rad).astype(np.float64)
    phase = np.exp(-2j * math.pi * (kx[None, :] * rx + ky[:, None] * ry))
    if aberrations is not None:
        phase = phase * np.exp(-1j * aberration_chi(kx, ky, lam, aberrations[0], aberrations[1]))
    psi = np.fft.ifft2(aperture * phase, norm="ortho")
    return psi / math.sqrt(np.sum(np.abs(psi) ** 2))


def window_origin(rx: float, ry: float, dx: float, dy: float, nx: int, ny: int):
    """Window origin pixel floor(r/d) - N/2 (not wrapped) for a probe at (rx, ry)."""
    ox = int(math.floor(rx / dx)) - nx // 2
    oy = int(math.floor(ry / dy)) - ny // 2
    return ox, oy


# ---------------------------------------------------------------------------
# Whole job: exit waves psi(k, t) for every probe and frame (Methods 2.1, WFData)
# ---------------------------------------------------------------------------
def job_geometry(job):
    lx, ly, lz = (float(v) for v in job.cell)
    pot_nx = job.pot_nx or job.nx
    pot_ny = job.pot_ny or job.ny
    return lx, ly, lz, pot_nx, pot_ny, lx / pot_nx, ly / pot_ny


def exit_waves(job, frames=None, probes=None) -> np.ndarray:
    """psi_exit(k) for the requested frames and probes: [P, F, ny, nx] complex128."""
    lx, ly, lz, pot_nx, pot_ny, dx, dy = job_geometry(job)
    lam = wavelength_A(job.voltage_V)
    sig = sigma_rad_per_VA(job.voltage_V)
    dz = lz / job.n_slices
    prop = propagator(job.nx, job.ny, dx, dy, lam, dz)
    instant = bool(getattr(job, "slice_by_instant_z", False))
    slice_of = slice_index(job.positions, lz, job.n_slices, instant)
    frames = range(job.n_frames) if frames is None else list(frames)
    plane = job.aperture_mrad == 0
    n_p = 1 if plane else job.probe_xy.shape[0]
    probes = range(n_p) if probes is None else list(probes)
    windowed = (pot_nx, pot_ny) != (job.nx, job.ny)
    aberr = getattr(job, "aberrations", None)
    out = np.zeros((len(probes), len(frames), job.ny, job.nx), dtype=np.complex128)
    for fi, f in enumerate(frames):
        slices_f = slice_of[f] if instant else slice_of
        pots = frame_potentials(job.positions[f], job.atom_species, slices_f, job.gauss_a,
                                job.gauss_b, lx, ly, pot_nx, pot_ny, job.n_slices,
                                getattr(job, "kirkland", None))
        for pi, p in enumerate(probes):
            if plane:
                psi0 = plane_wave(job.nx, job.ny)
                win = pots
            else:
                rx, ry = (float(v) for v in job.probe_xy[p])
                if windowed:
                    ox, oy = window_origin(rx, ry, dx, dy, job.nx, job.ny)
                    iy = (oy + np.arange(job.ny)) % pot_ny
                    ix = (ox + np.arange(job.nx)) % pot_nx
                    win = pots[:, iy][:, :, ix]
                    psi0 = probe_wave(job.nx, job.ny, dx, dy, lam, job.aperture_mrad * 1e-3,
                                      rx - ox * dx, ry - oy * dy, aberr)
                else:
                    win = pots
                    psi0 = probe_wave(job.nx, job.ny, dx, dy, lam, job.aperture_mrad * 1e-3,
                                      rx, ry, aberr)
            out[pi, fi] = multislice(psi0, win, sig, prop)
    return out


# ---------------------------------------------------------------------------
# TACAW time transform (Methods 2.1; reading R-time)
# ---------------------------------------------------------------------------
def tacaw_spectrum(exit_k: np.ndarray, two_sided: bool = False) -> np.ndarray:
    """I(k, w_m) = |(1/F) sum_f (psi_f - mean_f psi) exp(-2 pi i m f / F)|^2.

    exit_k: [P, F, ny, nx] complex; returns [P, M, ny, nx] float64 with M = F/2
    (one-sided) or F (two-sided).
    """
    n_f = exit_k.shape[1]
    mean = exit_k.mean(axis=1, keepdims=True)
    dpsi = exit_k - mean
    spec = np.fft.fft(dpsi, axis=1) / n_f
    inten = np.abs(spec) ** 2
    return inten if two_sided else inten[:, : n_f // 2]


def autocorrelation_spectrum(exit_k: np.ndarray, two_sided: bool = False) -> np.ndarray:
    """The same spectrum by the time-autocorrelation route that names the method:
    C(tau) = (1/F) sum_f conj(dpsi_f) dpsi_{(f+tau) mod F}, then
    I_m = (1/F) sum_tau C(tau) exp(-2 pi i m tau / F) (Wiener-Khinchin)."""
    n_f = exit_k.shape[1]
    dpsi = exit_k - exit_k.mean(axis=1, keepdims=True)
    corr = np.zeros_like(dpsi)
    for tau in range(n_f):
        corr[:, tau] = np.mean(np.conj(dpsi) * np.roll(dpsi, -tau, axis=1), axis=1)
    m = np.arange(n_f)
    kern = np.exp(-2j * math.pi * np.outer(m, m) / n_f)
    spec = np.tensordot(kern, corr, axes=([1], [1])) / n_f       # [M, P, ny, nx]
    spec = np.moveaxis(spec, 0, 1).real
    return spec if two_sided else spec[:, : n_f // 2]


def run_job(job, frames=None):
    """Exit waves and spectrum of a whole job (frames subset allowed)."""
    ex = exit_waves(job, frames=frames)
    return ex, tacaw_spectrum(ex, two_sided=job.two_sided)


# ---------------------------------------------------------------------------
# Analysis of the spectrum (Methods 2.1, "Data Structure Design": dispersion
# along k-space paths, momentum-resolved intensity at a frequency, position-
# resolved maps over a probe scan; Supplement MWE: dispersion(kx, ky),
# spectral_diffraction(15.0), spectrum_image(15.0)).  Readings: the frequency
# is the kept bin nearest to f (lowest index on ties); a k-space point is the
# nearest grid node (index round(k L) mod N, fftfreq order); probes are summed
# for dispersion and spectral diffraction; a spectrum image sums the k-nodes
# with k_inner <= |k| < k_outer (k_outer <= 0: no outer bound).
# ---------------------------------------------------------------------------
def frequency_bin(f_THz: float, n_frames: int, dt_fs: float, two_sided: bool = False) -> int:
    """Index of the kept frequency bin nearest to f_THz."""
    f = freq_axis_THz(n_frames, dt_fs, two_sided)
    return int(np.argmin(np.abs(f - f_THz)))


def spectral_diffraction(spec: np.ndarray, m: int) -> np.ndarray:
    """D[ky, kx] = sum over probes of I[p, m, ky, kx] (spec: [P, M, ny, nx])."""
    return spec[:, m].astype(np.float64).sum(axis=0)


def spectrum_image(spec: np.ndarray, m: int, kx: np.ndarray, ky: np.ndarray,
                   k_inner: float = 0.0, k_outer: float = 0.0) -> np.ndarray:
    """S[p] = sum of I[p, m, k] over the k-nodes with k_inner <= |k| < k_outer."""
    kk = np.sqrt(kx[None, :] ** 2 + ky[:, None] ** 2)
    mask = kk >= k_inner
    if k_outer > 0:
        mask &= kk < k_outer
    return np.array([spec[p, m].astype(np.float64)[mask].sum() for p in range(spec.shape[0])])


def dispersion(spec: np.ndarray, kx_path: np.ndarray, ky_path: np.ndarray, lx: float, ly: float) -> np.ndarray:
    """D[i, m] = sum over probes of I[p, m] at the grid node nearest (kx_i, ky_i)."""
    ny, nx = spec.shape[2], spec.shape[3]
    out = np.zeros((len(kx_path), spec.shape[1]))
    for i, (kx, ky) in enumerate(zip(kx_path, ky_path)):
        ix = int(np.floor(kx * lx + 0.5)) % nx
        iy = int(np.floor(ky * ly + 0.5)) % ny
        out[i] = spec[:, :, iy, ix].astype(np.float64).sum(axis=0)
    return out


# ---------------------------------------------------------------------------
# Conventional STEM from the same exit waves (Methods 2.1 HAADFData; "Beyond
# Vibrational Spectroscopy"; reading R-adf)
# ---------------------------------------------------------------------------
def mean_diffraction(exit_k: np.ndarray) -> np.ndarray:
    """D[p, ky, kx] = (1/F) sum_f |psi(p, f, k)|^2 (exit_k: [P, F, ny, nx])."""
    return (np.abs(exit_k.astype(np.complex128)) ** 2).mean(axis=1)


def adf(mean_diff: np.ndarray, kx: np.ndarray, ky: np.ndarray, lam: float,
        inner_mrad: float, outer_mrad: float) -> np.ndarray:
    """A[p] = sum of D[p, k] over the nodes with inner <= lambda |k| < outer (mrad)."""
    theta_mrad = 1e3 * lam * np.sqrt(kx[None, :] ** 2 + ky[:, None] ** 2)
    mask = (theta_mrad >= inner_mrad) & (theta_mrad < outer_mrad)
    return np.array([mean_diff[p][mask].sum() for p in range(mean_diff.shape[0])])


# ---------------------------------------------------------------------------
# Trajectory averaging (Methods 2.1 "Molecular Dynamics"; Supplement
# "Trajectory averaging"): the spectra of independent trajectories, or of
# consecutive segments of one trajectory, are averaged with equal weights.
# ---------------------------------------------------------------------------
def average_spectra(spectra) -> np.ndarray:
    """(1/J) sum_j I_j over spectra of one shape."""
    return np.mean(np.stack([np.asarray(s, dtype=np.float64) for s in spectra]), axis=0)


def segment_average_spectrum(exit_k: np.ndarray, n_segments: int, two_sided: bool = False) -> np.ndarray:
    """Average of the spectra of n_segments consecutive, equal, non-overlapping
    frame segments (each with its own mean subtraction and transform length)."""
    n_f = exit_k.shape[1]
    length = n_f // n_segments
    return average_spectra(tacaw_spectrum(exit_k[:, s * length:(s + 1) * length], two_sided)
                           for s in range(n_segments))
