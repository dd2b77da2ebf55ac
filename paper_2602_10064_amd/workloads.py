"""Seeded synthetic inputs for TACAW jobs.

This module only *synthesizes inputs*: lattices, harmonic-phonon trajectories,
species assignments, Gaussian form-factor coefficients and probe scan grids.
It holds none of the method's arithmetic (no potentials, no propagation, no
transforms), so both the HIP path and the FP64 oracle consume exactly the same
arrays from it.

The paper obtains trajectories from ORB-driven molecular dynamics (Methods,
"Molecular Dynamics"; Supplement, "Automated Molecular Dynamics
Equilibration"); its only requirement on a trajectory is a positions array of
shape (frames, atoms, 3), the species and the cell (Supplement, "Extensibility
to Other Atomistic Dynamics").  Those trajectories are not available, so a
seeded sum of commensurate plane-wave phonon modes stands in for them, with the
paper's shapes: hundreds of frames (Workflow Architecture), 0.1 A sampling, a
30 mrad probe and a 32x32 scan over 20 A (Supplement, Minimal Working Example).

Random draws use numpy's PCG64 (`default_rng`) in the fixed order documented
in each function, so a seed fully determines a job.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

HBAR_MEV_FS = 658.2119569  # hbar in meV*fs (CODATA 2018)


# --------------------------------------------------------------------------
# Job description (plain data, mirrors the C struct tacaw_job_desc)
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Job:
    cell: np.ndarray              # (3,) orthorhombic Lx, Ly, Lz [A]
    nx: int                       # wave grid (window grid when windowed)
    ny: int
    n_slices: int
    voltage_V: float
    aperture_mrad: float          # 0 -> plane wave
    dt_fs: float
    positions: np.ndarray         # (F, A, 3) float64 [A]
    atom_species: np.ndarray      # (A,) int32 index into species_Z
    species_Z: np.ndarray         # (S,) int32
    gauss_a: np.ndarray           # (S, 5) float64 [A]  electron form-factor amplitudes
    gauss_b: np.ndarray           # (S, 5) float64 [A^2]
    probe_xy: np.ndarray = dataclasses.field(
        default_factory=lambda: np.zeros((0, 2)))   # (P, 2) [A]
    pot_nx: int = 0               # full-cell potential grid when windowed (0 -> nx)
    pot_ny: int = 0
    two_sided: bool = False
    keep_exit_waves: bool = True
    # probe aberrations: None, or (2, 14) = (C_nm [A], phi_nm [rad]) for
    # (n, m) = 10, 12, 21, 23, 30, 32, 34, 41, 43, 45, 50, 52, 54, 56
    aberrations: Optional[np.ndarray] = None
    # bin atoms into slices by each frame's own z instead of the frame-mean z
    slice_by_instant_z: bool = False
    # the paper's reciprocal-space potential route: None, or (S, 12) per-species
    # coefficients (a1..a3 [1/A], b1..b3 [1/A^2], c1..c3 [A], d1..d3 [A^2]) of
    # f(q) = sum_i a_i / (q^2 + b_i) + c_i exp(-d_i q^2)
    kirkland: Optional[np.ndarray] = None
    name: str = ""

    @property
    def n_frames(self) -> int:
        return int(self.positions.shape[0])

    @property
    def n_atoms(self) -> int:
        return int(self.positions.shape[1])

    @property
    def n_probes(self) -> int:
        return 1 if self.aperture_mrad == 0 else int(self.probe_xy.shape[0])

    @property
    def windowed(self) -> bool:
        return self.pot_nx not in (0, self.nx) or self.pot_ny not in (0, self.ny)

    @property
    def n_bins(self) -> int:
        return self.n_frames if self.two_sided else self.n_frames // 2

    def slice_steps(self) -> int:
        return self.nx * self.ny * self.n_slices * self.n_frames * self.n_probes

    def replace(self, **kw) -> "Job":
        return dataclasses.replace(self, **kw)


# --------------------------------------------------------------------------
# Lattices
# --------------------------------------------------------------------------
_DIAMOND_BASIS = np.array([
    [0.00, 0.00, 0.00], [0.00, 0.50, 0.50], [0.50, 0.00, 0.50], [0.50, 0.50, 0.00],
    [0.25, 0.25, 0.25], [0.25, 0.75, 0.75], [0.75, 0.25, 0.75], [0.75, 0.75, 0.25],
])


def diamond_cubic(a: float, reps: Sequence[int], z_shift: float = 0.0):
    """Diamond-cubic supercell: returns (positions (A,3), cell (3,))."""
    rx, ry, rz = (int(r) for r in reps)
    cells = np.stack(np.meshgrid(np.arange(rx), np.arange(ry), np.arange(rz),
                                 indexing="ij"), axis=-1).reshape(-1, 3)
    pos = (cells[:, None, :] + _DIAMOND_BASIS[None, :, :]).reshape(-1, 3) * a
    pos[:, 2] += z_shift
    cell = np.array([rx * a, ry * a, rz * a], dtype=np.float64)
    return pos, cell


def hexagonal_layers(a: float, reps_xy: Sequence[int], n_layers: int,
                     layer_spacing: float, z_offset: float):
    """Honeycomb layers in the orthohexagonal cell (a, sqrt(3) a), 4 atoms per
    layer per rectangle (two per sublattice), AA' stacking (sublattices swap
    from one layer to the next).

    Returns (positions (A,3), sublattice (A,) in {0,1}, cell (3,)).
    """
    rx, ry = (int(r) for r in reps_xy)
    b = math.sqrt(3.0) * a
    d = a / math.sqrt(3.0)
    sub0 = np.array([[0.0, 0.0], [0.5 * a, 0.5 * b]])
    sub1 = sub0 + np.array([0.0, d])
    cells = np.stack(np.meshgrid(np.arange(rx), np.arange(ry), indexing="ij"),
                     axis=-1).reshape(-1, 2) * np.array([a, b])
    layer_xy = np.concatenate([(cells[:, None, :] + sub0[None]).reshape(-1, 2),
                               (cells[:, None, :] + sub1[None]).reshape(-1, 2)])
    layer_sub = np.concatenate([np.zeros(len(cells) * 2, np.int32),
                                np.ones(len(cells) * 2, np.int32)])
    pos, sub = [], []
    for k in range(n_layers):
        z = z_offset + k * layer_spacing
        pos.append(np.column_stack([layer_xy, np.full(len(layer_xy), z)]))
        sub.append(layer_sub if k % 2 == 0 else 1 - layer_sub)
    cell = np.array([rx * a, ry * b, n_layers * layer_spacing])
    return np.concatenate(pos), np.concatenate(sub).astype(np.int32), cell


def snap_to_slice_centres(lattice: np.ndarray, dz: float) -> np.ndarray:
    """Move every lattice plane to the centre of the slice it falls in, so no
    mean position sits on a slice boundary (where the binning rule would be
    decided by rounding)."""
    out = lattice.copy()
    out[:, 2] = (np.floor(out[:, 2] / dz) + 0.5) * dz
    return out


# --------------------------------------------------------------------------
# Harmonic-phonon trajectory
# --------------------------------------------------------------------------
def harmonic_trajectory(lattice: np.ndarray, cell: np.ndarray, reps: Sequence[int],
                        n_frames: int, dt_fs: float, rng: np.random.Generator,
                        n_modes: int = 32, hw_range_meV=(2.0, 60.0),
                        rms: float = 0.08, wrap_xy: bool = True) -> np.ndarray:
    """u_j(t) = sum_m A_m e_m cos(2 pi q_m . R_j - w_m t + phi_m).

    Draw order: integer wave-vector indices n_m (M,3) in [-R_a, R_a] per axis,
    then polarisations e_m (M,3) standard normal (normalised), then hbar*w_m
    ~ U[2,60] meV, then phases ~ U[0, 2 pi).  q_m = n_m / L keeps the supercell
    periodic.  A_m = 1 / w_m, then each Cartesian component is rescaled so its
    rms over (frames, atoms) is exactly `rms`.  x and y are wrapped into
    [0, L); z is not wrapped (the layers sit away from the z boundaries).
    """
    reps = np.asarray(reps, dtype=np.int64)
    n = np.stack([rng.integers(-reps[ax], reps[ax] + 1, size=n_modes) for ax in range(3)],
                 axis=1)
    e = rng.standard_normal((n_modes, 3))
    e /= np.linalg.norm(e, axis=1, keepdims=True)
    hw = rng.uniform(hw_range_meV[0], hw_range_meV[1], size=n_modes)
    phi = rng.uniform(0.0, 2.0 * math.pi, size=n_modes)
    omega = hw / HBAR_MEV_FS                       # rad / fs
    amp = 1.0 / omega
    q = n / cell[None, :]                          # cycles / A
    t = np.arange(n_frames, dtype=np.float64) * dt_fs
    spatial = 2.0 * math.pi * (lattice @ q.T) + phi[None, :]      # (A, M)
    # cos(s - w t) = cos(s) cos(w t) + sin(s) sin(w t): the mode sum becomes
    # two (F x M) @ (M x A) products per Cartesian component
    ct, st = np.cos(np.outer(t, omega)), np.sin(np.outer(t, omega))  # (F, M)
    cs, ss = np.cos(spatial).T, np.sin(spatial).T                    # (M, A)
    u = np.empty((n_frames, lattice.shape[0], 3), dtype=np.float64)
    for ax in range(3):
        wgt = (amp * e[:, ax])[:, None]
        u[:, :, ax] = ct @ (wgt * cs) + st @ (wgt * ss)
    scale = rms / np.sqrt(np.mean(u * u, axis=(0, 1)))
    u *= scale[None, None, :]
    x = lattice[None, :, :] + u
    if wrap_xy:
        x[:, :, 0] = np.mod(x[:, :, 0], cell[0])
        x[:, :, 1] = np.mod(x[:, :, 1], cell[1])
    return x


def gaussian_coefficients(seed: int, species_Z: Sequence[int]):
    """Per-species 5-term Gaussian electron form factors f(q) = sum a_i exp(-b_i q^2).

    For each Z: rng = default_rng([seed, Z]); a = U[0.1, 2] x5 (A), then
    b = U[0.1, 10] x5 (A^2).
    """
    a = np.zeros((len(species_Z), 5))
    b = np.zeros((len(species_Z), 5))
    for s, z in enumerate(species_Z):
        rng = np.random.default_rng([int(seed), int(z)])
        a[s] = rng.uniform(0.1, 2.0, size=5)
        b[s] = rng.uniform(0.1, 10.0, size=5)
    return a, b


def kirkland_coefficients(seed: int, species_Z: Sequence[int]) -> np.ndarray:
    """Per-species coefficients of the 3 Lorentzian + 3 Gaussian form factor
    f(q) = sum_i a_i / (q^2 + b_i) + c_i exp(-d_i q^2) (the tabulated values are
    not available; these stand in with magnitudes of the same order).

    For each Z: rng = default_rng([seed, Z, 3]); a = U[0.05, 1] x3 (1/A), then
    b = U[0.5, 50] x3 (1/A^2), then c = U[0.005, 0.2] x3 (A), then
    d = U[0.1, 4] x3 (A^2).  Returns (S, 12) in that order.
    """
    out = np.zeros((len(species_Z), 12))
    for s, z in enumerate(species_Z):
        rng = np.random.default_rng([int(seed), int(z), 3])
        out[s, 0:3] = rng.uniform(0.05, 1.0, size=3)
        out[s, 3:6] = rng.uniform(0.5, 50.0, size=3)
        out[s, 6:9] = rng.uniform(0.005, 0.2, size=3)
        out[s, 9:12] = rng.uniform(0.1, 4.0, size=3)
    return out


def with_kirkland(job: "Job", seed: int = 0) -> "Job":
    """The same job with the paper's reciprocal-space potential route (seeded
    coefficients per species of the job)."""
    return dataclasses.replace(job, kirkland=kirkland_coefficients(seed, job.species_Z),
                               name=f"{job.name}_kspace")


def probe_scan(x0: float, x1: float, nxp: int, y0: float, y1: float, nyp: int) -> np.ndarray:
    """Raster of probe positions (row-major over y then x), as linspace grids."""
    xs = np.linspace(x0, x1, nxp)
    ys = np.linspace(y0, y1, nyp)
    yy, xx = np.meshgrid(ys, xs, indexing="ij")
    return np.column_stack([xx.ravel(), yy.ravel()])


# --------------------------------------------------------------------------
# The five reference workloads and reduced variants of them
# --------------------------------------------------------------------------
def c1_tiny(n_frames: int = 64, seed: int = 1) -> Job:
    """2x2x2 diamond-cubic Si (64 atoms, Z=14), 64^2 grid, 8 slices, 200 kV
    plane wave, 64 frames at 5 fs."""
    a = 5.43
    n_slices = 8
    dz = 2 * a / n_slices
    lat, cell = diamond_cubic(a, (2, 2, 2), z_shift=dz / 2)
    rng = np.random.default_rng(seed)
    pos = harmonic_trajectory(lat, cell, (2, 2, 2), n_frames, 5.0, rng)
    species_Z = np.array([14], np.int32)
    ga, gb = gaussian_coefficients(seed, species_Z)
    return Job(cell=cell, nx=64, ny=64, n_slices=n_slices, voltage_V=200e3,
               aperture_mrad=0.0, dt_fs=5.0, positions=pos,
               atom_species=np.zeros(len(lat), np.int32), species_Z=species_Z,
               gauss_a=ga, gauss_b=gb, name="c1_tiny")


def c2_plain(n_frames: int = 1024, seed: int = 2, grid: int = 512, n_slices: int = 32,
             reps=(12, 12, 8)) -> Job:
    """12x12x8 diamond-cubic C/Si (9216 atoms, exact 50/50 Z=6/14), 512^2 grid,
    32 slices, 100 kV plane wave, 1024 frames at 2 fs."""
    a = 5.43
    lz = reps[2] * a
    dz = lz / n_slices
    lat, cell = diamond_cubic(a, reps, z_shift=dz / 2)
    rng = np.random.default_rng(seed)
    species_Z = np.array([6, 14], np.int32)
    n_atoms = len(lat)
    sp = np.zeros(n_atoms, np.int32)
    sp[n_atoms // 2:] = 1
    sp = rng.permutation(sp).astype(np.int32)
    pos = harmonic_trajectory(lat, cell, reps, n_frames, 2.0, rng)
    ga, gb = gaussian_coefficients(seed, species_Z)
    return Job(cell=cell, nx=grid, ny=grid, n_slices=n_slices, voltage_V=100e3,
               aperture_mrad=0.0, dt_fs=2.0, positions=pos, atom_species=sp,
               species_Z=species_Z, gauss_a=ga, gauss_b=gb, name="c2_plain")


def c3_probe(n_frames: int = 256, seed: int = 3, n_scan: int = 32, reps_xy=(40, 20),
             n_cells_z: int = 6, win: int = 256, pot_grid=(1000, 866), n_slices: int = 20,
             scan_extent: float = 20.0, dt_fs: float = 10.0) -> Job:
    """Hexagonal B/N layer stack (a=2.5 A, 40x20 orthohexagonal rectangles, 6 cells
    of 2 AA' layers 3.33 A apart), 20 slices, 30 mrad probe at 60 kV, 256^2 windows
    cropped from a 1000x866 full-cell potential grid, a 32x32 scan over 20 A and
    256 frames."""
    spacing = 3.33
    n_layers = 2 * n_cells_z
    lat, sub, cell = hexagonal_layers(2.5, reps_xy, n_layers, spacing, 0.5 * spacing)
    rng = np.random.default_rng(seed)
    pos = harmonic_trajectory(lat, cell, (reps_xy[0], reps_xy[1], n_cells_z),
                              n_frames, dt_fs, rng)
    species_Z = np.array([5, 7], np.int32)
    ga, gb = gaussian_coefficients(seed, species_Z)
    probes = probe_scan(0.0, scan_extent, n_scan, 0.0, scan_extent, n_scan)
    return Job(cell=cell, nx=win, ny=win, n_slices=n_slices, voltage_V=60e3,
               aperture_mrad=30.0, dt_fs=dt_fs, positions=pos, atom_species=sub,
               species_Z=species_Z, gauss_a=ga, gauss_b=gb, probe_xy=probes,
               pot_nx=pot_grid[0], pot_ny=pot_grid[1], name="c3_probe")


def smooth235(lo: int, hi: int) -> List[int]:
    out = []
    for v in range(lo, hi + 1):
        w = v
        for p in (2, 3, 5):
            while w % p == 0:
                w //= p
        if w == 1:
            out.append(v)
    return out


def c4_job(j: int, seed_base: int = 4000, grids=(128, 256, 384, 512),
           frames_range=(128, 1024), big: bool = False) -> Job:
    """One job of the uneven mix: grid from {128,256,384,512}^2, 8-48 slices,
    a 2*3*5-smooth frame count in [128,1024], 1-3 species with Z in [3,40],
    diamond-cubic or hexagonal layers with a in [2.5,5.5] A, 60/100/200 kV,
    2/5/10 fs, plane wave (p=1/2) or one 30 mrad probe at the cell centre.

    Draw order: grid, slices, frames, number of species, the Z values,
    lattice kind, a, voltage, dt, illumination; then the trajectory draws.
    `big` turns the job into a 1024^2-grid, 2048-frame job with the rest
    drawn the same way.
    """
    rng = np.random.default_rng(seed_base + j)
    grid = int(rng.choice(grids))
    n_slices = int(rng.integers(8, 49))
    frames = int(rng.choice(smooth235(*frames_range)))
    n_sp = int(rng.integers(1, 4))
    zs = rng.choice(np.arange(3, 41), size=n_sp, replace=False).astype(np.int32)
    kind = int(rng.integers(0, 2))
    a = float(rng.uniform(2.5, 5.5))
    volt = float(rng.choice([60e3, 100e3, 200e3]))
    dt = float(rng.choice([2.0, 5.0, 10.0]))
    probe = bool(rng.uniform() < 0.5)
    if big:
        grid, frames = 1024, 2048
    target_dx = float(rng.uniform(0.10, 0.15))
    if kind == 0:
        reps_xy = max(1, int(round(grid * target_dx / a)))
        thickness_target = n_slices * float(rng.uniform(1.0, 2.5))
        rz = max(1, int(round(thickness_target / a)))
        dz = rz * a / n_slices
        lat, cell = diamond_cubic(a, (reps_xy, reps_xy, rz), z_shift=dz / 2)
        lat = snap_to_slice_centres(lat, cell[2] / n_slices)
        reps = (reps_xy, reps_xy, rz)
    else:
        b = math.sqrt(3.0) * a
        rx = max(1, int(round(grid * target_dx / a)))
        ry = max(1, int(round(grid * target_dx / b)))
        spacing = 3.33
        n_layers = max(1, int(round(n_slices * float(rng.uniform(1.0, 2.5)) / spacing)))
        lat, _, cell = hexagonal_layers(a, (rx, ry), n_layers, spacing, 0.5 * spacing)
        lat = snap_to_slice_centres(lat, cell[2] / n_slices)
        reps = (rx, ry, max(1, n_layers // 2))
    sp = rng.integers(0, n_sp, size=len(lat)).astype(np.int32)
    pos = harmonic_trajectory(lat, cell, reps, frames, dt, rng)
    ga, gb = gaussian_coefficients(seed_base + j, zs)
    probes = np.array([[cell[0] / 2, cell[1] / 2]]) if probe else np.zeros((0, 2))
    return Job(cell=cell, nx=grid, ny=grid, n_slices=n_slices, voltage_V=volt,
               aperture_mrad=30.0 if probe else 0.0, dt_fs=dt, positions=pos,
               atom_species=sp, species_Z=zs, gauss_a=ga, gauss_b=gb, probe_xy=probes,
               name=f"c4_job{j}")


def c5_arrivals(n: int, rate_per_s: float = 4.0, seed: int = 5):
    """Poisson arrival times (s) and job kinds (True = the 1024^2 x 2048-frame
    kind, 10%) for the serving workload."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=n)
    big = rng.uniform(size=n) < 0.10
    return np.cumsum(gaps), big


def random_small_job(seed: int, nx: int = 16, ny: int = 16, n_slices: int = 3,
                     n_frames: int = 8, n_atoms: int = 6, aperture_mrad: float = 0.0,
                     n_probes: int = 1, cell=(6.0, 6.0, 4.0), voltage_V: float = 100e3,
                     n_species: int = 2, pot_grid: Optional[Sequence[int]] = None,
                     two_sided: bool = False) -> Job:
    """Small random job (uniform random atoms, random displacements) for
    property tests and brute-force checks."""
    rng = np.random.default_rng(seed)
    cell = np.asarray(cell, dtype=np.float64)
    base = rng.uniform(0, 1, size=(n_atoms, 3)) * cell
    n_sl = n_slices
    dz = cell[2] / n_sl
    base[:, 2] = (rng.integers(0, n_sl, size=n_atoms) + 0.5) * dz
    disp = 0.05 * rng.standard_normal((n_frames, n_atoms, 3))
    pos = base[None] + disp
    pos[:, :, 0] = np.mod(pos[:, :, 0], cell[0])
    pos[:, :, 1] = np.mod(pos[:, :, 1], cell[1])
    zs = np.arange(6, 6 + n_species, dtype=np.int32)
    sp = rng.integers(0, n_species, size=n_atoms).astype(np.int32)
    ga, gb = gaussian_coefficients(seed, zs)
    probes = rng.uniform(0, 1, size=(n_probes, 2)) * cell[:2] if aperture_mrad > 0 \
        else np.zeros((0, 2))
    pnx, pny = (pot_grid if pot_grid is not None else (0, 0))
    return Job(cell=cell, nx=nx, ny=ny, n_slices=n_sl, voltage_V=voltage_V,
               aperture_mrad=aperture_mrad, dt_fs=5.0, positions=pos, atom_species=sp,
               species_Z=zs, gauss_a=ga, gauss_b=gb, probe_xy=probes, pot_nx=pnx,
               pot_ny=pny, two_sided=two_sided, name=f"random{seed}")


def frame_segments(job: Job, n_segments: int) -> List[Job]:
    """Consecutive, equal, non-overlapping frame segments of a job's trajectory,
    one job each (frames beyond n_segments * (F // n_segments) are dropped)."""
    length = job.n_frames // n_segments
    if length < 2:
        raise ValueError("segments need at least two frames")
    return [dataclasses.replace(job, positions=job.positions[s * length:(s + 1) * length].copy(),
                                name=f"{job.name}_seg{s}")
            for s in range(n_segments)]
