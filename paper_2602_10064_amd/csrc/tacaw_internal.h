// Internal declarations shared by the host runtime and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tacaw {

// Atom position of one frame, in pixel units of the potential grid: the
// integer pixel (ix, iy) and the sub-pixel offset (fx, fy) in [0, 1).  The
// split keeps FP32 distances exact to ~1e-7 pixel on any grid size.
struct AtomPos {
  int32_t ix, iy;
  float fx, fy;
};

constexpr int N_GAUSS = 5;
constexpr int SPLAT_TX = 32;   // splat tile: columns
constexpr int SPLAT_TY = 32;   // splat tile: rows
constexpr int COEF_STRIDE = 6; // per (species, term): amplitude, exp2 x, exp2 y, cutoff x, cutoff y,
                               // log2 of the amplitude
constexpr int SPLAT_MAX_SPECIES = 16;  // species whose coefficients are staged in LDS
constexpr int COL_CT = 16;     // columns per column-pass workgroup (128-byte rows)

// Projected potentials of a batch of frames.
struct SplatArgs {
  const AtomPos* pos;          // [F][A], atoms sorted by slice
  const int32_t* species;      // [A] species index, sorted order
  const int32_t* tile_start;   // [n_slices * tiles + 1] CSR offsets
  const int32_t* tile_atoms;   // candidate pairs: sorted-atom index * 8 + Gaussian term
  const float* coef;           // [S][5][COEF_STRIDE]: amplitude (V A), exp2 factor per pixel^2
                               // along x and y, truncation radius in pixels along x and y
  float* V;                    // [fb][n][pny][pnx]: slices slice0 .. slice0+n-1, n = the lane's
                               // n_slices_launch
  int n_atoms, n_species, f0, fb, n_slices, slice0, pnx, pny, tiles_x, tiles_y;
  float rcx, rcy;              // truncation radius in pixels along x and y
  int img_x, img_y;            // periodic images -img..img searched per axis
  const int16_t* fslice;       // [F][A] each frame's own slice (sorted order), or nullptr:
                               // a pair adds nothing in frames where its atom is elsewhere
};

// One row or column pass over a batch of (probe, frame) waves.
struct PassArgs {
  float2* exit;                // [P][F][ny][nx] exit store, also the in-flight waves
  const float* V;              // [fb][v_slices][pny][pnx]: slices v_slice0 .. v_slice0+v_slices-1
  const float2* probe0;        // [P][ny][nx] incident probes (real space)
  const int32_t* origin;       // [P][2] window origin on the potential grid
  const float2* tw_x;          // [nx] exp(-2 pi i m / nx)
  const float2* tw_y;          // [ny]
  const float2* px;            // [nx] propagator factor along kx (scaled)
  const float2* py;            // [ny]
  int nx, ny, pnx, pny, n_frames, f0, fb, n_probes, n_slices, slice;
  int v_slices, v_slice0;      // slices per frame held in V and the first of them
  float sigma;                 // interaction parameter [rad / (V A)]
  float plane_amp;             // 1 / sqrt(nx ny)
  int plane;                   // 1: plane-wave incident wave
  float* vout;                 // inverse-only row pass of the reciprocal-space potentials: when set,
                               // wave w's real part goes to plane 2w of vout and its imaginary part to
                               // plane 2w + 1 ([2 W][ny][nx] float) instead of back into exit
};

// The paper's reciprocal-space potential route for one batch of frames and a
// group of slices taken in pairs (2q, 2q + 1): W = V(k) of slice 2q + i V(k)
// of slice 2q + 1, V(k) = sum over the slice's atoms of f_Z(|k|) exp(-2 pi i
// k.r_j) at the potential grid's frequencies, with f the 3 Lorentzian + 3
// Gaussian form factor times C/A.  Both slices' potentials are real, so one
// unnormalised inverse 2D FFT of W gives them as its real and imaginary parts.
// The kernel computes the rows ky index 0 .. pny/2 and writes the others as
// W(-k) = conj V_2q(k) + i conj V_2q+1(k).  W is then the Hermitian part of
// the literal sum, so the transform gives the real part of the literal
// potential: a Nyquist frequency of an even side takes cos(pi n x) (the mean
// of its +k and -k terms), and the corner where both are Nyquist takes
// cos(a + b) = cos a cos b - sin a sin b.
struct KPotArgs {
  const AtomPos* pos;          // [F][A], atoms in slice-sorted order
  const int32_t* ks_start;     // [n_slices * n_species + 1]: CSR offsets per (slice, species)
  const int32_t* ks_atoms;     // sorted-atom indices, by (slice, species)
  const int16_t* fslice;       // [F][A] each frame's own slice (sorted order), or nullptr
  const float* kcoef;          // [S][12]: a1..a3 (times C/A), b1..b3, c1..c3 (times C/A),
                               // d1..d3 (times log2 e)
  float2* W;                   // [fb][npairs][pny][pnx]
  int n_atoms, n_species, f0, fb, n_slices, slice0, npairs, pnx, pny;
  int row_tiles, col_tiles;    // tiles over rows 0 .. pny/2 and over the columns
  float kx_unit, ky_unit;      // 1/Lx, 1/Ly [1/A]
};
constexpr int KP_TY = 32;      // reciprocal-space potential tile: rows
constexpr int KP_TX = 128;     // columns (four wavefronts of 32)
constexpr int KP_K = 16;       // atoms per LDS stage
constexpr int KP_NCOEF = 12;

struct TimeArgs {
  const float2* exit;          // [P][F][n_k]
  float* spec;                 // [P][M][n_k]
  const float2* tw;            // [F] exp(-2 pi i m / F)
  int n_k, n_frames, n_bins, n_probes, kt;
  float inv_f2;                // 1 / F^2
};

constexpr int MAX_LANES = 8;
struct PassLane {
  PassArgs a;
  int mode;          // RowMode or ColMode
  int block_start;   // set by the launcher
};
struct PassTable {
  int n;
  PassLane l[MAX_LANES];
};
struct SplatLane {
  SplatArgs a;
  int n_slices_launch;  // slices slice0 .. slice0 + n - 1 of frames f0 .. f0 + fb - 1
  int block_start;      // set by the launcher
  int fpw;              // frames per wavefront, set by the launcher
};
struct SplatTable {
  int n;
  SplatLane l[MAX_LANES];
};

// A batch of waves carried through a run of slices with each wave resident
// in one workgroup's LDS (square grids of 64 and 128): one lane is one frame
// batch of one job and the slices a.slice .. a.slice + n_slices_launch - 1,
// whose potentials V holds (a.v_slice0, a.v_slices).  The last slice of the
// job ends in reciprocal space with the last-slice propagator.
struct ResLane {
  PassArgs a;
  const float2* px_last;
  const float2* py_last;
  int n_slices_launch;
  int block_start;   // set by the launcher
};
struct ResTable {
  int n;
  ResLane l[MAX_LANES];
};

enum RowMode { ROW_FIRST = 0, ROW_REGULAR = 1, ROW_INVERSE_ONLY = 2 };
enum ColMode { COL_REGULAR = 0, COL_LAST = 1, COL_INVERSE_ONLY = 2 };

// Events the next main-kernel launch on this thread records itself (start
// and end of the kernel); cleared by that launch.
void set_launch_events(hipEvent_t start, hipEvent_t stop);

// Kernel launchers (kernels.hip).  Each returns hipSuccess or the launch error.
bool grid_supported(int n);
hipError_t launch_splat(const SplatArgs& a, int n_slices_launch, hipStream_t s);
hipError_t launch_row_pass(const PassArgs& a, int mode, hipStream_t s);
hipError_t launch_row_lanes(const PassLane* lanes, int n, int variant, hipStream_t s);
hipError_t launch_col_lanes(const PassLane* lanes, int n, int variant, hipStream_t s);
hipError_t launch_splat_lanes(const SplatLane* lanes, int n, hipStream_t s);
hipError_t launch_col_pass(const PassArgs& a, int mode, hipStream_t s);
hipError_t launch_time_stage(const TimeArgs& a, hipStream_t s);
hipError_t launch_kpot(const KPotArgs& a, hipStream_t s);
bool resident_supported(int nx, int ny);
hipError_t kernels_init();   // per-kernel attributes on the current device
hipError_t launch_res_lanes(const ResLane* lanes, int n, hipStream_t s);
int time_stage_kt(int n_frames, int n_k);

// Setup kernels: twiddle table exp(-2 pi i m / n) (FP64 -> FP32); separable
// propagator factors exp(-i pi lambda dz k^2) * scale along one axis; probe
// aperture fill in reciprocal space.
hipError_t launch_twiddles(float2* tw, int n, hipStream_t s);
hipError_t launch_prop_factor(float2* out, int n, double d, double lam, double dz, double scale,
                              hipStream_t s);
hipError_t launch_aperture_count(int* count, int nx, int ny, double dx, double dy, double lam,
                                 double alpha, hipStream_t s);
// Probe aberrations: polar coefficients C_nm [A] and angles phi_nm [rad] for
// (n, m) = 10, 12, 21, 23, 30, 32, 34, 41, 43, 45, 50, 52, 54, 56; the probe
// factor is exp(-i chi(k)), chi = (2 pi / lambda) sum C_nm alpha^(n+1) / (n+1)
// cos(m (phi - phi_nm)), alpha = lambda |k|.
constexpr int N_ABERR = 14;
struct Aberrations {
  double c[N_ABERR];
  double phi[N_ABERR];
  int on;
};
hipError_t launch_probe_fill(float2* out, const double* rloc /*[P][2]*/, const int* count, int n_probes,
                             int nx, int ny, double dx, double dy, double lam, double alpha,
                             const Aberrations& ab, hipStream_t s);

// Spectrum analysis reductions (FP64 sums of I[p][m][k]).
hipError_t launch_spectral_diffraction(const float* spec, double* out, int n_probes, int n_bins, int n_k, int m,
                                       hipStream_t s);
hipError_t launch_spectrum_image(const float* spec, double* out, int n_probes, int n_bins, int nx, int ny, int m,
                                 const double* kx, const double* ky, double k_in2, double k_out2, hipStream_t s);
hipError_t launch_dispersion(const float* spec, double* out, int n_probes, int n_bins, int n_k, const int* node,
                             int n_points, hipStream_t s);

// Conventional STEM from kept exit waves: D[p][k] = (1/F) sum_f |psi[p][f][k]|^2
// in FP64; A[p] = sum of D[p][k] over inner <= 1e3 lambda |k| < outer (mrad).
// Trajectory averaging: out[i] = (1/J) sum_j specs[j][i] (FP64 sums in order).
hipError_t launch_average_spectra(const float* const* specs /*device array of J*/, int n_jobs, float* out,
                                  size_t n, hipStream_t s);
hipError_t launch_mean_diffraction(const float2* exit, double* out, int n_probes, int n_frames, int n_k,
                                   hipStream_t s);
hipError_t launch_adf(const double* diff, double* out, int n_probes, int nx, int ny, const double* kx,
                      const double* ky, double lam, double inner_mrad, double outer_mrad, hipStream_t s);

}  // namespace tacaw
