/*
 * tacaw.h - C ABI of libtacaw, the MI355X (gfx950) TACAW hot path.
 *
 * The library computes, for a trajectory of atomic positions, the exit waves
 * of a frame-resolved multislice simulation and the TACAW spectrum
 *     I(k, w) = | F_t[ psi(k, t) - <psi(k, t)>_t ] |^2
 * (PySlice, arXiv 2602.10064: Methods 2.1 "Workflow Architecture" for the
 * time transform; Methods 2.2 "Multislice Propagation" and "Atomic Scattering
 * Potentials" for the scattering; Supplement "Extensibility to Other Atomistic
 * Dynamics" for the inputs: positions (frames, atoms, 3), species and cell;
 * Supplement "Minimal Working Example" for the calculator parameters:
 * aperture, beam energy, sampling, slice thickness and probe positions).
 *
 * Conventions shared by every call:
 *   - Lengths in Angstrom, beam energy in volts, frame spacing in fs,
 *     frequencies in THz, spatial frequencies in cycles/Angstrom.
 *   - Arrays are C-contiguous (row-major).  Reciprocal-space arrays are
 *     unshifted (DC at index 0, numpy fftfreq order) with kx fastest:
 *     [ky][kx].
 *   - All pointers are host pointers unless the argument says a device
 *     pointer may be given.  Inputs are copied; the caller keeps ownership
 *     of everything it passes in.
 *   - Every call returns a tacaw_status.  No C++ exception crosses the ABI.
 *     On failure tacaw_last_error() returns a message for the calling thread.
 *   - A job is used by one caller thread at a time.
 */
#ifndef TACAW_H
#define TACAW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TACAW_OK = 0,
  TACAW_EINVAL = 1,        /* an argument is out of range or inconsistent          */
  TACAW_ENOMEM = 2,        /* the job can never fit the context's memory budget   */
  TACAW_EDEVICE = 3,       /* a HIP runtime call failed                            */
  TACAW_EBUSY = 4,         /* the job is queued or running in the serving loop     */
  TACAW_ENOTREADY = 5,     /* no result yet (the job has not been run)             */
  TACAW_ECANCELLED = 6,    /* the job was cancelled before it finished             */
  TACAW_EUNSUPPORTED = 7   /* valid, but a grid size the library has no kernel for */
} tacaw_status;

/* Number of Gaussian terms per species in the form factor. */
#define TACAW_N_GAUSS 5

/* tacaw_job_desc.flags */
#define TACAW_TWO_SIDED 1u        /* keep all F frequency bins instead of F/2      */
#define TACAW_KEEP_EXIT_WAVES 2u  /* keep psi(k, t) readable after the time stage  */
#define TACAW_DEFER_ALLOC 4u      /* allocate device memory only when the job is run
                                     or admitted by the serving loop                 */
#define TACAW_USE_GRAPH 8u        /* tacaw_run captures the job's whole launch
                                     sequence into a HIP graph once and replays it   */
#define TACAW_SLICE_BY_INSTANT_Z 16u /* bin atoms into slices by each frame's own z
                                     (Methods 2.2: atoms within the slice z-bounds,
                                     taken frame by frame) instead of the FP64
                                     frame-mean z; n_slices < 32768               */

typedef struct tacaw_ctx tacaw_ctx;
typedef struct tacaw_job tacaw_job;

/*
 * Problem statement of one job.
 *
 * Potential (Methods 2.2, "Atomic Scattering Potentials", with the tabulated
 * Kirkland form replaced by a Gaussian form factor):  species s has the
 * electron form factor f_s(q) = C sum_i gauss_a[s][i] exp(-gauss_b[s][i] q^2),
 * q in cycles/A, a in A, b in A^2, C = 2 pi a0 e = 47.8776 V A^2.  Its
 * projected potential v_s(r) = C sum_i a_i (pi/b_i) exp(-pi^2 r^2 / b_i) (V A)
 * is point-sampled at grid nodes r_p = (p_x Lx/Nx, p_y Ly/Ny) and summed over
 * the atoms of a slice and their periodic images.  The library evaluates each
 * Gaussian term of an atom exactly on the 32 x 32 tiles of the potential grid
 * that its box of half-width r_i = sqrt(b_i ln 1e8)/pi (the radius where the
 * term has fallen to 1e-8 of its peak), widened by the atom's largest
 * displacement from its mean position, reaches; other tiles get nothing from
 * that term.
 *
 * Slices (Methods 2.2, "atoms within the slice z-bounds"): atom j belongs to
 * slice floor((zbar_j mod Lz)/dz), clamped to [0, n_slices), where zbar_j is
 * its FP64 mean z over all frames and dz = Lz / n_slices.
 *
 * Multislice (Methods 2.2, "Multislice Propagation"): in every slice the wave
 * is multiplied by t = exp(i sigma V) and then propagated by
 * P(k) = exp(-i pi lambda dz |k|^2) in reciprocal space (relativistic lambda
 * and sigma = 2 pi gamma m0 e lambda / h^2).  The exit wave is the
 * reciprocal-space wave after the last propagator, with unitary (ortho) FFTs.
 *
 * Illumination (Supplement, Minimal Working Example: aperture=0 is a parallel
 * beam, aperture=30 a 30 mrad convergent probe at probe_xs/probe_ys):
 * aperture_mrad == 0 -> plane wave 1/sqrt(Nx Ny) (probe_xy ignored, one wave
 * per frame).  aperture_mrad > 0 -> for each probe position an aberration-free
 * hard-aperture probe: A(k) = 1 where lambda |k| <= alpha, times
 * exp(-2 pi i k.r_p), inverse-transformed and normalised to unit norm.
 *
 * Windows: pot_nx/pot_ny == 0 (or equal to nx/ny) -> the wave grid covers the
 * cell.  Otherwise the potential is built on the full-cell pot_nx x pot_ny
 * grid and every probe propagates on an nx x ny window of it (same pixel
 * size), cropped with periodic wrap at origin floor(r_p / d) - N/2.
 *
 * Time transform (Methods 2.1): per (probe, k), the FP64 mean over all frames
 * is subtracted and I_m = |(1/F) sum_f dpsi_f exp(-2 pi i m f / F)|^2 is
 * returned for m = 0..F/2-1 (or all F with TACAW_TWO_SIDED).  Frequencies
 * f_m = m / (F dt) (Supplement, "Sampling Considerations").
 */
typedef struct {
  double cell[3];              /* orthorhombic Lx, Ly, Lz [A], all > 0                  */
  int32_t nx, ny;              /* wave grid; each a product of 2, 3, 5 (EINVAL otherwise);
                                  EUNSUPPORTED for sizes without compiled FFT plans:
                                  16 32 48 64 96 128 160 192 256 320 384 512 640 768 1024 */
  int32_t n_slices;            /* >= 1                                                   */
  double voltage_V;            /* beam energy [V], > 0                                   */
  double aperture_mrad;        /* 0 -> plane wave; > 0 -> probe semi-angle [mrad]        */
  int32_t n_probes;            /* probe count (>= 1 when aperture_mrad > 0)              */
  const double* probe_xy;      /* n_probes x 2 probe positions [A] (host)                */
  int32_t pot_nx, pot_ny;      /* full-cell potential grid for windows, or 0             */
  double dt_fs;                /* frame spacing [fs], > 0                                */
  int32_t n_frames;            /* >= 2, a product of 2, 3, 5                             */
  int32_t n_atoms;             /* >= 0                                                   */
  int32_t n_species;           /* >= 1                                                   */
  const int32_t* species_Z;    /* n_species atomic numbers (labels only)                 */
  const double* gauss_a;       /* n_species x 5 form-factor amplitudes [A], > 0
                                  (ignored, may be NULL, with kspace_coef)               */
  const double* gauss_b;       /* n_species x 5 form-factor widths [A^2], > 0 (ditto)    */
  uint32_t flags;              /* TACAW_TWO_SIDED, TACAW_KEEP_EXIT_WAVES, TACAW_DEFER_ALLOC,
                                  TACAW_USE_GRAPH                                        */
  const double* kspace_coef;   /* NULL, or n_species x 12 coefficients of the paper's own
                                  potential route (see below)                            */
} tacaw_job_desc;

/*
 * Reciprocal-space potential route (Methods 2.2, "Atomic Scattering
 * Potentials", the paper's own construction), chosen by a non-NULL
 * kspace_coef: species s has the form factor
 *   f_s(q) = sum_{i<3} a_i / (q^2 + b_i) + c_i exp(-d_i q^2)
 * with kspace_coef[s] = {a1, a2, a3, b1, b2, b3, c1, c2, c3, d1, d2, d3}
 * (q in cycles/A; a in 1/A, b in 1/A^2 with b > 0, c in A, d in A^2 with
 * d >= 0; all finite; EINVAL otherwise).  Each slice's potential is
 *   V(r) = (C / A) sum_k V(k) exp(2 pi i k.r),  V(k) = sum_j f_{Z_j}(|k|)
 *   exp(-2 pi i k.r_j)
 * over the atoms of the slice, with k the potential grid's own frequencies
 * (one period: the potential is band-limited), C = 2 pi a0 e and A = Lx Ly.
 * A side of even length has an unpaired Nyquist frequency; its term is taken as the
 * mean of its +k and -k images, which is the real part of the sum.  The
 * potential grid (pot_nx x pot_ny, or nx x ny) must be one of the compiled
 * FFT sizes (EUNSUPPORTED otherwise).  The gauss_a / gauss_b form is not
 * used.
 */

/* ---- context ------------------------------------------------------------ */

/* Create a context on HIP device `device`.  hbm_budget_bytes caps the device
 * memory that jobs of this context may hold at once (0 -> 90% of the device's
 * free memory at creation).  The context owns the serving thread and the
 * tuning state.  Errors: EINVAL (bad device), EDEVICE. */
tacaw_status tacaw_ctx_create(int device, size_t hbm_budget_bytes, tacaw_ctx** out);

/* Destroy a context.  Jobs still queued in its serving loop are cancelled and
 * waited for; jobs themselves must still be destroyed by the caller, before
 * or after. */
tacaw_status tacaw_ctx_destroy(tacaw_ctx* ctx);

/* ---- jobs ---------------------------------------------------------------- */

/* Device bytes a job with this description holds while resident (positions,
 * potentials, exit waves, spectrum, tables).  Validates the description. */
tacaw_status tacaw_job_footprint(const tacaw_job_desc* desc, size_t* bytes);

/* Create a job: validate, bin atoms into slices, encode positions, allocate
 * the job's device buffers and upload its inputs.  atom_species: n_atoms
 * indices into species_Z (host).  positions: n_frames x n_atoms x 3 [A]
 * (host, float64).  Errors: EINVAL (invalid description or species index),
 * ENOMEM (footprint above the context budget), EUNSUPPORTED (grid size
 * without a kernel in the library), EDEVICE. */
tacaw_status tacaw_job_create(tacaw_ctx* ctx, const tacaw_job_desc* desc,
                              const int32_t* atom_species, const double* positions,
                              tacaw_job** out);

/* ---- probe aberrations ------------------------------------------------------
 * ("Beyond Vibrational Spectroscopy": the standard aberration function with
 * defocus, astigmatism, coma, spherical aberration and higher orders, applied
 * at probe formation.)  The incident probe in reciprocal space becomes
 * A(k) exp(-i chi(k)) exp(-2 pi i k.r_p), with
 *   chi(k) = (2 pi / lambda) sum_nm C_nm alpha^(n+1) / (n+1) cos(m (phi - phi_nm)),
 * alpha = lambda |k|, phi = atan2(ky, kx), over the TACAW_N_ABERRATIONS polar
 * coefficients in this order of (n, m): 10 (defocus; C10 = z is a Fresnel
 * propagation of the focused probe over z), 12 (two-fold astigmatism), 21
 * (coma), 23, 30 (spherical, Cs), 32, 34, 41, 43, 45, 50 (C5), 52, 54, 56.
 * c_angstrom: TACAW_N_ABERRATIONS magnitudes in A (host; NULL clears every
 * aberration); phi_rad: as many angles in rad (host; NULL means all 0; ignored
 * for m = 0).  The values are copied.  Takes effect from the next run (a job
 * that already holds its incident probes rebuilds them at once, synchronously).
 * EINVAL for a plane-wave job or a non-finite value; EBUSY while the job is in
 * the serving loop. */
#define TACAW_N_ABERRATIONS 14
tacaw_status tacaw_job_set_aberrations(tacaw_job* job, const double* c_angstrom, const double* phi_rad);

/* Plain per-job form: enqueue the whole hot path (potentials, multislice over
 * every (probe, frame) wave, exit-wave capture, FP64 frame mean, time FFT and
 * |.|^2) on `hip_stream` (a hipStream_t, or NULL for the default stream) and
 * return without waiting.  May be called again to recompute.  EBUSY while the
 * job is in the serving loop. */
tacaw_status tacaw_run(tacaw_job* job, void* hip_stream);

/* Batched form for uneven jobs (several grids, slice and frame counts): run
 * n_jobs jobs of one context together, ordered on `hip_stream`.  Jobs whose
 * frame batches fill the device on their own (at least 64 MiB of waves,
 * $TACAW_BATCH_LARGE_MB) run one after another on one of the context's
 * streams.  The smaller jobs with the same grid share launches: each launch
 * advances up to 8 frame batches of different jobs by one pass, each at its
 * own slice, and a finished frame batch is replaced by the next one at once;
 * groups of different grid sizes run on the context's other streams.  All
 * streams are joined back to `hip_stream`.  Every result equals the job's
 * tacaw_run result bit for bit. */
tacaw_status tacaw_run_batch(tacaw_job* const* jobs, int n_jobs, void* hip_stream);

/* Captured batch (the benchmark spec's graph-captured frame loops for uneven
 * jobs): the whole batched launch sequence of a fixed set of jobs, exactly as
 * tacaw_run_batch enqueues it, recorded once as one HIP graph and replayed on
 * any stream, so a repeated batch costs one graph launch instead of thousands
 * of kernel launches.  Capture materialises every job first (allocation and
 * uploads stay outside the graph) and records nothing while context timing is
 * on.  The graph holds the jobs' device addresses: the jobs must outlive the
 * batch, and a launch after a job's buffers were reallocated (a serving-loop
 * submission, for one) is refused with EINVAL.  Results after a launch are
 * bitwise those of tacaw_run.  Errors as tacaw_run_batch. */
typedef struct tacaw_batch tacaw_batch;
tacaw_status tacaw_batch_capture(tacaw_job* const* jobs, int32_t n_jobs, tacaw_batch** out);
tacaw_status tacaw_batch_launch(tacaw_batch* batch, void* hip_stream);
tacaw_status tacaw_batch_destroy(tacaw_batch* batch);

/* Autotuner: time the row-pass variants (rows per workgroup, and for grids
 * of 64 to 1024 register-resident kernels with one or two rows in flight; at
 * 384 also the six-step row kernel, 384 = 6 x 64) and
 * the column-pass variants (tile widths, and for 64 to 1024 rows
 * register-resident kernels on 8- to 32-column tiles; at 512 rows also
 * 16-column tiles and the six-step kernels 512 = 8 x 64 with lanes along x
 * on 8- and 16-column tiles, at 256 rows the six-step kernel 256 = 8 x 32 on
 * 16-column tiles, at 384 rows the six-step kernel 384 = 6 x 64) on one
 * frame batch of `job` and keep the faster of each for the job's grid size
 * in the context (appended to the JSON-lines file named by
 * $TACAW_TUNE_CACHE, read back by later contexts).  Writes the chosen
 * variants (row 0-4, column 0-3 or 5-8) when the pointers are not NULL.
 * Resets the context's timing totals. */
tacaw_status tacaw_autotune(tacaw_job* job, void* hip_stream, int* row_variant, int* col_variant);

/* Serving form: hand the job to the context's continuous-batching loop.
 * The loop admits it once its footprint fits the budget next to the jobs
 * already resident and interleaves its slice steps with theirs.  Jobs whose
 * frame batches are small (under TACAW_BATCH_LARGE_MB MiB of waves) share
 * launches with the other running jobs of their grid size: one launch
 * advances one frame batch of each by one slice.  Larger jobs run on their
 * own stream, one frame batch in flight, overlapping the others.  The result
 * is bitwise the one the job gets alone.  TACAW_SERVE_BATCH_WINDOW_MS (default
 * 0) holds a new grid size's first shared launch that long after its first
 * request is ready, so that requests arriving together start together. */
tacaw_status tacaw_submit(tacaw_ctx* ctx, tacaw_job* job);

/* *done = 1 once a submitted job has its spectrum (or was cancelled). */
tacaw_status tacaw_poll(tacaw_job* job, int* done);

/* Block until a submitted job finishes.  ECANCELLED if it was cancelled. */
tacaw_status tacaw_wait(tacaw_job* job);

/* Cancel a submitted job.  Jobs not yet admitted are dropped; a running job
 * stops at its next frame batch.  Other jobs are unaffected. */
tacaw_status tacaw_cancel(tacaw_job* job);

/* Latency of a job that finished in the serving loop: time from submit to
 * admission (queued_ms) and from submit to the spectrum being ready on the
 * device (total_ms), in milliseconds.  ENOTREADY before it finishes. */
tacaw_status tacaw_job_latency(const tacaw_job* job, double* queued_ms, double* total_ms);

/* Counters of the context's serving loop since the context was created:
 * pass launches (row, column, or LDS-resident multislice) that served more
 * than one job (*shared_launches), and served jobs that shared at least one
 * such launch with another job (*grouped_jobs).  Either pointer may be
 * NULL. */
tacaw_status tacaw_serve_stats(tacaw_ctx* ctx, int64_t* shared_launches, int64_t* grouped_jobs);

/* Copy the spectrum I[p][m][ky][kx] (float32, n = n_probes * M * ny * nx,
 * M = F/2 or F) into dst, a host pointer or (dst_on_device != 0) a device
 * pointer.  Waits for the job's work first.  ENOTREADY before a run. */
tacaw_status tacaw_get_spectrum(tacaw_job* job, float* dst, size_t n, int dst_on_device);

/* Copy the exit waves psi[p][f][ky][kx] (complex64 as interleaved float re,im;
 * n = n_probes * F * ny * nx complex values) into dst (host or device).
 * Needs TACAW_KEEP_EXIT_WAVES. */
tacaw_status tacaw_get_exit_waves(tacaw_job* job, void* dst_c64, size_t n, int dst_on_device);

/* Output axes: kx[nx], ky[ny] in cycles/A (fftfreq order, spacing 1/(N d)),
 * f_THz[M] (m / (F dt), fftfreq order when two-sided).  Any pointer may be
 * NULL. */
tacaw_status tacaw_axes(const tacaw_job_desc* desc, double* kx, double* ky, double* f_THz);

/* ---- frame ranges, checkpoints, trajectory averaging ----------------------
 * (Methods 2.1 "Workflow Architecture": exit waves are kept per frame so that
 * an interrupted simulation restarts without recomputing finished frames, and
 * analyses run on stored waves; Methods 2.1 "Molecular Dynamics" and the
 * Supplement's "Trajectory averaging": spectra of independent trajectories or
 * of trajectory segments are averaged to reduce noise.)
 *
 * tacaw_run_frames computes the exit waves of frames [f_begin, f_end) into
 * the job's exit store, asynchronously on hip_stream, exactly as tacaw_run
 * computes them (per-frame arithmetic does not depend on the range), and
 * leaves the spectrum alone.  tacaw_finish runs the time stage once every
 * frame's exit waves are in the store (from tacaw_run_frames or
 * tacaw_put_exit_frames; ENOTREADY otherwise) and makes the spectrum ready.
 * Ranges must be non-empty within [0, n_frames) (EINVAL); EBUSY while the job
 * is in the serving loop.  A job created without TACAW_KEEP_EXIT_WAVES keeps
 * its store between these calls in the plain form too. */
tacaw_status tacaw_run_frames(tacaw_job* job, int32_t f_begin, int32_t f_end, void* hip_stream);
tacaw_status tacaw_finish(tacaw_job* job, void* hip_stream);

/* Copy frames [f_begin, f_end) of the exit store out (get) or in (put), laid
 * out [P][f_end - f_begin][ny][nx] complex64 (n = P * frames * ny * nx), for
 * checkpoints.  Synchronous; host or (on_device != 0) device memory.  get
 * needs frames that hold exit waves (ENOTREADY otherwise); put marks the
 * frames as present, so a restarted job computes only the others. */
tacaw_status tacaw_get_exit_frames(tacaw_job* job, int32_t f_begin, int32_t f_end, void* dst, size_t n,
                                   int dst_on_device);
tacaw_status tacaw_put_exit_frames(tacaw_job* job, int32_t f_begin, int32_t f_end, const void* src, size_t n,
                                   int src_on_device);

/* dst = (1/J) sum_j I_j over n_jobs jobs with spectra of one shape (P, bins,
 * ny, nx) on one device (EINVAL otherwise), summed in FP64 in job order and
 * rounded to float32; n = P * bins * ny * nx; host or (dst_on_device != 0)
 * device destination.  Waits for every job's last run.  Averaging the
 * segments of one trajectory is the same call over one job per segment. */
tacaw_status tacaw_average_spectra(tacaw_job* const* jobs, int32_t n_jobs, float* dst, size_t n,
                                   int dst_on_device);

/* ---- spectrum analysis ----------------------------------------------------
 * Reductions of the job's resident spectrum I[p][m][ky][kx] (Methods 2.1,
 * "Data Structure Design": dispersion along reciprocal-space paths,
 * momentum-resolved intensity at a frequency, position-resolved maps over a
 * probe scan; Supplement MWE: dispersion(kx, ky), spectral_diffraction(15.0),
 * spectrum_image(15.0)).  The frequency f_THz selects the kept bin nearest to
 * it (lowest index on ties; EINVAL more than half a bin outside the kept
 * range).  Sums run on the device in FP64 in a fixed order; results are
 * float64, copied to a host pointer or (dst_on_device != 0) a device pointer.
 * ENOTREADY before a run, EBUSY while serving, ECANCELLED after a cancel. */

/* D[ky][kx] = sum over probes of I[p][m][ky][kx]; n = ny * nx. */
tacaw_status tacaw_spectral_diffraction(tacaw_job* job, double f_THz, double* dst, size_t n, int dst_on_device);

/* S[p] = sum of I[p][m][k] over the k-nodes with k_inner <= |k| < k_outer
 * (cycles/A; k_outer <= 0: no outer bound), one value per probe position in
 * probe_xy order (a virtual detector); n = n_probes. */
tacaw_status tacaw_spectrum_image(tacaw_job* job, double f_THz, double k_inner, double k_outer, double* dst,
                                  size_t n, int dst_on_device);

/* Allocation-free variant of tacaw_spectrum_image, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): same arguments, same result, same kernel.
 * The per-probe sums and the k-axis tables sit in one fixed device array of
 * the library (544 KiB per GPU, held until the process ends) instead of
 * buffers allocated per call; the call allocates and frees nothing.
 * Limits: n_probes <= 65536 and nx + ny <= 4096, else EINVAL (use
 * tacaw_spectrum_image).  Every call on one GPU shares that GPU's array:
 * calls that overlap in time on one GPU (from several threads, or while an
 * earlier call's copy is still in flight) race and must be serialised by the
 * caller.  Each call writes every value it reads, so no clearing is needed. */
tacaw_status tacaw_spectrum_image_noalloc(tacaw_job* job, double f_THz, double k_inner, double k_outer,
                                          double* dst, size_t n, int dst_on_device);

/* D[i][m] = sum over probes of I[p][m] at the grid node nearest to the path
 * point (kx[i], ky[i]) (cycles/A; node index round(k L) mod N with L = N d
 * the wave grid's extent, fftfreq order), for every kept bin m; kx, ky are host arrays of n_points;
 * n = n_points * M. */
tacaw_status tacaw_dispersion(tacaw_job* job, const double* kx, const double* ky, int32_t n_points, double* dst,
                              size_t n, int dst_on_device);

/* ---- conventional STEM from the same exit waves ----------------------------
 * ("Beyond Vibrational Spectroscopy": ADF/HAADF images integrate the scattered
 * intensity over a range of collection angles, from the stored exit waves;
 * Methods 2.1: HAADFData over the x, y, kx, ky dataset.)  Both calls need a
 * job created with TACAW_KEEP_EXIT_WAVES (EINVAL otherwise) that has run;
 * ENOTREADY / EBUSY / ECANCELLED as for the spectrum analysis.  Results are
 * float64, computed in FP64 on the device, copied to a host pointer or
 * (dst_on_device != 0) a device pointer. */

/* D[p][ky][kx] = (1/F) sum_f |psi[p][f][ky][kx]|^2: the frame-averaged
 * (frozen-phonon) diffraction pattern of every probe, the 4D-STEM dataset;
 * n = n_probes * ny * nx. */
tacaw_status tacaw_mean_diffraction(tacaw_job* job, double* dst, size_t n, int dst_on_device);

/* A[p] = sum of D[p][k] over the k-nodes with inner_mrad <= 1e3 lambda |k| <
 * outer_mrad (small-angle scattering angle; 0 <= inner < outer, else EINVAL),
 * one value per probe in probe_xy order: an annular detector image (HAADF for
 * inner angles of 50-80 mrad, bright field from 0); n = n_probes. */
tacaw_status tacaw_adf(tacaw_job* job, double inner_mrad, double outer_mrad, double* dst, size_t n,
                       int dst_on_device);

/* ---- job inspection and teardown -------------------------------------------- */

/* Slice index of every atom (n_atoms int32, host) from the FP64 frame-mean z,
 * as the planner binned it.  With TACAW_SLICE_BY_INSTANT_Z this binning only
 * orders the atoms; the potentials use each frame's own slice. */
tacaw_status tacaw_job_slices(const tacaw_job* job, int32_t* slice_of_atom, size_t n);

/* The planner's launch shapes for a job: frames advanced together through
 * the slices (every row or column pass launch covers one such batch and one
 * slice), and slices per potential launch.  NULL outputs are skipped. */
tacaw_status tacaw_job_plan(const tacaw_job* job, int32_t* frame_batch, int32_t* slices_per_potential_launch);

/* Release a job's device memory.  EBUSY while it is in the serving loop. */
tacaw_status tacaw_job_destroy(tacaw_job* job);

/* Message of the last failed call on this thread ("" if none). */
const char* tacaw_last_error(void);

/* ---- measurement ---------------------------------------------------------- */

/* Kernel classes timed by the library when timing is on. */
typedef enum {
  TACAW_K_SPLAT = 0,      /* projected potentials (real-space sum, or the
                             structure factors of the reciprocal-space route) */
  TACAW_K_ROW = 1,        /* row pass: iFFT_x, transmission, FFT_x     */
  TACAW_K_COL = 2,        /* column pass: FFT_y, propagator, iFFT_y    */
  TACAW_K_TIME = 3,       /* FP64 mean, time FFT, |.|^2                */
  TACAW_K_OTHER = 4,      /* tables, incident probes, and the inverse FFT
                             of the reciprocal-space potentials           */
  TACAW_K_COUNT = 5
} tacaw_kernel_class;

/* Turn per-kernel HIP-event timing on (1) or off (0) for jobs of this
 * context; turning it on clears the accumulated figures.  A timed launch
 * records a start and an end event itself, on the stream the kernel runs on
 * (hipExtLaunchKernel), for the launches tacaw_timing_select picks. */
tacaw_status tacaw_timing_enable(tacaw_ctx* ctx, int on);

/* Select what timing measures: the kernel classes (bit c of class_mask for
 * class c; default all) and one launch in `every` of each selected class
 * (default 1: every launch; the first launch of a class after this call is
 * timed).  Other launches run without events and are not counted.  EINVAL if
 * every < 1. */
tacaw_status tacaw_timing_select(tacaw_ctx* ctx, unsigned class_mask, int every);

/* Accumulated kernel time (ms) and launch count of one class since timing
 * was enabled; synchronises the recorded events first. */
tacaw_status tacaw_timing_get(tacaw_ctx* ctx, int kernel_class, double* total_ms,
                              int64_t* launches);

/* Library version string. */
const char* tacaw_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TACAW_H */
