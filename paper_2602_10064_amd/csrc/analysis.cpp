// Conventional STEM from the kept exit waves (Methods 2.1 HAADFData; "Beyond
// Vibrational Spectroscopy"): frame-averaged diffraction patterns and ADF
// detector sums over an annulus of scattering angles.
//
// Spectrum analysis on the device: spectral diffraction at a frequency,
// spectrum images over a probe scan, dispersion along a k-space path (Methods
// 2.1, "Data Structure Design": dispersion along reciprocal-space paths,
// momentum-resolved intensity at a frequency, position-resolved vibrational
// maps; Supplement MWE: dispersion(kx, ky), spectral_diffraction(15.0),
// spectrum_image(15.0)).  Each call reduces the job's resident spectrum
// I[p][m][ky][kx] with one kernel in FP64 and copies the result out.
#include <math.h>

#include <algorithm>
#include <vector>

#include "runtime.h"

using namespace tacaw;

namespace {

#define A_TRY(call)                                                         \
  do {                                                                      \
    hipError_t e_ = (call);                                                 \
    if (e_ != hipSuccess) {                                                 \
      set_error("%s failed: %s", #call, hipGetErrorString(e_));             \
      return TACAW_EDEVICE;                                                 \
    }                                                                       \
  } while (0)

}  // namespace

namespace tacaw {

// the job must hold a spectrum
tacaw_status check_ready(const tacaw_job* job) {
  if (!job) {
    set_error("job is NULL");
    return TACAW_EINVAL;
  }
  const int ss = job->serve_state.load();
  if (ss == 1 || ss == 2) {
    set_error("job is still in the serving loop");
    return TACAW_EBUSY;
  }
  if (ss == 4) {
    set_error("job was cancelled");
    return TACAW_ECANCELLED;
  }
  if (!job->has_result || !job->d_spec) {
    set_error("job has not been run");
    return TACAW_ENOTREADY;
  }
  return TACAW_OK;
}

// f_m = m / (F dt) for the kept bins: one-sided m < F/2, two-sided fftfreq order
double bin_freq(const tacaw_job* job, int m) {
  const int F = job->hp.F;
  const double dt_ps = job->desc.dt_fs * 1e-3;
  const int mm = (job->desc.flags & TACAW_TWO_SIDED) && m >= (F + 1) / 2 ? m - F : m;
  return mm / (F * dt_ps);
}

// kept bin nearest to f (lowest index on ties); EINVAL beyond half a bin
// outside the kept range
tacaw_status nearest_bin(const tacaw_job* job, double f, int* m_out) {
  const int M = job->hp.M;
  int best = 0;
  double dbest = fabs(bin_freq(job, 0) - f), fmin = bin_freq(job, 0), fmax = fmin;
  for (int m = 1; m < M; ++m) {
    const double fm = bin_freq(job, m);
    fmin = std::min(fmin, fm);
    fmax = std::max(fmax, fm);
    if (fabs(fm - f) < dbest) {
      dbest = fabs(fm - f);
      best = m;
    }
  }
  const double half = 0.5 / (job->hp.F * job->desc.dt_fs * 1e-3);
  if (!(f >= fmin - half && f <= fmax + half)) {
    set_error("frequency %g THz outside the kept bins [%g, %g] THz", f, fmin, fmax);
    return TACAW_EINVAL;
  }
  *m_out = best;
  return TACAW_OK;
}

}  // namespace tacaw

namespace {

// device scratch of the analysis calls, freed on return
struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

tacaw_status finish_copy(tacaw_job* job, hipStream_t s, double* dst, const double* src, size_t n, int on_device) {
  if (on_device) {
    A_TRY(hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    A_TRY(hipStreamSynchronize(s));
  } else {
    A_TRY(hipStreamSynchronize(s));
    A_TRY(hipMemcpy(dst, src, n * sizeof(double), hipMemcpyDeviceToHost));
  }
  (void)job;
  return TACAW_OK;
}

}  // namespace

namespace tacaw {

// unshifted axes kx then ky, k = fftfreq(N, d): i * (1 / (N d)), i wrapped to
// negative values from (N + 1) / 2 on
std::vector<double> k_axes(const HostPlan& hp) {
  std::vector<double> ax(hp.nx + hp.ny);
  const double fx = 1.0 / (hp.nx * hp.dx), fy = 1.0 / (hp.ny * hp.dy);
  for (int i = 0; i < hp.nx; ++i) ax[i] = (i < (hp.nx + 1) / 2 ? i : i - hp.nx) * fx;
  for (int i = 0; i < hp.ny; ++i) ax[hp.nx + i] = (i < (hp.ny + 1) / 2 ? i : i - hp.ny) * fy;
  return ax;
}

}  // namespace tacaw

namespace {

// the job must hold its exit waves
tacaw_status check_exit(const tacaw_job* job) {
  tacaw_status st = check_ready(job);
  if (st != TACAW_OK) return st;
  if (!(job->desc.flags & TACAW_KEEP_EXIT_WAVES) || !job->d_exit) {
    set_error("job was created without TACAW_KEEP_EXIT_WAVES");
    return TACAW_EINVAL;
  }
  return TACAW_OK;
}

// frame-averaged diffraction patterns into a fresh device buffer
tacaw_status mean_diffraction_dev(tacaw_job* job, hipStream_t s, DevBuf& out) {
  const HostPlan& hp = job->hp;
  A_TRY(hipMalloc(&out.p, (size_t)hp.P * hp.nx * hp.ny * sizeof(double)));
  A_TRY(launch_mean_diffraction(job->d_exit, (double*)out.p, hp.P, hp.F, hp.nx * hp.ny, s));
  return TACAW_OK;
}

}  // namespace

extern "C" {

tacaw_status tacaw_average_spectra(tacaw_job* const* jobs, int32_t n_jobs, float* dst, size_t n,
                                   int dst_on_device) {
  clear_error();
  if (!jobs || n_jobs < 1 || !dst) {
    set_error("need n_jobs >= 1 jobs and a destination");
    return TACAW_EINVAL;
  }
  std::vector<const float*> specs(n_jobs);
  const tacaw_job* j0 = jobs[0];
  for (int i = 0; i < n_jobs; ++i) {
    tacaw_status st = check_ready(jobs[i]);
    if (st != TACAW_OK) return st;
    const HostPlan &a = j0->hp, &b = jobs[i]->hp;
    if (a.P != b.P || a.M != b.M || a.nx != b.nx || a.ny != b.ny || jobs[i]->ctx->device != j0->ctx->device) {
      set_error("job %d's spectrum shape or device differs from job 0's", i);
      return TACAW_EINVAL;
    }
    specs[i] = jobs[i]->d_spec;
  }
  const HostPlan& hp = j0->hp;
  if (n != (size_t)hp.P * hp.M * hp.nx * hp.ny) {
    set_error("dst must hold n_probes * bins * ny * nx = %zu values", (size_t)hp.P * hp.M * hp.nx * hp.ny);
    return TACAW_EINVAL;
  }
  A_TRY(hipSetDevice(j0->ctx->device));
  // every job's last run must be complete before its spectrum is read
  for (int i = 0; i < n_jobs; ++i) A_TRY(hipStreamSynchronize(jobs[i]->last_stream));
  hipStream_t s = j0->last_stream;
  DevBuf ptrs, out;
  A_TRY(hipMalloc(&ptrs.p, n_jobs * sizeof(const float*)));
  A_TRY(hipMemcpy(ptrs.p, specs.data(), n_jobs * sizeof(const float*), hipMemcpyHostToDevice));
  float* o = dst;
  if (!dst_on_device) {
    A_TRY(hipMalloc(&out.p, n * sizeof(float)));
    o = (float*)out.p;
  }
  A_TRY(launch_average_spectra((const float* const*)ptrs.p, n_jobs, o, n, s));
  A_TRY(hipStreamSynchronize(s));
  if (!dst_on_device) A_TRY(hipMemcpy(dst, o, n * sizeof(float), hipMemcpyDeviceToHost));
  return TACAW_OK;
}

tacaw_status tacaw_mean_diffraction(tacaw_job* job, double* dst, size_t n, int dst_on_device) {
  clear_error();
  tacaw_status st = check_exit(job);
  if (st != TACAW_OK) return st;
  const HostPlan& hp = job->hp;
  if (!dst || n != (size_t)hp.P * hp.nx * hp.ny) {
    set_error("dst must hold n_probes * ny * nx = %zu values", (size_t)hp.P * hp.nx * hp.ny);
    return TACAW_EINVAL;
  }
  A_TRY(hipSetDevice(job->ctx->device));
  hipStream_t s = job->last_stream;
  DevBuf d;
  if ((st = mean_diffraction_dev(job, s, d)) != TACAW_OK) return st;
  return finish_copy(job, s, dst, (const double*)d.p, n, dst_on_device);
}

tacaw_status tacaw_adf(tacaw_job* job, double inner_mrad, double outer_mrad, double* dst, size_t n,
                       int dst_on_device) {
  clear_error();
  tacaw_status st = check_exit(job);
  if (st != TACAW_OK) return st;
  const HostPlan& hp = job->hp;
  if (!dst || n != (size_t)hp.P) {
    set_error("dst must hold one value per probe (%d)", hp.P);
    return TACAW_EINVAL;
  }
  if (!(inner_mrad >= 0.0) || !(outer_mrad > inner_mrad)) {
    set_error("need 0 <= inner_mrad < outer_mrad");
    return TACAW_EINVAL;
  }
  const std::vector<double> ax = k_axes(hp);
  A_TRY(hipSetDevice(job->ctx->device));
  hipStream_t s = job->last_stream;
  DevBuf d, out, axes;
  if ((st = mean_diffraction_dev(job, s, d)) != TACAW_OK) return st;
  A_TRY(hipMalloc(&out.p, n * sizeof(double)));
  A_TRY(hipMalloc(&axes.p, ax.size() * sizeof(double)));
  A_TRY(hipMemcpyAsync(axes.p, ax.data(), ax.size() * sizeof(double), hipMemcpyHostToDevice, s));
  const double* kx = (const double*)axes.p;
  A_TRY(launch_adf((const double*)d.p, (double*)out.p, hp.P, hp.nx, hp.ny, kx, kx + hp.nx, hp.lam, inner_mrad,
                   outer_mrad, s));
  return finish_copy(job, s, dst, (const double*)out.p, n, dst_on_device);
}

tacaw_status tacaw_spectral_diffraction(tacaw_job* job, double f_THz, double* dst, size_t n, int dst_on_device) {
  clear_error();
  tacaw_status st = check_ready(job);
  if (st != TACAW_OK) return st;
  if (!dst || n != (size_t)job->hp.nx * job->hp.ny) {
    set_error("dst must hold ny * nx = %d values", job->hp.nx * job->hp.ny);
    return TACAW_EINVAL;
  }
  int m = 0;
  if ((st = nearest_bin(job, f_THz, &m)) != TACAW_OK) return st;
  A_TRY(hipSetDevice(job->ctx->device));
  hipStream_t s = job->last_stream;
  DevBuf out;
  A_TRY(hipMalloc(&out.p, n * sizeof(double)));
  A_TRY(launch_spectral_diffraction(job->d_spec, (double*)out.p, job->hp.P, job->hp.M, (int)n, m, s));
  return finish_copy(job, s, dst, (const double*)out.p, n, dst_on_device);
}

tacaw_status tacaw_spectrum_image(tacaw_job* job, double f_THz, double k_inner, double k_outer, double* dst,
                                  size_t n, int dst_on_device) {
  clear_error();
  tacaw_status st = check_ready(job);
  if (st != TACAW_OK) return st;
  if (!dst || n != (size_t)job->hp.P) {
    set_error("dst must hold one value per probe (%d)", job->hp.P);
    return TACAW_EINVAL;
  }
  if (!(k_inner >= 0.0) || !(k_outer <= 0.0 || k_outer > k_inner)) {
    set_error("need 0 <= k_inner and (k_outer <= 0 or k_outer > k_inner)");
    return TACAW_EINVAL;
  }
  int m = 0;
  if ((st = nearest_bin(job, f_THz, &m)) != TACAW_OK) return st;
  const HostPlan& hp = job->hp;
  const std::vector<double> ax = k_axes(hp);
  A_TRY(hipSetDevice(job->ctx->device));
  hipStream_t s = job->last_stream;
  DevBuf out, axes;
  A_TRY(hipMalloc(&out.p, n * sizeof(double)));
  A_TRY(hipMalloc(&axes.p, ax.size() * sizeof(double)));
  A_TRY(hipMemcpyAsync(axes.p, ax.data(), ax.size() * sizeof(double), hipMemcpyHostToDevice, s));
  const double* kx = (const double*)axes.p;
  A_TRY(launch_spectrum_image(job->d_spec, (double*)out.p, hp.P, hp.M, hp.nx, hp.ny, m, kx, kx + hp.nx,
                              k_inner * k_inner, k_outer > 0.0 ? k_outer * k_outer : 0.0, s));
  return finish_copy(job, s, dst, (const double*)out.p, n, dst_on_device);
}

tacaw_status tacaw_dispersion(tacaw_job* job, const double* kx, const double* ky, int32_t n_points, double* dst,
                              size_t n, int dst_on_device) {
  clear_error();
  tacaw_status st = check_ready(job);
  if (st != TACAW_OK) return st;
  const HostPlan& hp = job->hp;
  if (!kx || !ky || n_points < 1 || (long long)n_points * hp.M > (1LL << 30) || !dst ||
      n != (size_t)n_points * hp.M) {
    set_error("need 1 <= n_points, n_points * M <= 2^30 and dst of n_points * M = %lld values",
              (long long)n_points * hp.M);
    return TACAW_EINVAL;
  }
  // nearest grid node: index round(k L) mod N, L = N d the extent of the wave
  // grid (the window's when the probe sees a window of the potential grid)
  const double wx = hp.nx * hp.dx, wy = hp.ny * hp.dy;
  std::vector<int> node(n_points);
  for (int i = 0; i < n_points; ++i) {
    if (!isfinite(kx[i]) || !isfinite(ky[i])) {
      set_error("path point %d is not finite", i);
      return TACAW_EINVAL;
    }
    long ix = (long)floor(kx[i] * wx + 0.5) % hp.nx;
    long iy = (long)floor(ky[i] * wy + 0.5) % hp.ny;
    if (ix < 0) ix += hp.nx;
    if (iy < 0) iy += hp.ny;
    node[i] = (int)(iy * hp.nx + ix);
  }
  A_TRY(hipSetDevice(job->ctx->device));
  hipStream_t s = job->last_stream;
  DevBuf out, nodes;
  A_TRY(hipMalloc(&out.p, n * sizeof(double)));
  A_TRY(hipMalloc(&nodes.p, node.size() * sizeof(int)));
  A_TRY(hipMemcpyAsync(nodes.p, node.data(), node.size() * sizeof(int), hipMemcpyHostToDevice, s));
  A_TRY(launch_dispersion(job->d_spec, (double*)out.p, hp.P, hp.M, hp.nx * hp.ny, (const int*)nodes.p, n_points, s));
  return finish_copy(job, s, dst, (const double*)out.p, n, dst_on_device);
}

}  // extern "C"
