// Host planner: validation, constants, slice binning, position encoding,
// splat candidate lists, probe windows and device footprint (FP64 on the host).
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <numeric>
#include <thread>

#include "runtime.h"

namespace tacaw {

// CODATA 2018 (SI)
static const double kH = 6.62607015e-34;
static const double kMe = 9.1093837015e-31;
static const double kQe = 1.602176634e-19;
static const double kC = 299792458.0;
static const double kBohrA = 0.529177210903;        // A
static const double kCoulombEVA = 14.399645478425668;  // e^2 / (4 pi eps0) in eV A

static thread_local char g_err[1024];

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}
void clear_error() { g_err[0] = 0; }
const char* last_error_text() { return g_err; }

// Relativistic wavelength lambda = h / sqrt(2 m0 e E (1 + e E / (2 m0 c^2))), in A
// (Methods 2.2, Multislice Propagation: "m_e includes relativistic corrections").
double wavelength_A(double volt) {
  const double ej = kQe * volt;
  const double p = sqrt(2.0 * kMe * ej * (1.0 + ej / (2.0 * kMe * kC * kC)));
  return kH / p * 1e10;
}

// sigma = 2 pi gamma m0 e lambda / h^2 in rad / (V A).  The paper prints the
// interaction parameter without the electron charge; it is restored here.
double sigma_rad_per_VA(double volt) {
  const double gamma = 1.0 + kQe * volt / (kMe * kC * kC);
  const double lam = wavelength_A(volt) * 1e-10;
  return 2.0 * M_PI * gamma * kMe * kQe * lam / (kH * kH) * 1e-10;
}

static bool smooth235(int n) {
  if (n < 1) return false;
  for (int p : {2, 3, 5})
    while (n % p == 0) n /= p;
  return n == 1;
}

tacaw_status validate_desc(const tacaw_job_desc* d) {
  if (!d) {
    set_error("job description is NULL");
    return TACAW_EINVAL;
  }
  for (int i = 0; i < 3; ++i)
    if (!(d->cell[i] > 0.0) || !isfinite(d->cell[i])) {
      set_error("cell[%d] must be a positive finite length (got %g)", i, d->cell[i]);
      return TACAW_EINVAL;
    }
  if (d->nx <= 0 || d->ny <= 0 || !smooth235(d->nx) || !smooth235(d->ny)) {
    set_error("grid %dx%d: each side must be a positive product of 2, 3 and 5", d->nx, d->ny);
    return TACAW_EINVAL;
  }
  if ((d->flags & TACAW_SLICE_BY_INSTANT_Z) && d->n_slices >= 32768) {
    set_error("per-frame slice binning holds slice indices in 16 bits (n_slices %d)", d->n_slices);
    return TACAW_EINVAL;
  }
  if (d->n_slices < 1) {
    set_error("n_slices must be >= 1 (got %d)", d->n_slices);
    return TACAW_EINVAL;
  }
  if (!(d->voltage_V > 0.0) || !isfinite(d->voltage_V)) {
    set_error("voltage_V must be positive (got %g)", d->voltage_V);
    return TACAW_EINVAL;
  }
  if (!(d->dt_fs > 0.0) || !isfinite(d->dt_fs)) {
    set_error("dt_fs must be positive (got %g)", d->dt_fs);
    return TACAW_EINVAL;
  }
  if (d->n_frames < 2 || !smooth235(d->n_frames)) {
    set_error("n_frames must be >= 2 and a product of 2, 3 and 5 (got %d)", d->n_frames);
    return TACAW_EINVAL;
  }
  if (d->n_frames > 2048) {
    set_error("n_frames %d above the 2048 the time stage holds in LDS", d->n_frames);
    return TACAW_EUNSUPPORTED;
  }
  if (d->n_atoms < 0) {
    set_error("n_atoms must be >= 0");
    return TACAW_EINVAL;
  }
  const bool kspace = d->kspace_coef != nullptr;
  if (d->n_species < 1 || !d->species_Z || (!kspace && (!d->gauss_a || !d->gauss_b))) {
    set_error("need n_species >= 1 with species_Z, and gauss_a and gauss_b unless kspace_coef is given");
    return TACAW_EINVAL;
  }
  if (kspace) {
    for (int s = 0; s < d->n_species; ++s)
      for (int i = 0; i < 12; ++i) {
        const double v = d->kspace_coef[s * 12 + i];
        const bool bad = !isfinite(v) || (i >= 3 && i < 6 && !(v > 0.0)) || (i >= 9 && !(v >= 0.0));
        if (bad) {
          set_error("kspace_coef[%d][%d] = %g: need finite values, b > 0 and d >= 0", s, i, v);
          return TACAW_EINVAL;
        }
      }
  } else {
    for (int i = 0; i < d->n_species * TACAW_N_GAUSS; ++i)
      if (!(d->gauss_a[i] > 0.0) || !(d->gauss_b[i] > 0.0) || !isfinite(d->gauss_a[i]) ||
          !isfinite(d->gauss_b[i])) {
        set_error("gauss_a and gauss_b must be positive and finite (entry %d)", i);
        return TACAW_EINVAL;
      }
  }
  if (d->aperture_mrad < 0.0 || !isfinite(d->aperture_mrad)) {
    set_error("aperture_mrad must be >= 0");
    return TACAW_EINVAL;
  }
  const bool plane = d->aperture_mrad == 0.0;
  const int pnx = d->pot_nx > 0 ? d->pot_nx : d->nx;
  const int pny = d->pot_ny > 0 ? d->pot_ny : d->ny;
  const bool windowed = pnx != d->nx || pny != d->ny;
  if (windowed) {
    if (plane) {
      set_error("a plane wave covers the cell: pot_nx/pot_ny must be 0 or equal nx/ny");
      return TACAW_EINVAL;
    }
    if (pnx < d->nx || pny < d->ny) {
      set_error("window %dx%d larger than the potential grid %dx%d", d->nx, d->ny, pnx, pny);
      return TACAW_EINVAL;
    }
  }
  if (!plane) {
    if (d->n_probes < 1 || !d->probe_xy) {
      set_error("a probe needs n_probes >= 1 and probe_xy");
      return TACAW_EINVAL;
    }
    for (int i = 0; i < 2 * d->n_probes; ++i)
      if (!isfinite(d->probe_xy[i])) {
        set_error("probe_xy[%d] is not finite", i);
        return TACAW_EINVAL;
      }
    const double dx = d->cell[0] / pnx, dy = d->cell[1] / pny;
    const double kny = 0.5 / std::max(dx, dy);
    const double ka = d->aperture_mrad * 1e-3 / wavelength_A(d->voltage_V);
    if (ka >= kny) {
      set_error("probe aperture alpha/lambda = %.4f 1/A does not fit below the Nyquist frequency %.4f 1/A",
                ka, kny);
      return TACAW_EINVAL;
    }
  }
  if (d->n_atoms >= (1 << 27)) {
    set_error("n_atoms %d above the 2^27 the pair lists encode", d->n_atoms);
    return TACAW_EUNSUPPORTED;
  }
  if (!grid_supported(d->nx) || !grid_supported(d->ny)) {
    set_error("grid %dx%d: the library has kernels for 16, 32, 48, 64, 96, 128, 160, 192, 256, 320, "
              "384, 512, 640, 768, 1024",
              d->nx, d->ny);
    return TACAW_EUNSUPPORTED;
  }
  if (kspace && (!grid_supported(pnx) || !grid_supported(pny))) {
    set_error("the reciprocal-space potential transforms the %dx%d potential grid: each side must be one of "
              "16, 32, 48, 64, 96, 128, 160, 192, 256, 320, 384, 512, 640, 768, 1024",
              pnx, pny);
    return TACAW_EUNSUPPORTED;
  }
  return TACAW_OK;
}

// Potentials of one slice are built right before that slice's row pass
// (per-slice mode) unless TACAW_SPLAT_ALL=1 asks for all slices of a frame
// batch at once.
bool splat_per_slice() {
  const char* e = getenv("TACAW_SPLAT_ALL");
  return !(e && atoi(e) != 0);
}

// TACAW_OVERLAP=1: per-slice potentials are built one slice ahead on a side
// stream (two alternating potential buffers).  Off by default: at 512^2 the
// concurrent potential launches take occupancy from the column pass and the
// whole step gets slower.
bool overlap_splat() {
  const char* e = getenv("TACAW_OVERLAP");
  return splat_per_slice() && e && atoi(e) != 0;
}

// Slices whose potentials one launch builds in the serial form.  Default:
// all slices of a frame batch at its start, while the potentials of the batch
// stay within TACAW_V_MB (default 4096 MiB), else the largest group that
// fits.  Building them up front keeps the potential writes from evicting the
// batch's waves from the last-level cache between the row and column passes
// (measured at 512^2 x 32 slices: 73.8 ms per step against 77.5 ms with
// groups of 4).  TACAW_SPLAT_GROUP overrides; TACAW_SPLAT_ALL=0 gives one
// slice per launch; the overlapped form builds one at a time.
int splat_group(int n_slices, int fb, int pnx, int pny) {
  if (overlap_splat()) return 1;
  if (const char* e = getenv("TACAW_SPLAT_GROUP")) return std::max(1, std::min(atoi(e), n_slices));
  if (!splat_per_slice()) return n_slices;
  if (const char* e = getenv("TACAW_SPLAT_ALL"))
    if (atoi(e) == 0) return 1;
  double cap = 4096.0 * (1 << 20);
  if (const char* e = getenv("TACAW_V_MB")) cap = atof(e) * (1 << 20);
  const double per_slice = (double)fb * pnx * pny * sizeof(float);
  return std::max(1, std::min(n_slices, (int)(cap / per_slice)));
}

// Slices per structure-factor launch of the reciprocal-space route: all
// slices of a frame batch while their potentials (4 B per point) and slice-pair
// structure factors (8 B per point per pair) stay within TACAW_V_MB (default
// 4096 MiB), else the largest even group that fits (at least 2).
int kspace_group(int n_slices, int fb, int pnx, int pny) {
  double cap = 4096.0 * (1 << 20);
  if (const char* e = getenv("TACAW_V_MB")) cap = atof(e) * (1 << 20);
  const double per_slice = (double)fb * pnx * pny * 8.0;   // V (4 B) + half a pair's W (4 B)
  int g = (int)std::min<double>(n_slices, std::max(2.0, floor(cap / per_slice)));
  if (g < n_slices && (g & 1)) --g;
  return std::max(1, g);
}

// Frames per batch: the waves and one slice of potentials of one batch should
// stay within ~240 MiB, so that between the row and column passes of a slice
// they can live in the 256 MiB last-level cache (at 512^2, 80-frame batches
// measured 72.7 ms per 1024-frame step against 73.7 ms at 64 and 82 ms at
// 112).  TACAW_FB overrides the choice and TACAW_BATCH_MB the target.
int choose_frame_batch(const tacaw_job_desc* d) {
  if (const char* e = getenv("TACAW_FB")) {
    const int fb = atoi(e);
    if (fb > 0) return std::min(fb, d->n_frames);
  }
  const int pnx = d->pot_nx > 0 ? d->pot_nx : d->nx;
  const int pny = d->pot_ny > 0 ? d->pot_ny : d->ny;
  const double P = d->aperture_mrad == 0.0 ? 1.0 : (double)d->n_probes;
  const double per_frame = P * d->nx * d->ny * 8.0 + pnx * pny * 4.0;
  double target = 240.0 * (1 << 20);
  if (const char* e = getenv("TACAW_BATCH_MB")) target = atof(e) * (1 << 20);
  const int fb = (int)std::max(1.0, floor(target / per_frame));
  return std::min(fb, d->n_frames);
}

Footprint footprint_of(const tacaw_job_desc* d, int fb, size_t n_tile_atoms) {
  Footprint f;
  const bool plane = d->aperture_mrad == 0.0;
  const size_t P = plane ? 1 : (size_t)d->n_probes;
  const size_t nk = (size_t)d->nx * d->ny;
  const int pnx = d->pot_nx > 0 ? d->pot_nx : d->nx;
  const int pny = d->pot_ny > 0 ? d->pot_ny : d->ny;
  const size_t M = (d->flags & TACAW_TWO_SIDED) ? d->n_frames : d->n_frames / 2;
  f.exit = P * d->n_frames * nk * sizeof(float2);
  f.spec = P * M * nk * sizeof(float);
  if (d->kspace_coef) {
    const int g = kspace_group(d->n_slices, fb, pnx, pny);
    const size_t pairs = (size_t)(g + 1) / 2;
    f.V = (size_t)fb * 2 * pairs * pnx * pny * sizeof(float);
    f.W = (size_t)fb * pairs * pnx * pny * sizeof(float2);
  } else {
    f.V = (size_t)fb * (overlap_splat() ? 2 : splat_group(d->n_slices, fb, pnx, pny)) * pnx * pny * sizeof(float);
  }
  f.pos = (size_t)d->n_frames * d->n_atoms * sizeof(AtomPos) + (size_t)d->n_atoms * sizeof(int32_t);
  if (d->flags & TACAW_SLICE_BY_INSTANT_Z) f.pos += (size_t)d->n_frames * d->n_atoms * sizeof(int16_t);
  f.tiles = n_tile_atoms * sizeof(int32_t);
  f.probes = plane ? 0 : P * nk * sizeof(float2) + P * (2 * sizeof(int32_t) + 2 * sizeof(double));
  f.tables = (size_t)(2 * d->nx + 2 * d->ny + d->nx + d->ny + d->n_frames) * sizeof(float2) +
             (size_t)d->n_species * N_GAUSS * COEF_STRIDE * sizeof(float) + 64;
  if (d->kspace_coef)
    f.tables += (size_t)(pnx + pny) * sizeof(float2) + (size_t)d->n_species * KP_NCOEF * sizeof(float) +
                ((size_t)d->n_slices * d->n_species + 1) * sizeof(int32_t);
  return f;
}

static inline double wrap_min_image(double d, double L) { return d - L * nearbyint(d / L); }

// fn(begin, end) over [0, n) in contiguous chunks on up to 16 threads (the
// host share of one GPU) when there are at least 2^22 work units (n times
// `units` per item); one thread otherwise.  Callers keep every per-item result
// independent of the split.
template <typename Fn>
static void parallel_for(size_t n, size_t units, Fn&& fn) {
  const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
  const unsigned nt = (unsigned)std::min<size_t>(std::min(16u, hw), n);
  if (nt <= 1 || n * units < ((size_t)1 << 22)) {
    fn((size_t)0, n);
    return;
  }
  std::vector<std::thread> th;
  const size_t chunk = (n + nt - 1) / nt;
  for (unsigned t = 0; t < nt; ++t) {
    const size_t b = t * chunk, e = std::min(n, b + chunk);
    if (b < e) th.emplace_back([&fn, b, e] { fn(b, e); });
  }
  for (auto& x : th) x.join();
}

// Reciprocal-space route: atoms of each (slice, species), in sorted order,
// and the form-factor coefficients (a and c times C/A, d times log2 e).
static void plan_kspace(const tacaw_job_desc* d, HostPlan& hp,
                        const std::vector<std::vector<int32_t>>& slice_atoms) {
  const double cpref_k = 2.0 * M_PI * kBohrA * kCoulombEVA / (hp.lx * hp.ly);
  hp.ks_start.assign((size_t)hp.ns * hp.S + 1, 0);
  hp.ks_atoms.clear();
  for (int s = 0; s < hp.ns; ++s)
    for (int z = 0; z < hp.S; ++z) {
      hp.ks_start[(size_t)s * hp.S + z] = (int32_t)hp.ks_atoms.size();
      for (const int j : slice_atoms[s])
        if (hp.sorted_species[j] == z) hp.ks_atoms.push_back(j);
    }
  hp.ks_start[(size_t)hp.ns * hp.S] = (int32_t)hp.ks_atoms.size();
  hp.kcoef.resize((size_t)hp.S * KP_NCOEF);
  for (int z = 0; z < hp.S; ++z)
    for (int i = 0; i < 3; ++i) {
      const double* c = d->kspace_coef + (size_t)z * 12;
      hp.kcoef[z * KP_NCOEF + i] = (float)(cpref_k * c[i]);
      hp.kcoef[z * KP_NCOEF + 3 + i] = (float)c[3 + i];
      hp.kcoef[z * KP_NCOEF + 6 + i] = (float)(cpref_k * c[6 + i]);
      hp.kcoef[z * KP_NCOEF + 9 + i] = (float)(c[9 + i] / M_LN2);
    }
  // no real-space tiles
  hp.tiles_x = (hp.pnx + SPLAT_TX - 1) / SPLAT_TX;
  hp.tiles_y = (hp.pny + SPLAT_TY - 1) / SPLAT_TY;
  hp.tile_start.assign((size_t)hp.ns * hp.tiles_x * hp.tiles_y + 1, 0);
  hp.tile_atoms.clear();
  hp.coef.assign((size_t)hp.S * N_GAUSS * COEF_STRIDE, 0.f);
}

// Real-space route: per-term coefficients and the candidate (atom, term)
// pairs of every (slice, 32 x 32 tile).
static void plan_real_space(const tacaw_job_desc* d, const double* pos, HostPlan& hp,
                            const std::vector<std::vector<int32_t>>& slice_atoms) {
  // Truncation radius: exp(-pi^2 r^2 / b) <= 1e-8 for the widest term.
  double bmax = 0.0;
  for (int i = 0; i < hp.S * TACAW_N_GAUSS; ++i) bmax = std::max(bmax, d->gauss_b[i]);
  hp.rc = sqrt(bmax * log(1e8)) / M_PI;
  hp.rcx = (float)(hp.rc / hp.dx);
  hp.rcy = (float)(hp.rc / hp.dy);
  auto images = [](double rcp, int n) {
    if (rcp < n / 2 - 1) return 0;
    return (int)ceil((rcp + n / 2 + 1) / n);
  };
  hp.img_x = images(hp.rcx, hp.pnx);
  hp.img_y = images(hp.rcy, hp.pny);

  // Per-species coefficients: amplitude C a pi / b (V A), exp2 factors per
  // pixel^2 along x and y, and each term's own truncation radius
  // sqrt(b ln 1e8)/pi in pixels (narrow terms reach far less than rc).
  const double cpref = 2.0 * M_PI * kBohrA * kCoulombEVA;
  hp.coef.resize((size_t)hp.S * N_GAUSS * COEF_STRIDE);
  for (int s = 0; s < hp.S; ++s)
    for (int i = 0; i < N_GAUSS; ++i) {
      const double a = d->gauss_a[s * N_GAUSS + i], b = d->gauss_b[s * N_GAUSS + i];
      const double c = M_PI * M_PI / b;
      const double rci = sqrt(b * log(1e8)) / M_PI;
      float* o = &hp.coef[((size_t)s * N_GAUSS + i) * COEF_STRIDE];
      o[0] = (float)(cpref * a * M_PI / b);
      o[1] = (float)(c * hp.dx * hp.dx / M_LN2);
      o[2] = (float)(c * hp.dy * hp.dy / M_LN2);
      o[3] = (float)(rci / hp.dx);
      o[4] = (float)(rci / hp.dy);
      o[5] = (float)log2(cpref * a * M_PI / b);   // amplitudes are positive (validated)
    }

  // Candidate (atom, term) pairs per (slice, tile): a term of an atom is listed
  // for a tile when its own truncation box, widened by that atom's largest
  // displacement from its mean position (and half a pixel for the rounding
  // of positions), can reach the tile along both axes (periodic).  Entries
  // are sorted-atom * 8 + term, in atom order then term order.
  // per atom: mean position (minimum-image displacements from frame 0, summed
  // over frames in order) and largest displacement from it
  std::vector<double> xbar(hp.A, 0.0), ybar(hp.A, 0.0), dmx(hp.A, 0.0), dmy(hp.A, 0.0);
  parallel_for((size_t)hp.A, (size_t)hp.F, [&](size_t j0, size_t j1) {
    for (int f = 0; f < hp.F; ++f)
      for (size_t j = j0; j < j1; ++j) {
        xbar[j] += wrap_min_image(pos[((size_t)f * hp.A + j) * 3] - pos[j * 3], hp.lx);
        ybar[j] += wrap_min_image(pos[((size_t)f * hp.A + j) * 3 + 1] - pos[j * 3 + 1], hp.ly);
      }
    for (size_t j = j0; j < j1; ++j) {
      xbar[j] = pos[j * 3] + xbar[j] / hp.F;
      ybar[j] = pos[j * 3 + 1] + ybar[j] / hp.F;
    }
    for (int f = 0; f < hp.F; ++f)
      for (size_t j = j0; j < j1; ++j) {
        dmx[j] = std::max(dmx[j], fabs(wrap_min_image(pos[((size_t)f * hp.A + j) * 3] - xbar[j], hp.lx)));
        dmy[j] = std::max(dmy[j], fabs(wrap_min_image(pos[((size_t)f * hp.A + j) * 3 + 1] - ybar[j], hp.ly)));
      }
  });
  hp.tiles_x = (hp.pnx + SPLAT_TX - 1) / SPLAT_TX;
  hp.tiles_y = (hp.pny + SPLAT_TY - 1) / SPLAT_TY;
  const int nt = hp.tiles_x * hp.tiles_y;
  hp.tile_start.assign((size_t)hp.ns * nt + 1, 0);
  hp.tile_atoms.clear();
  auto reached = [](double u, double L, double d, int n, int tile_w, int n_tiles, double reach,
                    std::vector<int>& out) {
    out.clear();
    for (int t = 0; t < n_tiles; ++t) {
      const double a0 = t * tile_w * d;
      const double a1 = (std::min((t + 1) * tile_w, n) - 1) * d;
      const double c = 0.5 * (a0 + a1), h = 0.5 * (a1 - a0);
      if (fabs(wrap_min_image(u - c, L)) - h <= reach) out.push_back(t);
    }
  };
  std::vector<std::vector<int32_t>> bucket(nt);
  std::vector<int> txs, tys;
  for (int s = 0; s < hp.ns; ++s) {
    for (auto& b : bucket) b.clear();
    for (const int j : slice_atoms[s]) {
      const int oj = hp.order[j];
      const int sp = hp.sorted_species[j];
      for (int i = 0; i < N_GAUSS; ++i) {
        const double rci = sqrt(d->gauss_b[sp * N_GAUSS + i] * log(1e8)) / M_PI;
        reached(xbar[oj], hp.lx, hp.dx, hp.pnx, SPLAT_TX, hp.tiles_x, rci + dmx[oj] + 0.5 * hp.dx, txs);
        reached(ybar[oj], hp.ly, hp.dy, hp.pny, SPLAT_TY, hp.tiles_y, rci + dmy[oj] + 0.5 * hp.dy, tys);
        for (int ty : tys)
          for (int tx : txs) bucket[ty * hp.tiles_x + tx].push_back((int32_t)(j * 8 + i));
      }
    }
    for (int t = 0; t < nt; ++t) {
      hp.tile_start[(size_t)s * nt + t] = (int32_t)hp.tile_atoms.size();
      hp.tile_atoms.insert(hp.tile_atoms.end(), bucket[t].begin(), bucket[t].end());
    }
  }
  hp.tile_start[(size_t)hp.ns * nt] = (int32_t)hp.tile_atoms.size();
}

tacaw_status plan_job(const tacaw_job_desc* d, const int32_t* atom_species, const double* pos,
                      HostPlan& hp) {
  hp.nx = d->nx;
  hp.ny = d->ny;
  hp.pnx = d->pot_nx > 0 ? d->pot_nx : d->nx;
  hp.pny = d->pot_ny > 0 ? d->pot_ny : d->ny;
  hp.ns = d->n_slices;
  hp.F = d->n_frames;
  hp.A = d->n_atoms;
  hp.S = d->n_species;
  hp.plane = d->aperture_mrad == 0.0;
  hp.P = hp.plane ? 1 : d->n_probes;
  hp.windowed = hp.pnx != hp.nx || hp.pny != hp.ny;
  hp.two_sided = (d->flags & TACAW_TWO_SIDED) != 0;
  hp.M = hp.two_sided ? hp.F : hp.F / 2;
  hp.lx = d->cell[0];
  hp.ly = d->cell[1];
  hp.lz = d->cell[2];
  hp.dx = hp.lx / hp.pnx;
  hp.dy = hp.ly / hp.pny;
  hp.dz = hp.lz / hp.ns;
  hp.lam = wavelength_A(d->voltage_V);
  hp.sigma = sigma_rad_per_VA(d->voltage_V);
  hp.alpha = d->aperture_mrad * 1e-3;
  hp.fb = choose_frame_batch(d);
  hp.kspace = d->kspace_coef != nullptr;
  hp.splat_per_slice = splat_per_slice();
  hp.overlap = overlap_splat() && !hp.kspace;
  hp.splat_group = splat_group(d->n_slices, hp.fb, hp.pnx, hp.pny);
  hp.kgroup = hp.kspace ? kspace_group(d->n_slices, hp.fb, hp.pnx, hp.pny) : 0;

  for (int j = 0; j < hp.A; ++j)
    if (atom_species[j] < 0 || atom_species[j] >= hp.S) {
      set_error("atom %d has species index %d outside [0, %d)", j, atom_species[j], hp.S);
      return TACAW_EINVAL;
    }
  {
    // first non-finite coordinate, if any (per-frame chunks, lowest index wins)
    const size_t per_frame = (size_t)hp.A * 3;
    std::vector<size_t> bad(hp.F, SIZE_MAX);
    parallel_for((size_t)hp.F, per_frame, [&](size_t f0, size_t f1) {
      for (size_t f = f0; f < f1; ++f)
        for (size_t i = f * per_frame; i < (f + 1) * per_frame; ++i)
          if (!isfinite(pos[i])) {
            bad[f] = i;
            break;
          }
    });
    for (size_t f = 0; f < (size_t)hp.F; ++f)
      if (bad[f] != SIZE_MAX) {
        set_error("positions[%zu] is not finite", bad[f]);
        return TACAW_EINVAL;
      }
  }

  // Slice binning by the FP64 frame-mean z; half-open slices, clamped.
  hp.slice_of.assign(hp.A, 0);
  std::vector<double> zbar(hp.A, 0.0);
  parallel_for((size_t)hp.A, (size_t)hp.F, [&](size_t j0, size_t j1) {
    for (int f = 0; f < hp.F; ++f)
      for (size_t j = j0; j < j1; ++j) zbar[j] += pos[((size_t)f * hp.A + j) * 3 + 2];
  });
  for (int j = 0; j < hp.A; ++j) {
    const double z = zbar[j] / (double)hp.F;
    double zm = fmod(z, hp.lz);
    if (zm != 0.0 && zm < 0.0) zm += hp.lz;
    long s = (long)floor(zm / hp.dz);
    if (s < 0) s = 0;
    if (s > hp.ns - 1) s = hp.ns - 1;
    hp.slice_of[j] = (int32_t)s;
  }
  hp.order.resize(hp.A);
  std::iota(hp.order.begin(), hp.order.end(), 0);
  std::stable_sort(hp.order.begin(), hp.order.end(),
                   [&](int a, int b) { return hp.slice_of[a] < hp.slice_of[b]; });
  std::vector<int32_t> slice_start(hp.ns + 1, 0);
  for (int j = 0; j < hp.A; ++j) slice_start[hp.slice_of[j] + 1]++;
  for (int s = 0; s < hp.ns; ++s) slice_start[s + 1] += slice_start[s];
  hp.sorted_species.resize(hp.A);
  for (int j = 0; j < hp.A; ++j) hp.sorted_species[j] = atom_species[hp.order[j]];

  // Per-frame binning (TACAW_SLICE_BY_INSTANT_Z): each frame's own z, the same
  // half-open clamped slices; an atom is a candidate in every slice it visits,
  // and the potential kernel skips it in frames where it is elsewhere.
  hp.instant_z = (d->flags & TACAW_SLICE_BY_INSTANT_Z) != 0;
  std::vector<std::vector<int32_t>> slice_atoms(hp.ns);   // sorted atom indices per slice
  if (hp.instant_z) {
    hp.fslice.assign((size_t)hp.F * hp.A, 0);
    parallel_for((size_t)hp.F, (size_t)hp.A, [&](size_t f0, size_t f1) {
      for (int f = (int)f0; f < (int)f1; ++f)
        for (int j = 0; j < hp.A; ++j) {
          double zm = fmod(pos[((size_t)f * hp.A + hp.order[j]) * 3 + 2], hp.lz);
          if (zm != 0.0 && zm < 0.0) zm += hp.lz;
          long s = (long)floor(zm / hp.dz);
          if (s < 0) s = 0;
          if (s > hp.ns - 1) s = hp.ns - 1;
          hp.fslice[(size_t)f * hp.A + j] = (int16_t)s;
        }
    });
    std::vector<int16_t> visited;
    for (int j = 0; j < hp.A; ++j) {   // atoms in sorted order, so every list stays sorted
      visited.clear();
      for (int f = 0; f < hp.F; ++f) visited.push_back(hp.fslice[(size_t)f * hp.A + j]);
      std::sort(visited.begin(), visited.end());
      visited.erase(std::unique(visited.begin(), visited.end()), visited.end());
      for (int16_t s : visited) slice_atoms[s].push_back(j);
    }
  } else {
    for (int s = 0; s < hp.ns; ++s)
      for (int j = slice_start[s]; j < slice_start[s + 1]; ++j) slice_atoms[s].push_back(j);
  }

  if (hp.kspace)
    plan_kspace(d, hp, slice_atoms);
  else
    plan_real_space(d, pos, hp, slice_atoms);

  // Probe windows: origin floor(r/d) - N/2 (wrapped for the crop); the probe
  // sits at r - origin * d inside the window.
  hp.origin.assign((size_t)hp.P * 2, 0);
  hp.rloc.assign((size_t)hp.P * 2, 0.0);
  if (!hp.plane) {
    for (int p = 0; p < hp.P; ++p) {
      const double rx = d->probe_xy[2 * p], ry = d->probe_xy[2 * p + 1];
      if (hp.windowed) {
        const long ox = (long)floor(rx / hp.dx) - hp.nx / 2;
        const long oy = (long)floor(ry / hp.dy) - hp.ny / 2;
        hp.origin[2 * p] = (int32_t)(((ox % hp.pnx) + hp.pnx) % hp.pnx);
        hp.origin[2 * p + 1] = (int32_t)(((oy % hp.pny) + hp.pny) % hp.pny);
        hp.rloc[2 * p] = rx - (double)ox * hp.dx;
        hp.rloc[2 * p + 1] = ry - (double)oy * hp.dy;
      } else {
        hp.rloc[2 * p] = rx;
        hp.rloc[2 * p + 1] = ry;
      }
    }
  }
  return TACAW_OK;
}

// Encode positions of frames [f0, f1) in sorted atom order: integer pixel and
// sub-pixel offset on the potential grid.
void encode_positions(const HostPlan& hp, const double* pos, int f0, int f1, AtomPos* out) {
  parallel_for((size_t)(f1 - f0), (size_t)hp.A, [&](size_t c0, size_t c1) {
    for (int f = f0 + (int)c0; f < f0 + (int)c1; ++f)
      for (int j = 0; j < hp.A; ++j) {
        const double* p = pos + ((size_t)f * hp.A + hp.order[j]) * 3;
        const double ux = p[0] / hp.dx, uy = p[1] / hp.dy;
        const double fxl = floor(ux), fyl = floor(uy);
        long ix = (long)fxl, iy = (long)fyl;
        AtomPos a;
        a.fx = (float)(ux - fxl);
        a.fy = (float)(uy - fyl);
        if (a.fx >= 1.0f) { a.fx = 0.0f; ix += 1; }  // rounding up to 1.0f
        if (a.fy >= 1.0f) { a.fy = 0.0f; iy += 1; }
        a.ix = (int32_t)(((ix % hp.pnx) + hp.pnx) % hp.pnx);
        a.iy = (int32_t)(((iy % hp.pny) + hp.pny) % hp.pny);
        out[(size_t)(f - f0) * hp.A + j] = a;
      }
  });
}

}  // namespace tacaw
