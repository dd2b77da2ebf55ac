// C ABI of libtacaw: contexts, jobs, the plain per-job run, results, timing.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <functional>
#include <vector>

#include "runtime.h"

namespace tacaw {
const char* last_error_text();
void encode_positions(const HostPlan& hp, const double* pos, int f0, int f1, AtomPos* out);
tacaw_status run_batch_range(tacaw_job* job, hipStream_t s, int f_begin, int f_end);
tacaw_status run_time_stage(tacaw_job* job, hipStream_t s);
tacaw_status materialize(tacaw_job* j, hipStream_t s = nullptr);
void release_working(tacaw_job* j);
}  // namespace tacaw

using namespace tacaw;

#define HIP_TRY(call)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess) {                                                               \
      set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, __LINE__); \
      return TACAW_EDEVICE;                                                               \
    }                                                                                     \
  } while (0)

namespace {

template <typename T>
hipError_t dalloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  return hipMalloc((void**)p, count * sizeof(T));
}

void drop_graph(tacaw_job* j) {
  if (j->graph_exec) (void)hipGraphExecDestroy(j->graph_exec);
  if (j->graph) (void)hipGraphDestroy(j->graph);
  j->graph_exec = nullptr;
  j->graph = nullptr;
}

// Free the job's device buffers.  keep_results: the spectrum and, with
// TACAW_KEEP_EXIT_WAVES, the exit store stay, and their pointer fields are
// not written (a reader of the results may run meanwhile).
void free_buffers(tacaw_job* j, bool keep_results) {
  drop_graph(j);
  const bool keep_exit = keep_results && (j->desc.flags & TACAW_KEEP_EXIT_WAVES);
  if (!keep_exit) {
    if (j->d_exit) {
      j->present.clear();   // a new exit store holds no frames
      (void)hipFree(j->d_exit);
    }
    j->d_exit = nullptr;
  }
  if (!keep_results) {
    if (j->d_spec) (void)hipFree(j->d_spec);
    j->d_spec = nullptr;
  }
  void* bufs[] = {j->d_V,       j->d_pos,     j->d_species,  j->d_tile_start, j->d_tile_atoms, j->d_coef,
                  j->d_tw_x,    j->d_tw_y,    j->d_tw_t,     j->d_px,         j->d_py,         j->d_px_last,
                  j->d_py_last, j->d_probe0,  j->d_origin,   j->d_rloc,       j->d_count,      j->d_fslice,
                  j->d_W,       j->d_ks_start, j->d_ks_atoms, j->d_kcoef,     j->d_tw_px,      j->d_tw_py};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  j->d_V = nullptr;
  j->d_pos = nullptr;
  j->d_species = nullptr;
  j->d_tile_start = nullptr;
  j->d_tile_atoms = nullptr;
  j->d_coef = nullptr;
  j->d_tw_x = j->d_tw_y = j->d_tw_t = nullptr;
  j->d_px = j->d_py = j->d_px_last = j->d_py_last = nullptr;
  j->d_probe0 = nullptr;
  j->d_origin = nullptr;
  j->d_rloc = nullptr;
  j->d_count = nullptr;
  j->d_fslice = nullptr;
  j->d_W = nullptr;
  j->d_ks_start = j->d_ks_atoms = nullptr;
  j->d_kcoef = nullptr;
  j->d_tw_px = j->d_tw_py = nullptr;
}

void free_job_buffers(tacaw_job* j) { free_buffers(j, false); }

hipEvent_t take_event(tacaw_ctx* c) {
  if (!c->event_pool.empty()) {
    hipEvent_t e = c->event_pool.back();
    c->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void drain_records(tacaw_ctx* c) {
  for (auto& r : c->records) {
    float ms = 0.f;
    if (hipEventSynchronize(r.stop) == hipSuccess && hipEventElapsedTime(&ms, r.start, r.stop) == hipSuccess) {
      c->total_ms[r.cls] += ms;
      c->launches[r.cls] += 1;
    }
    c->event_pool.push_back(r.start);
    c->event_pool.push_back(r.stop);
  }
  c->records.clear();
}

}  // namespace

namespace tacaw {

// Tile variant of the row pass (0: base rows per block, 1: doubled, 2: the
// register kernel for 64, 128, 256 and 512 (12- or 16-value registers for
// 384, 768 and 1024), 3: the same with two rows in flight per wavefront, 4:
// the six-step row kernel for 384 = 6 x 64, the default there) and of the
// column pass (0: half
// width, 1: full width, 2: register kernel on 8-16 column tiles for 64-512
// rows, 3: 16-column register tiles for 256 and 512 rows (variant 2 where the
// width is not a multiple of 16), 4: variant 2 with two LDS buffers, 5:
// six-step kernel for 512 rows, the default there, 6: the six-step kernel on
// 16-column tiles, 7: the six-step kernel for 256 rows on 16-column tiles,
// the default there (variant 3 where the width is not a multiple of 16), 8:
// the six-step kernel for 384 = 6 x 64 rows, the default there (variant 2
// where the width is not a multiple of 8)).  Tuned choices win;
// $TACAW_ROW_VARIANT and $TACAW_COL_VARIANT override untuned defaults.
static bool has_register_fft(int n) {
  return n == 64 || n == 128 || n == 256 || n == 384 || n == 512 || n == 768 || n == 1024;
}
int row_variant_for(tacaw_ctx* c, int n) {
  const int v = (n > 0 && n < 2048) ? c->row_variant[n] : 0;
  if (v) return v - 1;
  if (const char* e = getenv("TACAW_ROW_VARIANT")) return atoi(e);
  return n == 384 ? 4 : has_register_fft(n) ? 2 : 1;
}
int col_variant_for(tacaw_ctx* c, int n) {
  const int v = (n > 0 && n < 2048) ? c->col_variant[n] : 0;
  if (v) return v - 1;
  if (const char* e = getenv("TACAW_COL_VARIANT")) return atoi(e);
  return n == 512 ? 5 : n == 256 ? 7 : n == 384 ? 8 : has_register_fft(n) ? 2 : 0;
}

// Launch wrapper: when timing, the launch records a start and an end event
// on its stream.
tacaw_status timed_launch(tacaw_ctx* c, int cls, hipStream_t s, const std::function<hipError_t()>& launch) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  bool tm = false;
  {
    std::lock_guard<std::mutex> lk(c->mu);
    tm = c->timing && ((c->timing_mask >> cls) & 1u) && (c->launch_seq[cls]++ % c->timing_every) == 0;
    if (tm) {
      if (c->records.size() > 8192) drain_records(c);
      e0 = take_event(c);
      e1 = take_event(c);
    }
  }
  // the launch itself records the events (no separate event packets)
  if (tm && e0 && e1) set_launch_events(e0, e1);
  hipError_t e = launch();
  set_launch_events(nullptr, nullptr);
  if (tm && e0 && e1) {
    std::lock_guard<std::mutex> lk(c->mu);
    c->records.push_back({cls, e0, e1});
  }
  if (e != hipSuccess) {
    set_error("kernel launch failed: %s", hipGetErrorString(e));
    return TACAW_EDEVICE;
  }
  return TACAW_OK;
}

template <typename F>
static tacaw_status timed(tacaw_job* job, int cls, hipStream_t s, F&& launch) {
  return timed_launch(job->ctx, cls, s, std::function<hipError_t()>(launch));
}

PassArgs pass_args(tacaw_job* j) {
  const HostPlan& hp = j->hp;
  PassArgs a{};
  a.exit = j->d_exit;
  a.V = j->d_V;
  a.probe0 = j->d_probe0;
  a.origin = j->d_origin;
  a.tw_x = j->d_tw_x;
  a.tw_y = j->d_tw_y;
  a.px = j->d_px;
  a.py = j->d_py;
  a.nx = hp.nx;
  a.ny = hp.ny;
  a.pnx = hp.pnx;
  a.pny = hp.pny;
  a.n_frames = hp.F;
  a.n_probes = hp.P;
  a.n_slices = hp.ns;
  a.sigma = (float)hp.sigma;
  a.plane_amp = (float)(1.0 / sqrt((double)hp.nx * hp.ny));
  a.plane = hp.plane ? 1 : 0;
  return a;
}

// Whether waves of this job run resident in LDS (k_res): square 64 or 128
// grids, real-space potentials, unless TACAW_RESIDENT is 0 (then the row and
// column passes).  Measured faster than the passes at every wave count tried,
// 64 waves (64^2, one workgroup per wave) included.
bool resident_for(const tacaw_job* j) {
  const HostPlan& hp = j->hp;
  if (!resident_supported(hp.nx, hp.ny) || hp.kspace) return false;
  const char* e = getenv("TACAW_RESIDENT");
  return !(e && *e && atoi(e) == 0);
}

// One resident lane: frames [f0, f0 + fb) through slices sl .. sl + n - 1,
// whose potentials V holds as slices v_slice0 .. v_slice0 + v_slices - 1.
ResLane res_lane(tacaw_job* j, int f0, int fb, int sl, int n, int v_slices, int v_slice0) {
  ResLane l{};
  l.a = pass_args(j);
  l.a.f0 = f0;
  l.a.fb = fb;
  l.a.slice = sl;
  l.a.v_slices = v_slices;
  l.a.v_slice0 = v_slice0;
  l.px_last = j->d_px_last;
  l.py_last = j->d_py_last;
  l.n_slices_launch = n;
  return l;
}

static SplatArgs splat_args_of(tacaw_job* job, int f0, int fb) {
  const HostPlan& hp = job->hp;
  SplatArgs sa{};
  sa.pos = job->d_pos;
  sa.fslice = job->d_fslice;
  sa.species = job->d_species;
  sa.tile_start = job->d_tile_start;
  sa.tile_atoms = job->d_tile_atoms;
  sa.coef = job->d_coef;
  sa.V = job->d_V;
  sa.n_atoms = hp.A;
  sa.n_species = hp.S;
  sa.f0 = f0;
  sa.fb = fb;
  sa.n_slices = hp.ns;
  sa.slice0 = 0;
  sa.pnx = hp.pnx;
  sa.pny = hp.pny;
  sa.tiles_x = hp.tiles_x;
  sa.tiles_y = hp.tiles_y;
  sa.rcx = hp.rcx;
  sa.rcy = hp.rcy;
  sa.img_x = hp.img_x;
  sa.img_y = hp.img_y;
  return sa;
}

// Row pass then column pass of one slice for frames [f0, f0 + fb); the
// potential of that slice is read from V, which holds slices v_slice0 ..
// v_slice0 + v_slices - 1 of each frame.  after_row, if given, is recorded
// once the row pass (the potential's only reader) is queued.
static tacaw_status slice_passes(tacaw_job* job, hipStream_t s, int f0, int fb, int sl, float* V, int v_slices,
                                 int v_slice0, hipEvent_t after_row = nullptr) {
  const HostPlan& hp = job->hp;
  PassArgs a = pass_args(job);
  a.f0 = f0;
  a.fb = fb;
  a.V = V;
  a.v_slices = v_slices;
  a.v_slice0 = v_slice0;
  a.slice = sl;
  PassLane rl{};
  rl.a = a;
  rl.mode = sl == 0 ? ROW_FIRST : ROW_REGULAR;
  const int rv = row_variant_for(job->ctx, hp.nx);
  tacaw_status st = timed(job, TACAW_K_ROW, s, [&] { return launch_row_lanes(&rl, 1, rv, s); });
  if (st != TACAW_OK) return st;
  if (after_row) HIP_TRY(hipEventRecord(after_row, s));
  const bool last = sl == hp.ns - 1;
  PassLane cl{};
  cl.a = a;
  if (last) {
    cl.a.px = job->d_px_last;
    cl.a.py = job->d_py_last;
  }
  cl.mode = last ? COL_LAST : COL_REGULAR;
  const int cv = col_variant_for(job->ctx, hp.ny);
  return timed(job, TACAW_K_COL, s, [&] { return launch_col_lanes(&cl, 1, cv, s); });
}

// Potentials + all slices for frames [f_begin, f_end) (one or more frame batches).
//
// Overlapped form (per-slice potentials): the potential of step k + 1 (a
// (frame batch, slice) pair) is built on the job's side stream while the row
// and column passes of step k run on s.  Potentials alternate between two
// buffers; step k's row pass waits for its potential, and the potential of
// step k + 2 waits for step k's row pass, the last reader of that buffer.
// Every side-stream launch is waited on by s, so s alone orders completion
// (and a capture of s takes in the side stream's work).
// Potentials of slices g0 .. g0 + gn - 1 of frames [f0, f0 + fb) by the
// paper's reciprocal-space route: structure factors of the slice pairs into
// W, an unnormalised inverse 2D FFT of W (column pass, then row pass), whose
// real and imaginary parts land in V as the pair's two potentials.
static tacaw_status kspace_potentials(tacaw_job* job, hipStream_t s, int f0, int fb, int g0, int gn) {
  const HostPlan& hp = job->hp;
  KPotArgs k{};
  k.pos = job->d_pos;
  k.ks_start = job->d_ks_start;
  k.ks_atoms = job->d_ks_atoms;
  k.fslice = job->d_fslice;
  k.kcoef = job->d_kcoef;
  k.W = job->d_W;
  k.n_atoms = hp.A;
  k.n_species = hp.S;
  k.f0 = f0;
  k.fb = fb;
  k.n_slices = hp.ns;
  k.slice0 = g0;
  k.npairs = (gn + 1) / 2;
  k.pnx = hp.pnx;
  k.pny = hp.pny;
  k.row_tiles = (hp.pny / 2 + 1 + KP_TY - 1) / KP_TY;
  k.col_tiles = (hp.pnx + KP_TX - 1) / KP_TX;
  k.kx_unit = (float)(1.0 / hp.lx);
  k.ky_unit = (float)(1.0 / hp.ly);
  tacaw_status st = timed(job, TACAW_K_SPLAT, s, [&] { return launch_kpot(k, s); });
  if (st != TACAW_OK) return st;
  PassArgs a{};
  a.exit = job->d_W;
  a.tw_x = hp.windowed ? job->d_tw_px : job->d_tw_x;
  a.tw_y = hp.windowed ? job->d_tw_py : job->d_tw_y;
  a.nx = a.pnx = hp.pnx;
  a.ny = a.pny = hp.pny;
  a.n_probes = 1;
  a.n_frames = a.fb = fb * k.npairs;
  a.f0 = 0;
  a.plane = 1;
  // the register kernels where the size has them (else the LDS kernels)
  PassLane l{};
  l.a = a;
  l.mode = COL_INVERSE_ONLY;
  st = timed(job, TACAW_K_OTHER, s, [&] { return launch_col_lanes(&l, 1, 2, s); });
  if (st != TACAW_OK) return st;
  l.a.vout = job->d_V;
  l.mode = ROW_INVERSE_ONLY;
  return timed(job, TACAW_K_OTHER, s, [&] { return launch_row_lanes(&l, 1, 2, s); });
}

tacaw_status run_batch_range(tacaw_job* job, hipStream_t s, int f_begin, int f_end) {
  const HostPlan& hp = job->hp;
  if (hp.kspace) {
    const int G = hp.kgroup;
    for (int f0 = f_begin; f0 < f_end; f0 += hp.fb) {
      const int fb = std::min(hp.fb, f_end - f0);
      for (int g0 = 0; g0 < hp.ns; g0 += G) {
        const int gn = std::min(G, hp.ns - g0);
        tacaw_status st = kspace_potentials(job, s, f0, fb, g0, gn);
        if (st != TACAW_OK) return st;
        for (int sl = g0; sl < g0 + gn; ++sl)
          if ((st = slice_passes(job, s, f0, fb, sl, job->d_V, 2 * ((gn + 1) / 2), g0)) != TACAW_OK) return st;
      }
    }
    return TACAW_OK;
  }
  if (!hp.overlap) {
    // serial form: potentials of hp.splat_group slices (all slices when not
    // per slice), then their row and column passes, or one resident launch
    // that carries the waves through all of them
    const int G = hp.splat_group;
    for (int f0 = f_begin; f0 < f_end; f0 += hp.fb) {
      const int fb = std::min(hp.fb, f_end - f0);
      const bool res = resident_for(job);
      for (int g0 = 0; g0 < hp.ns; g0 += G) {
        const int gn = std::min(G, hp.ns - g0);
        SplatArgs sa = splat_args_of(job, f0, fb);
        sa.slice0 = g0;
        tacaw_status st = timed(job, TACAW_K_SPLAT, s, [&] { return launch_splat(sa, gn, s); });
        if (st != TACAW_OK) return st;
        if (res) {
          const ResLane rl = res_lane(job, f0, fb, g0, gn, gn, g0);
          st = timed(job, TACAW_K_ROW, s, [&] { return launch_res_lanes(&rl, 1, s); });
          if (st != TACAW_OK) return st;
          continue;
        }
        for (int sl = g0; sl < g0 + gn; ++sl)
          if ((st = slice_passes(job, s, f0, fb, sl, job->d_V, gn, g0)) != TACAW_OK) return st;
      }
    }
    return TACAW_OK;
  }
  if (f_begin >= f_end) return TACAW_OK;
  const size_t slab = (size_t)hp.fb * hp.pnx * hp.pny;
  const int n_batches = (f_end - f_begin + hp.fb - 1) / hp.fb;
  const long n_steps = (long)n_batches * hp.ns;
  auto step_f0 = [&](long k) { return f_begin + (int)(k / hp.ns) * hp.fb; };
  auto splat_step = [&](long k) -> tacaw_status {
    const int f0 = step_f0(k), fb = std::min(hp.fb, f_end - f0), b = (int)(k & 1);
    if (k >= 2) HIP_TRY(hipStreamWaitEvent(job->side, job->ev_row[b], 0));
    SplatArgs sa = splat_args_of(job, f0, fb);
    sa.V = job->d_V + b * slab;
    sa.slice0 = (int)(k % hp.ns);
    tacaw_status st = timed(job, TACAW_K_SPLAT, job->side, [&] { return launch_splat(sa, 1, job->side); });
    if (st != TACAW_OK) return st;
    HIP_TRY(hipEventRecord(job->ev_splat[b], job->side));
    return TACAW_OK;
  };
  // fork: the side stream starts after the work already queued on s
  HIP_TRY(hipEventRecord(job->ev_fork, s));
  HIP_TRY(hipStreamWaitEvent(job->side, job->ev_fork, 0));
  tacaw_status st = splat_step(0);
  for (long k = 0; k < n_steps && st == TACAW_OK; ++k) {
    if (k + 1 < n_steps && (st = splat_step(k + 1)) != TACAW_OK) break;
    HIP_TRY(hipStreamWaitEvent(s, job->ev_splat[k & 1], 0));
    const int f0 = step_f0(k), fb = std::min(hp.fb, f_end - f0);
    const int sl = (int)(k % hp.ns);
    st = slice_passes(job, s, f0, fb, sl, job->d_V + (k & 1) * slab, 1, sl, job->ev_row[k & 1]);
  }
  if (st != TACAW_OK) {
    // join the side stream so nothing it holds outlives an error return
    (void)hipEventRecord(job->ev_fork, job->side);
    (void)hipStreamWaitEvent(s, job->ev_fork, 0);
  }
  return st;
}

tacaw_status run_time_stage(tacaw_job* job, hipStream_t s) {
  const HostPlan& hp = job->hp;
  TimeArgs t{};
  t.exit = job->d_exit;
  t.spec = job->d_spec;
  t.tw = job->d_tw_t;
  t.n_k = hp.nx * hp.ny;
  t.n_frames = hp.F;
  t.n_bins = hp.M;
  t.n_probes = hp.P;
  t.kt = time_stage_kt(hp.F, t.n_k);
  t.inv_f2 = (float)(1.0 / ((double)hp.F * hp.F));
  return timed(job, TACAW_K_TIME, s, [&] { return launch_time_stage(t, s); });
}


// Allocate the job's device buffers, upload its inputs and build its tables
// and incident probes.  Synchronous.
// Incident probes in real space: aperture (and aberration phase) filled in
// reciprocal space, then brought to real space by the inverse-only passes.
hipError_t build_probe(tacaw_job* j, hipStream_t s0) {
  const HostPlan& hp = j->hp;
  hipError_t e;
  if ((e = hipMemsetAsync(j->d_count, 0, sizeof(int), s0)) != hipSuccess) return e;
  if ((e = launch_aperture_count(j->d_count, hp.nx, hp.ny, hp.dx, hp.dy, hp.lam, hp.alpha, s0)) != hipSuccess)
    return e;
  if ((e = launch_probe_fill(j->d_probe0, j->d_rloc, j->d_count, hp.P, hp.nx, hp.ny, hp.dx, hp.dy, hp.lam,
                             hp.alpha, j->aberr, s0)) != hipSuccess)
    return e;
  PassArgs a = pass_args(j);
  a.exit = j->d_probe0;
  a.n_frames = 1;
  a.f0 = 0;
  a.fb = 1;
  if ((e = launch_col_pass(a, COL_INVERSE_ONLY, s0)) != hipSuccess) return e;
  return launch_row_pass(a, ROW_INVERSE_ONLY, s0);
}

tacaw_status materialize(tacaw_job* j, hipStream_t s0) {
  if (j->materialized) return TACAW_OK;
  HIP_TRY(hipSetDevice(j->ctx->device));
  HostPlan& hp = j->hp;
  auto fail = [&](const char* what, hipError_t e) {
    set_error("%s: %s", what, hipGetErrorString(e));
    free_job_buffers(j);
    return e == hipErrorOutOfMemory ? TACAW_ENOMEM : TACAW_EDEVICE;
  };
  hipError_t e;
  const size_t nk = (size_t)hp.nx * hp.ny;
#define ALLOC(ptr, count) \
  if ((e = dalloc(&(ptr), (count))) != hipSuccess) return fail("hipMalloc " #ptr, e);
  if (!j->d_exit) ALLOC(j->d_exit, (size_t)hp.P * hp.F * nk);
  if (!j->d_spec) ALLOC(j->d_spec, (size_t)hp.P * hp.M * nk);
  const int kpairs = (hp.kgroup + 1) / 2;
  ALLOC(j->d_V, (size_t)hp.fb * (hp.kspace ? 2 * kpairs : hp.overlap ? 2 : hp.splat_group) * hp.pnx * hp.pny);
  if (hp.kspace) {
    ALLOC(j->d_W, (size_t)hp.fb * kpairs * hp.pnx * hp.pny);
    ALLOC(j->d_ks_start, hp.ks_start.size());
    ALLOC(j->d_ks_atoms, hp.ks_atoms.size());
    ALLOC(j->d_kcoef, hp.kcoef.size());
    if (hp.windowed) {
      ALLOC(j->d_tw_px, (size_t)hp.pnx);
      ALLOC(j->d_tw_py, (size_t)hp.pny);
    }
  }
  ALLOC(j->d_pos, (size_t)hp.F * hp.A);
  ALLOC(j->d_species, (size_t)hp.A);
  if (hp.instant_z) ALLOC(j->d_fslice, hp.fslice.size());
  ALLOC(j->d_tile_start, hp.tile_start.size());
  ALLOC(j->d_tile_atoms, hp.tile_atoms.size());
  ALLOC(j->d_coef, hp.coef.size());
  ALLOC(j->d_tw_x, (size_t)hp.nx);
  ALLOC(j->d_tw_y, (size_t)hp.ny);
  ALLOC(j->d_tw_t, (size_t)hp.F);
  ALLOC(j->d_px, (size_t)hp.nx);
  ALLOC(j->d_py, (size_t)hp.ny);
  ALLOC(j->d_px_last, (size_t)hp.nx);
  ALLOC(j->d_py_last, (size_t)hp.ny);
  ALLOC(j->d_origin, (size_t)hp.P * 2);
  ALLOC(j->d_rloc, (size_t)hp.P * 2);
  ALLOC(j->d_count, 1);
  if (!hp.plane) ALLOC(j->d_probe0, (size_t)hp.P * nk);
#undef ALLOC
  if (hp.overlap && !j->side) {
    if ((e = hipStreamCreateWithFlags(&j->side, hipStreamNonBlocking)) != hipSuccess) return fail("side stream", e);
    hipEvent_t* evs[] = {&j->ev_fork, &j->ev_splat[0], &j->ev_splat[1], &j->ev_row[0], &j->ev_row[1]};
    for (hipEvent_t* ev : evs)
      if ((e = hipEventCreateWithFlags(ev, hipEventDisableTiming)) != hipSuccess) return fail("event", e);
  }

  if (hp.A > 0) {
    if ((e = hipMemcpyAsync(j->d_pos, j->enc.data(), j->enc.size() * sizeof(AtomPos), hipMemcpyHostToDevice, s0)) !=
        hipSuccess)
      return fail("upload positions", e);
    if ((e = hipMemcpyAsync(j->d_species, hp.sorted_species.data(), hp.A * sizeof(int32_t), hipMemcpyHostToDevice, s0)) !=
        hipSuccess)
      return fail("upload species", e);
    if (hp.instant_z &&
        (e = hipMemcpyAsync(j->d_fslice, hp.fslice.data(), hp.fslice.size() * sizeof(int16_t), hipMemcpyHostToDevice,
                            s0)) != hipSuccess)
      return fail("upload frame slices", e);
  }
  if ((e = hipMemcpyAsync(j->d_tile_start, hp.tile_start.data(), hp.tile_start.size() * sizeof(int32_t),
                     hipMemcpyHostToDevice, s0)) != hipSuccess)
    return fail("upload tiles", e);
  if (!hp.tile_atoms.empty() &&
      (e = hipMemcpyAsync(j->d_tile_atoms, hp.tile_atoms.data(), hp.tile_atoms.size() * sizeof(int32_t),
                     hipMemcpyHostToDevice, s0)) != hipSuccess)
    return fail("upload tile atoms", e);
  if ((e = hipMemcpyAsync(j->d_coef, hp.coef.data(), hp.coef.size() * sizeof(float), hipMemcpyHostToDevice, s0)) !=
      hipSuccess)
    return fail("upload coefficients", e);
  if (hp.kspace) {
    if ((e = hipMemcpyAsync(j->d_ks_start, hp.ks_start.data(), hp.ks_start.size() * sizeof(int32_t),
                            hipMemcpyHostToDevice, s0)) != hipSuccess)
      return fail("upload structure-factor lists", e);
    if (!hp.ks_atoms.empty() &&
        (e = hipMemcpyAsync(j->d_ks_atoms, hp.ks_atoms.data(), hp.ks_atoms.size() * sizeof(int32_t),
                            hipMemcpyHostToDevice, s0)) != hipSuccess)
      return fail("upload structure-factor lists", e);
    if ((e = hipMemcpyAsync(j->d_kcoef, hp.kcoef.data(), hp.kcoef.size() * sizeof(float), hipMemcpyHostToDevice,
                            s0)) != hipSuccess)
      return fail("upload form-factor coefficients", e);
    if (hp.windowed) {
      if ((e = launch_twiddles(j->d_tw_px, hp.pnx, s0)) != hipSuccess) return fail("twiddles", e);
      if ((e = launch_twiddles(j->d_tw_py, hp.pny, s0)) != hipSuccess) return fail("twiddles", e);
    }
  }
  if ((e = hipMemcpyAsync(j->d_origin, hp.origin.data(), hp.origin.size() * sizeof(int32_t), hipMemcpyHostToDevice, s0)) !=
      hipSuccess)
    return fail("upload origins", e);
  if ((e = hipMemcpyAsync(j->d_rloc, hp.rloc.data(), hp.rloc.size() * sizeof(double), hipMemcpyHostToDevice, s0)) !=
      hipSuccess)
    return fail("upload probe positions", e);

  // tables and incident probes on the device, then synchronise the stream
  const double sx = 1.0 / hp.nx, sy = 1.0 / hp.ny;
  const double lx = 1.0 / sqrt((double)hp.nx), ly = 1.0 / sqrt((double)hp.ny);
  if ((e = launch_twiddles(j->d_tw_x, hp.nx, s0)) != hipSuccess) return fail("twiddles", e);
  if ((e = launch_twiddles(j->d_tw_y, hp.ny, s0)) != hipSuccess) return fail("twiddles", e);
  if ((e = launch_twiddles(j->d_tw_t, hp.F, s0)) != hipSuccess) return fail("twiddles", e);
  if ((e = launch_prop_factor(j->d_px, hp.nx, hp.dx, hp.lam, hp.dz, sx, s0)) != hipSuccess) return fail("prop", e);
  if ((e = launch_prop_factor(j->d_py, hp.ny, hp.dy, hp.lam, hp.dz, sy, s0)) != hipSuccess) return fail("prop", e);
  if ((e = launch_prop_factor(j->d_px_last, hp.nx, hp.dx, hp.lam, hp.dz, lx, s0)) != hipSuccess)
    return fail("prop", e);
  if ((e = launch_prop_factor(j->d_py_last, hp.ny, hp.dy, hp.lam, hp.dz, ly, s0)) != hipSuccess)
    return fail("prop", e);
  if (!hp.plane && (e = build_probe(j, s0)) != hipSuccess) return fail("incident probe", e);
  if ((e = hipStreamSynchronize(s0)) != hipSuccess) return fail("job setup", e);
  j->materialized = true;
  return TACAW_OK;
}

// Free every device buffer except the spectrum and (when kept) the exit waves.
void release_working(tacaw_job* j) {
  free_buffers(j, true);
  j->materialized = false;
}

void mark_all_present(tacaw_job* j) { j->present.assign(j->hp.F, 1); }

size_t resident_bytes_after_done(const tacaw_job* j) {
  return j->fp.spec + ((j->desc.flags & TACAW_KEEP_EXIT_WAVES) ? j->fp.exit : 0);
}

}  // namespace tacaw

extern "C" {

const char* tacaw_last_error(void) { return last_error_text(); }

const char* tacaw_version(void) { return "libtacaw 0.1 (gfx950)"; }

tacaw_status tacaw_ctx_create(int device, size_t hbm_budget_bytes, tacaw_ctx** out) {
  clear_error();
  if (!out) {
    set_error("out is NULL");
    return TACAW_EINVAL;
  }
  *out = nullptr;
  int n = 0;
  HIP_TRY(hipGetDeviceCount(&n));
  if (device < 0 || device >= n) {
    set_error("device %d not in [0, %d)", device, n);
    return TACAW_EINVAL;
  }
  HIP_TRY(hipSetDevice(device));
  size_t fr = 0, tot = 0;
  HIP_TRY(hipMemGetInfo(&fr, &tot));
  // device address of the allocation-free entry points' fixed scratch array
  tacaw_status st = noalloc_init(device);
  if (st != TACAW_OK) return st;
  // kernel attributes (large dynamic LDS) set before any launch, so that no
  // first launch inside a graph capture has to set them
  hipError_t ke = kernels_init();
  if (ke != hipSuccess) {
    set_error("kernel attributes: %s", hipGetErrorString(ke));
    return TACAW_EDEVICE;
  }
  tacaw_ctx* c = new tacaw_ctx();
  c->device = device;
  load_tune_cache(c);   // tuned row and column variants of earlier runs, if any
  c->budget = hbm_budget_bytes ? hbm_budget_bytes : (size_t)(0.9 * (double)fr);
  *out = c;
  return TACAW_OK;
}

void tacaw_serve_shutdown(tacaw_ctx* c);

tacaw_status tacaw_ctx_destroy(tacaw_ctx* c) {
  clear_error();
  if (!c) return TACAW_OK;
  tacaw_serve_shutdown(c);
  {
    std::lock_guard<std::mutex> lk(c->mu);
    drain_records(c);
    for (hipEvent_t e : c->event_pool) (void)hipEventDestroy(e);
    c->event_pool.clear();
  }
  delete c;
  return TACAW_OK;
}

tacaw_status tacaw_job_footprint(const tacaw_job_desc* d, size_t* bytes) {
  clear_error();
  tacaw_status st = validate_desc(d);
  if (st != TACAW_OK) return st;
  if (!bytes) {
    set_error("bytes is NULL");
    return TACAW_EINVAL;
  }
  // candidate lists are not known before planning: bound them by 5 terms x 16 tiles per atom
  *bytes = footprint_of(d, choose_frame_batch(d), (size_t)d->n_atoms * 80 + 1).total();
  return TACAW_OK;
}

tacaw_status tacaw_job_create(tacaw_ctx* ctx, const tacaw_job_desc* d, const int32_t* atom_species,
                              const double* positions, tacaw_job** out) {
  clear_error();
  if (!ctx || !out) {
    set_error("ctx and out must not be NULL");
    return TACAW_EINVAL;
  }
  *out = nullptr;
  tacaw_status st = validate_desc(d);
  if (st != TACAW_OK) return st;
  if (d->n_atoms > 0 && (!atom_species || !positions)) {
    set_error("atom_species and positions must not be NULL when n_atoms > 0");
    return TACAW_EINVAL;
  }
  tacaw_job* j = new tacaw_job();
  j->ctx = ctx;
  j->desc = *d;
  const bool plane = d->aperture_mrad == 0.0;
  if (!plane) j->probe_xy.assign(d->probe_xy, d->probe_xy + 2 * (size_t)d->n_probes);
  j->species_Z.assign(d->species_Z, d->species_Z + d->n_species);
  if (d->gauss_a && d->gauss_b) {
    j->gauss_a.assign(d->gauss_a, d->gauss_a + (size_t)d->n_species * TACAW_N_GAUSS);
    j->gauss_b.assign(d->gauss_b, d->gauss_b + (size_t)d->n_species * TACAW_N_GAUSS);
  }
  if (d->kspace_coef) j->kspace_coef.assign(d->kspace_coef, d->kspace_coef + (size_t)d->n_species * 12);
  j->desc.probe_xy = plane ? nullptr : j->probe_xy.data();
  j->desc.species_Z = j->species_Z.data();
  j->desc.gauss_a = j->gauss_a.empty() ? nullptr : j->gauss_a.data();
  j->desc.gauss_b = j->gauss_b.empty() ? nullptr : j->gauss_b.data();
  j->desc.kspace_coef = j->kspace_coef.empty() ? nullptr : j->kspace_coef.data();
  if (plane) j->desc.n_probes = 1;

  static const double no_pos[1] = {0.0};
  static const int32_t no_sp[1] = {0};
  st = plan_job(&j->desc, d->n_atoms ? atom_species : no_sp, d->n_atoms ? positions : no_pos, j->hp);
  if (st != TACAW_OK) {
    delete j;
    return st;
  }
  j->fp = footprint_of(&j->desc, j->hp.fb, j->hp.kspace ? j->hp.ks_atoms.size() : j->hp.tile_atoms.size());
  // deferred jobs are checked against the budget when submitted
  if (!(d->flags & TACAW_DEFER_ALLOC) && j->fp.total() > ctx->budget) {
    set_error("job needs %.3f GiB of device memory, above the context budget of %.3f GiB",
              j->fp.total() / 1073741824.0, ctx->budget / 1073741824.0);
    delete j;
    return TACAW_ENOMEM;
  }
  if (j->hp.A > 0) {
    j->enc.resize((size_t)j->hp.F * j->hp.A);
    encode_positions(j->hp, positions, 0, j->hp.F, j->enc.data());
  }
  if (!(d->flags & TACAW_DEFER_ALLOC)) {
    st = materialize(j);
    if (st != TACAW_OK) {
      delete j;
      return st;
    }
  }
  *out = j;
  return TACAW_OK;
}

static void mark_present(tacaw_job* job, int f_begin, int f_end);

tacaw_status tacaw_run(tacaw_job* job, void* hip_stream) {
  clear_error();
  if (!job) {
    set_error("job is NULL");
    return TACAW_EINVAL;
  }
  const int ss = job->serve_state.load();
  if (ss == 1 || ss == 2) {
    set_error("job is in the serving loop");
    return TACAW_EBUSY;
  }
  leave_serving_state(job);
  HIP_TRY(hipSetDevice(job->ctx->device));
  tacaw_status st = materialize(job);
  if (st != TACAW_OK) return st;
  hipStream_t s = (hipStream_t)hip_stream;
  job->last_stream = s;
  bool timing = false;
  {
    std::lock_guard<std::mutex> lk(job->ctx->mu);
    timing = job->ctx->timing;
  }
  if ((job->desc.flags & TACAW_USE_GRAPH) && !timing) {
    if (!job->graph_exec) {
      // capture on the job's own stream, replay on any stream
      if (!job->capture_stream) HIP_TRY(hipStreamCreateWithFlags(&job->capture_stream, hipStreamNonBlocking));
      HIP_TRY(hipStreamBeginCapture(job->capture_stream, hipStreamCaptureModeThreadLocal));
      st = run_batch_range(job, job->capture_stream, 0, job->hp.F);
      if (st == TACAW_OK) st = run_time_stage(job, job->capture_stream);
      hipGraph_t g = nullptr;
      hipError_t e = hipStreamEndCapture(job->capture_stream, &g);
      if (st != TACAW_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
      }
      if (e != hipSuccess) {
        set_error("graph capture failed: %s", hipGetErrorString(e));
        return TACAW_EDEVICE;
      }
      job->graph = g;
      HIP_TRY(hipGraphInstantiate(&job->graph_exec, job->graph, nullptr, nullptr, 0));
    }
    HIP_TRY(hipGraphLaunch(job->graph_exec, s));
    mark_present(job, 0, job->hp.F);
    job->has_result = true;
    return TACAW_OK;
  }
  st = run_batch_range(job, s, 0, job->hp.F);
  if (st != TACAW_OK) return st;
  st = run_time_stage(job, s);
  if (st != TACAW_OK) return st;
  mark_present(job, 0, job->hp.F);
  job->has_result = true;
  return TACAW_OK;
}

// ---- frame ranges, checkpoints and the deferred time stage ----------------
static tacaw_status check_idle(tacaw_job* job) {
  if (!job) {
    set_error("job is NULL");
    return TACAW_EINVAL;
  }
  const int ss = job->serve_state.load();
  if (ss == 1 || ss == 2) {
    set_error("job is in the serving loop");
    return TACAW_EBUSY;
  }
  return TACAW_OK;
}

static tacaw_status check_range(const tacaw_job* job, int32_t f_begin, int32_t f_end) {
  if (f_begin < 0 || f_end > job->hp.F || f_begin >= f_end) {
    set_error("frame range [%d, %d) is empty or outside [0, %d)", f_begin, f_end, job->hp.F);
    return TACAW_EINVAL;
  }
  return TACAW_OK;
}

static void mark_present(tacaw_job* job, int f_begin, int f_end) {
  if (job->present.size() != (size_t)job->hp.F) job->present.assign(job->hp.F, 0);
  for (int f = f_begin; f < f_end; ++f) job->present[f] = 1;
}

tacaw_status tacaw_run_frames(tacaw_job* job, int32_t f_begin, int32_t f_end, void* hip_stream) {
  clear_error();
  tacaw_status st = check_idle(job);
  if (st != TACAW_OK) return st;
  if ((st = check_range(job, f_begin, f_end)) != TACAW_OK) return st;
  leave_serving_state(job);
  HIP_TRY(hipSetDevice(job->ctx->device));
  if ((st = materialize(job)) != TACAW_OK) return st;
  hipStream_t s = (hipStream_t)hip_stream;
  job->last_stream = s;
  if ((st = run_batch_range(job, s, f_begin, f_end)) != TACAW_OK) return st;
  mark_present(job, f_begin, f_end);
  return TACAW_OK;
}

tacaw_status tacaw_finish(tacaw_job* job, void* hip_stream) {
  clear_error();
  tacaw_status st = check_idle(job);
  if (st != TACAW_OK) return st;
  int missing = job->hp.F;
  if (job->present.size() == (size_t)job->hp.F)
    for (uint8_t v : job->present) missing -= v ? 1 : 0;
  if (missing > 0 || !job->materialized) {
    set_error("%d of %d frames have no exit waves yet", missing, job->hp.F);
    return TACAW_ENOTREADY;
  }
  leave_serving_state(job);
  HIP_TRY(hipSetDevice(job->ctx->device));
  hipStream_t s = (hipStream_t)hip_stream;
  job->last_stream = s;
  if ((st = run_time_stage(job, s)) != TACAW_OK) return st;
  job->has_result = true;
  return TACAW_OK;
}

// [P][f_end - f_begin][ny][nx] complex64 of the store's frames, per probe
static tacaw_status exit_frames_copy(tacaw_job* job, int32_t f_begin, int32_t f_end, void* host_or_dev,
                                     int on_device, bool to_store) {
  const HostPlan& hp = job->hp;
  const size_t nk = (size_t)hp.nx * hp.ny, nf = (size_t)(f_end - f_begin);
  const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice
                                       : (to_store ? hipMemcpyHostToDevice : hipMemcpyDeviceToHost);
  HIP_TRY(hipStreamSynchronize(job->last_stream));
  for (int p = 0; p < hp.P; ++p) {
    float2* store = job->d_exit + ((size_t)p * hp.F + f_begin) * nk;
    float2* user = (float2*)host_or_dev + (size_t)p * nf * nk;
    if (to_store)
      HIP_TRY(hipMemcpy(store, user, nf * nk * sizeof(float2), kind));
    else
      HIP_TRY(hipMemcpy(user, store, nf * nk * sizeof(float2), kind));
  }
  return TACAW_OK;
}

tacaw_status tacaw_get_exit_frames(tacaw_job* job, int32_t f_begin, int32_t f_end, void* dst, size_t n,
                                   int dst_on_device) {
  clear_error();
  tacaw_status st = check_idle(job);
  if (st != TACAW_OK) return st;
  if ((st = check_range(job, f_begin, f_end)) != TACAW_OK) return st;
  const HostPlan& hp = job->hp;
  if (!dst || n != (size_t)hp.P * (f_end - f_begin) * hp.nx * hp.ny) {
    set_error("dst must hold n_probes * frames * ny * nx = %zu complex values",
              (size_t)hp.P * (f_end - f_begin) * hp.nx * hp.ny);
    return TACAW_EINVAL;
  }
  for (int f = f_begin; f < f_end; ++f)
    if (!job->has_result && (job->present.size() != (size_t)hp.F || !job->present[f])) {
      set_error("frame %d has no exit waves yet", f);
      return TACAW_ENOTREADY;
    }
  HIP_TRY(hipSetDevice(job->ctx->device));
  return exit_frames_copy(job, f_begin, f_end, dst, dst_on_device, false);
}

tacaw_status tacaw_put_exit_frames(tacaw_job* job, int32_t f_begin, int32_t f_end, const void* src, size_t n,
                                   int src_on_device) {
  clear_error();
  tacaw_status st = check_idle(job);
  if (st != TACAW_OK) return st;
  if ((st = check_range(job, f_begin, f_end)) != TACAW_OK) return st;
  const HostPlan& hp = job->hp;
  if (!src || n != (size_t)hp.P * (f_end - f_begin) * hp.nx * hp.ny) {
    set_error("src must hold n_probes * frames * ny * nx = %zu complex values",
              (size_t)hp.P * (f_end - f_begin) * hp.nx * hp.ny);
    return TACAW_EINVAL;
  }
  HIP_TRY(hipSetDevice(job->ctx->device));
  if ((st = materialize(job)) != TACAW_OK) return st;
  if ((st = exit_frames_copy(job, f_begin, f_end, const_cast<void*>(src), src_on_device, true)) != TACAW_OK)
    return st;
  mark_present(job, f_begin, f_end);
  return TACAW_OK;
}

static tacaw_status copy_out(tacaw_job* job, void* dst, const void* src, size_t bytes, int on_device) {
  if (on_device) {
    HIP_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, job->last_stream));
    HIP_TRY(hipStreamSynchronize(job->last_stream));
  } else {
    HIP_TRY(hipStreamSynchronize(job->last_stream));
    HIP_TRY(hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost));
  }
  return TACAW_OK;
}

tacaw_status tacaw_get_spectrum(tacaw_job* job, float* dst, size_t n, int dst_on_device) {
  clear_error();
  if (!job || !dst) {
    set_error("job and dst must not be NULL");
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
  if (!job->has_result) {
    set_error("job has not been run");
    return TACAW_ENOTREADY;
  }
  const HostPlan& hp = job->hp;
  const size_t need = (size_t)hp.P * hp.M * hp.nx * hp.ny;
  if (n != need) {
    set_error("spectrum has %zu values, dst holds %zu", need, n);
    return TACAW_EINVAL;
  }
  HIP_TRY(hipSetDevice(job->ctx->device));
  return copy_out(job, dst, job->d_spec, need * sizeof(float), dst_on_device);
}

tacaw_status tacaw_get_exit_waves(tacaw_job* job, void* dst, size_t n, int dst_on_device) {
  clear_error();
  if (!job || !dst) {
    set_error("job and dst must not be NULL");
    return TACAW_EINVAL;
  }
  if (!(job->desc.flags & TACAW_KEEP_EXIT_WAVES)) {
    set_error("job was created without TACAW_KEEP_EXIT_WAVES");
    return TACAW_EINVAL;
  }
  const int ss = job->serve_state.load();
  if (ss == 1 || ss == 2) {
    set_error("job is still in the serving loop");
    return TACAW_EBUSY;
  }
  if (!job->has_result) {
    set_error("job has not been run");
    return TACAW_ENOTREADY;
  }
  const HostPlan& hp = job->hp;
  const size_t need = (size_t)hp.P * hp.F * hp.nx * hp.ny;
  if (n != need) {
    set_error("exit-wave store has %zu complex values, dst holds %zu", need, n);
    return TACAW_EINVAL;
  }
  HIP_TRY(hipSetDevice(job->ctx->device));
  return copy_out(job, dst, job->d_exit, need * sizeof(float2), dst_on_device);
}

tacaw_status tacaw_axes(const tacaw_job_desc* d, double* kx, double* ky, double* f) {
  clear_error();
  tacaw_status st = validate_desc(d);
  if (st != TACAW_OK && st != TACAW_EUNSUPPORTED) return st;
  const int pnx = d->pot_nx > 0 ? d->pot_nx : d->nx;
  const int pny = d->pot_ny > 0 ? d->pot_ny : d->ny;
  const double dx = d->cell[0] / pnx, dy = d->cell[1] / pny;
  auto fill = [](double* out, int n, double dd) {
    const double val = 1.0 / ((double)n * dd);
    for (int i = 0; i < n; ++i) out[i] = (double)((i < (n + 1) / 2) ? i : i - n) * val;
  };
  if (kx) fill(kx, d->nx, dx);
  if (ky) fill(ky, d->ny, dy);
  if (f) {
    const int F = d->n_frames;
    const bool two = (d->flags & TACAW_TWO_SIDED) != 0;
    const int M = two ? F : F / 2;
    const double val = 1.0 / ((double)F * (d->dt_fs * 1e-3));
    for (int m = 0; m < M; ++m) f[m] = (double)((m < (F + 1) / 2) ? m : m - F) * val;
  }
  return TACAW_OK;
}

tacaw_status tacaw_job_slices(const tacaw_job* job, int32_t* out, size_t n) {
  clear_error();
  if (!job || (!out && n)) {
    set_error("job and out must not be NULL");
    return TACAW_EINVAL;
  }
  if (n != job->hp.slice_of.size()) {
    set_error("job has %zu atoms, out holds %zu", job->hp.slice_of.size(), n);
    return TACAW_EINVAL;
  }
  std::copy(job->hp.slice_of.begin(), job->hp.slice_of.end(), out);
  return TACAW_OK;
}

tacaw_status tacaw_job_set_aberrations(tacaw_job* job, const double* c_angstrom, const double* phi_rad) {
  clear_error();
  if (!job) {
    set_error("job is NULL");
    return TACAW_EINVAL;
  }
  if (job->hp.plane) {
    set_error("a plane-wave job has no probe to aberrate");
    return TACAW_EINVAL;
  }
  const int ss = job->serve_state.load();
  if (ss == 1 || ss == 2) {
    set_error("job is still in the serving loop");
    return TACAW_EBUSY;
  }
  Aberrations ab{};
  if (c_angstrom) {
    for (int i = 0; i < N_ABERR; ++i) {
      const double c = c_angstrom[i], a = phi_rad ? phi_rad[i] : 0.0;
      if (!isfinite(c) || !isfinite(a)) {
        set_error("aberration coefficient %d is not finite", i);
        return TACAW_EINVAL;
      }
      ab.c[i] = c;
      ab.phi[i] = a;
      ab.on |= c != 0.0;
    }
  }
  job->aberr = ab;
  // a job that already holds its incident probes rebuilds them now; the
  // current spectrum stays until the next run replaces it
  if (job->materialized && job->d_probe0) {
    HIP_TRY(hipSetDevice(job->ctx->device));
    hipError_t e = build_probe(job, job->last_stream);
    if (e == hipSuccess) e = hipStreamSynchronize(job->last_stream);
    if (e != hipSuccess) {
      set_error("incident probe: %s", hipGetErrorString(e));
      return TACAW_EDEVICE;
    }
  }
  return TACAW_OK;
}

tacaw_status tacaw_job_plan(const tacaw_job* job, int32_t* frame_batch, int32_t* slices_per_potential_launch) {
  clear_error();
  if (!job) {
    set_error("job is NULL");
    return TACAW_EINVAL;
  }
  if (frame_batch) *frame_batch = job->hp.fb;
  if (slices_per_potential_launch) *slices_per_potential_launch = job->hp.splat_group;
  return TACAW_OK;
}

tacaw_status tacaw_job_destroy(tacaw_job* job) {
  clear_error();
  if (!job) return TACAW_OK;
  const int ss = job->serve_state.load();
  if (ss == 1 || ss == 2) {
    set_error("job is in the serving loop: cancel and wait first");
    return TACAW_EBUSY;
  }
  wait_released(job);   // the serving loop's release of this job has run
  (void)hipSetDevice(job->ctx->device);
  (void)hipDeviceSynchronize();
  if (job->retained) {
    std::lock_guard<std::mutex> lk(job->ctx->mu);
    job->ctx->resident -= job->retained;
  }
  free_job_buffers(job);
  if (job->capture_stream) (void)hipStreamDestroy(job->capture_stream);
  if (job->side) (void)hipStreamDestroy(job->side);
  for (hipEvent_t ev : {job->ev_fork, job->ev_splat[0], job->ev_splat[1], job->ev_row[0], job->ev_row[1]})
    if (ev) (void)hipEventDestroy(ev);
  delete job;
  return TACAW_OK;
}

tacaw_status tacaw_timing_enable(tacaw_ctx* c, int on) {
  clear_error();
  if (!c) {
    set_error("ctx is NULL");
    return TACAW_EINVAL;
  }
  std::lock_guard<std::mutex> lk(c->mu);
  drain_records(c);
  c->timing = on != 0;
  if (on)
    for (int i = 0; i < TACAW_K_COUNT; ++i) {
      c->total_ms[i] = 0.0;
      c->launches[i] = 0;
    }
  return TACAW_OK;
}

tacaw_status tacaw_timing_select(tacaw_ctx* c, unsigned class_mask, int every) {
  clear_error();
  if (!c || every < 1) {
    set_error("ctx is NULL or every < 1");
    return TACAW_EINVAL;
  }
  std::lock_guard<std::mutex> lk(c->mu);
  c->timing_mask = class_mask;
  c->timing_every = every;
  for (int i = 0; i < TACAW_K_COUNT; ++i) c->launch_seq[i] = 0;
  return TACAW_OK;
}

tacaw_status tacaw_timing_get(tacaw_ctx* c, int cls, double* total_ms, int64_t* launches) {
  clear_error();
  if (!c || cls < 0 || cls >= TACAW_K_COUNT) {
    set_error("bad context or kernel class");
    return TACAW_EINVAL;
  }
  std::lock_guard<std::mutex> lk(c->mu);
  drain_records(c);
  if (total_ms) *total_ms = c->total_ms[cls];
  if (launches) *launches = c->launches[cls];
  return TACAW_OK;
}

}  // extern "C"
