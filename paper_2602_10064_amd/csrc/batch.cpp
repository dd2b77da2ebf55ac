// Batched execution of uneven jobs, the autotuner, and HIP-graph replay of a
// job's launch sequence.
//
// Batched form: jobs whose frame batches hold at least TACAW_BATCH_LARGE_MB of
// waves run one after another on the first stream, one frame batch per round,
// exactly as the plain form runs them.  The smaller jobs are grouped by grid
// size; inside a group a launch advances up to MAX_LANES lanes by one pass, a
// lane being one frame batch of one job at its own slice (each lane has its
// own potentials, exit store, tables and mode).  A lane at the start of one of
// its job's slice groups builds that group's potential slices in the shared
// potential launch.  When a lane finishes its last slice the next frame batch
// (of the same or another job) takes its place, so slice steps of different
// jobs are batched continuously.  A job has at most one lane in flight (its
// potential buffer belongs to one frame batch), and lanes are admitted while
// their waves and potentials fit TACAW_BATCH_LANE_MB.  Groups and the large
// jobs are enqueued round-robin on up to four streams, joined back to the
// caller's stream.  Every wave is computed by the same per-row and per-column
// arithmetic as in tacaw_run, so results are bitwise those of the plain form.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <deque>
#include <fstream>
#include <map>
#include <sstream>
#include <vector>

#include "runtime.h"

namespace tacaw {
void mark_all_present(tacaw_job* j);   // every frame of the exit store holds exit waves
}

using namespace tacaw;

namespace {

tacaw_status ensure_streams(tacaw_ctx* c) {
  for (auto& st : c->batch_streams)
    if (!st && hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      set_error("hipStreamCreate failed");
      return TACAW_EDEVICE;
    }
  return TACAW_OK;
}

SplatArgs splat_args(tacaw_job* j, int f0, int fb, int slice) {
  const HostPlan& hp = j->hp;
  SplatArgs sa{};
  sa.pos = j->d_pos;
  sa.fslice = j->d_fslice;
  sa.species = j->d_species;
  sa.tile_start = j->d_tile_start;
  sa.tile_atoms = j->d_tile_atoms;
  sa.coef = j->d_coef;
  sa.V = j->d_V;
  sa.n_atoms = hp.A;
  sa.n_species = hp.S;
  sa.f0 = f0;
  sa.fb = fb;
  sa.n_slices = hp.ns;
  sa.slice0 = slice;
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

}  // namespace

namespace tacaw {

// Jobs whose frame batches hold at least TACAW_BATCH_LARGE_MB (default 64)
// MiB of waves fill the device on their own and run as the plain form runs
// them (sharing launches would only make the working set outgrow the
// last-level cache); jobs on the reciprocal-space potential route build their
// potentials with their own launch sequence.  The others share launches.
bool shares_launches(const tacaw_job* j) {
  double large_mb = 64.0;
  if (const char* e = getenv("TACAW_BATCH_LARGE_MB")) large_mb = atof(e);
  const HostPlan& hp = j->hp;
  const double wave_mb = (double)hp.fb * hp.P * hp.nx * hp.ny * 8.0 / (1 << 20);
  return wave_mb < large_mb && !hp.kspace;
}

// One group of same-grid jobs on one stream, advanced one iteration at a
// time: each iteration launches the potentials of the lanes that start a
// slice group, then one row pass and one column pass over all active lanes.
LaneGroup::LaneGroup(tacaw_ctx* ctx, hipStream_t stream, int nx, int ny, bool serving_)
    : c(ctx), s(stream), serving(serving_) {
  rv = row_variant_for(c, nx);
  cv = col_variant_for(c, ny);
}

void LaneGroup::add(tacaw_job* j) {
  for (int f0 = 0; f0 < j->hp.F; f0 += j->hp.fb) pending.push_back({j, f0, std::min(j->hp.fb, j->hp.F - f0), 0});
  left[j] = (j->hp.F + j->hp.fb - 1) / j->hp.fb;
}

bool LaneGroup::has(const tacaw_job* j) const { return left.count(const_cast<tacaw_job*>(j)) > 0; }

bool LaneGroup::drop(tacaw_job* j) {
  if (!has(j)) return true;
  for (auto it = pending.begin(); it != pending.end();) it = it->job == j ? pending.erase(it) : it + 1;
  for (auto& l : active)
    if (l.job == j) {
      dropped.insert(j);   // its lane ends with the frame batch in flight; no time stage
      return false;
    }
  left.erase(j);
  return true;
}

// waves and one potential slice of a lane's frame batch
static double lane_bytes(const LaneGroup::Lane& l) {
  const HostPlan& hp = l.job->hp;
  return (double)l.fb * ((double)hp.P * hp.nx * hp.ny * 8.0 + (double)hp.pnx * hp.pny * 4.0);
}

tacaw_status LaneGroup::step(std::vector<tacaw_job*>* finished) {
  // fill free lanes: at most one lane per job (a job has one potential
  // buffer), and while the lanes' waves fit the working-set target
  // (TACAW_BATCH_LANE_MB, default 256: the last-level cache), at least one
  const char* e = getenv("TACAW_BATCH_LANE_MB");
  const double cap = (e ? atof(e) : 256.0) * (1 << 20);
  double in_use = 0.0;
  for (auto& l : active) in_use += lane_bytes(l);
  for (auto it = pending.begin(); it != pending.end() && (int)active.size() < MAX_LANES;) {
    bool busy = false;
    for (auto& l : active) busy |= l.job == it->job;
    if (busy) {
      ++it;
      continue;
    }
    if (!active.empty() && in_use + lane_bytes(*it) > cap) break;
    in_use += lane_bytes(*it);
    active.push_back(*it);
    it = pending.erase(it);
  }
  const int n = (int)active.size();
  if (n == 0) return TACAW_OK;
  // resident step: every lane runs to the end of its slice group in one
  // launch, the waves held in LDS (square 64 and 128 grids)
  const bool res = resident_for(active[0].job);
  // potentials: a lane at the start of a slice group builds that group's
  // slices (the job's splat_group) in this iteration's potential launch
  SplatLane sl[MAX_LANES];
  PassLane rl[MAX_LANES], cl[MAX_LANES];
  ResLane xl[MAX_LANES];
  int n_splat = 0;
  for (int i = 0; i < n; ++i) {
    Lane& L = active[i];
    tacaw_job* j = L.job;
    const int G = j->hp.splat_group;
    const int g0 = L.slice - L.slice % G;
    const int gn = std::min(G, j->hp.ns - g0);
    if (L.slice == g0) {
      sl[n_splat] = SplatLane{};
      sl[n_splat].a = splat_args(j, L.f0, L.fb, g0);
      sl[n_splat].n_slices_launch = gn;
      ++n_splat;
    }
    xl[i] = res_lane(j, L.f0, L.fb, L.slice, g0 + gn - L.slice, gn, g0);
    PassArgs a = pass_args(j);
    a.f0 = L.f0;
    a.fb = L.fb;
    a.slice = L.slice;
    a.v_slices = gn;
    a.v_slice0 = g0;
    rl[i] = PassLane{};
    rl[i].a = a;
    rl[i].mode = L.slice == 0 ? ROW_FIRST : ROW_REGULAR;
    const bool last = L.slice == j->hp.ns - 1;
    cl[i] = PassLane{};
    cl[i].a = a;
    if (last) {
      cl[i].a.px = j->d_px_last;
      cl[i].a.py = j->d_py_last;
    }
    cl[i].mode = last ? COL_LAST : COL_REGULAR;
  }
  tacaw_status st = TACAW_OK;
  if (n_splat > 0) {
    st = timed_launch(c, TACAW_K_SPLAT, s, [&] { return launch_splat_lanes(sl, n_splat, s); });
    if (st != TACAW_OK) return st;
  }
  if (res) {
    st = timed_launch(c, TACAW_K_ROW, s, [&] { return launch_res_lanes(xl, n, s); });
    if (st != TACAW_OK) return st;
  } else {
    st = timed_launch(c, TACAW_K_ROW, s, [&] { return launch_row_lanes(rl, n, rv, s); });
    if (st != TACAW_OK) return st;
    st = timed_launch(c, TACAW_K_COL, s, [&] { return launch_col_lanes(cl, n, cv, s); });
    if (st != TACAW_OK) return st;
  }
  if (n > 1) {
    // the pass launches (one resident launch, or a row and a column launch)
    // served several jobs
    shared_launches += res ? 1 : 2;
    for (const Lane& L : active) L.job->shared_launch = true;
  }
  std::vector<Lane> still;
  for (int i = 0; i < n; ++i) {
    Lane& L = active[i];
    L.slice += res ? xl[i].n_slices_launch : 1;
    if (L.slice < L.job->hp.ns) {
      still.push_back(L);
      continue;
    }
    tacaw_job* j = L.job;
    if (dropped.count(j)) {
      // a dropped job ends with its lane: no time stage
      dropped.erase(j);
      left.erase(j);
      if (finished) finished->push_back(j);
      continue;
    }
    if (--left[j] == 0) {
      left.erase(j);
      st = run_time_stage(j, s);
      if (st != TACAW_OK) return st;
      if (!serving) {
        mark_all_present(j);
        j->has_result = true;
        j->last_stream = s;
      }
      if (finished) finished->push_back(j);
    }
  }
  active.swap(still);
  return TACAW_OK;
}

// The tuned variants of earlier runs (TACAW_TUNE_CACHE, JSON lines), read
// once per context: at creation, and by the autotuner and the batched
// executor for contexts created before the variable was set.
void load_tune_cache(tacaw_ctx* c) {
  if (c->tune_loaded) return;
  const char* path = getenv("TACAW_TUNE_CACHE");
  if (!path) return;   // read later, once the variable is set
  c->tune_loaded = true;
  c->tune_cache = path;
  std::ifstream in(path);
  std::string line;
  while (std::getline(in, line)) {
    int nx = 0, ny = 0, r = 0, cc = 0;
    if (sscanf(line.c_str(), "{\"nx\": %d, \"ny\": %d, \"row_variant\": %d, \"col_variant\": %d}", &nx, &ny, &r,
               &cc) == 4 &&
        nx > 0 && nx < 2048 && ny > 0 && ny < 2048 && r >= 0 && r <= 4 && cc >= 0 && cc <= 8) {
      c->row_variant[nx] = r + 1;
      c->col_variant[ny] = cc + 1;
    }
  }
}

}  // namespace tacaw

namespace {

// Checks of a batch: jobs of one context, none twice, none in the serving loop.
tacaw_status check_batch(tacaw_job* const* jobs, int n_jobs) {
  if (!jobs || n_jobs < 1) {
    set_error("need at least one job");
    return TACAW_EINVAL;
  }
  tacaw_ctx* c = jobs[0] ? jobs[0]->ctx : nullptr;
  for (int i = 0; i < n_jobs; ++i) {
    if (!jobs[i] || jobs[i]->ctx != c) {
      set_error("job %d is NULL or belongs to another context", i);
      return TACAW_EINVAL;
    }
    const int ss = jobs[i]->serve_state.load();
    if (ss == 1 || ss == 2) {
      set_error("job %d is in the serving loop", i);
      return TACAW_EBUSY;
    }
    for (int k = 0; k < i; ++k)
      if (jobs[k] == jobs[i]) {
        set_error("job %d appears twice", i);
        return TACAW_EINVAL;
      }
  }
  return TACAW_OK;
}

// Enqueue the batched form of every job on `user` (and the context's batch
// streams, forked from and joined back to it).  Host-side bookkeeping only;
// nothing here waits for the device, so a capture of `user` takes it all in.
tacaw_status enqueue_batch(tacaw_ctx* c, tacaw_job* const* jobs, int n_jobs, hipStream_t user) {
  load_tune_cache(c);
  tacaw_status st = ensure_streams(c);
  if (st != TACAW_OK) return st;
  // Large jobs run one after another on the first stream, exactly as the
  // plain form runs them; the others share launches, grouped by grid, on the
  // other streams.
  std::map<std::pair<int, int>, std::vector<tacaw_job*>> groups;
  std::vector<tacaw_job*> large;
  for (int i = 0; i < n_jobs; ++i) {
    st = materialize(jobs[i], nullptr);
    if (st != TACAW_OK) return st;
    const HostPlan& hp = jobs[i]->hp;
    if (shares_launches(jobs[i]))
      groups[{hp.nx, hp.ny}].push_back(jobs[i]);
    else
      large.push_back(jobs[i]);
  }
  hipEvent_t start;
  if (hipEventCreateWithFlags(&start, hipEventDisableTiming) != hipSuccess) {
    set_error("hipEventCreate failed");
    return TACAW_EDEVICE;
  }
  (void)hipEventRecord(start, user);
  std::vector<LaneGroup> runs;
  bool used[4] = {false, false, false, false};
  int n_streams = 4;   // TACAW_BATCH_STREAMS: streams the work spreads over (1-4)
  if (const char* e = getenv("TACAW_BATCH_STREAMS")) n_streams = std::max(1, std::min(4, atoi(e)));
  const int first_group_stream = (large.empty() || n_streams == 1) ? 0 : 1;
  for (auto& g : groups) {
    const int span = n_streams - first_group_stream;
    const int k = first_group_stream + (int)runs.size() % span;
    if (!used[k]) (void)hipStreamWaitEvent(c->batch_streams[k], start, 0);
    used[k] = true;
    runs.emplace_back(c, c->batch_streams[k], g.first.first, g.first.second, false);
    for (tacaw_job* j : g.second) runs.back().add(j);
  }
  // the large jobs advance one frame batch per round of the loop below
  size_t li = 0;
  int lf = 0;
  hipStream_t s0 = c->batch_streams[0];
  if (!large.empty()) {
    if (!used[0]) (void)hipStreamWaitEvent(s0, start, 0);
    used[0] = true;
  }
  auto large_step = [&]() -> tacaw_status {
    tacaw_job* j = large[li];
    const int f1 = std::min(lf + j->hp.fb, j->hp.F);
    tacaw_status r = run_batch_range(j, s0, lf, f1);
    if (r != TACAW_OK) return r;
    lf = f1;
    if (lf == j->hp.F) {
      r = run_time_stage(j, s0);
      if (r != TACAW_OK) return r;
      mark_all_present(j);
      j->has_result = true;
      ++li;
      lf = 0;
    }
    return TACAW_OK;
  };
  // enqueue the groups' iterations round-robin, so that every stream has
  // work queued while the others run
  for (bool more = st == TACAW_OK; more && st == TACAW_OK;) {
    more = false;
    if (li < large.size()) {
      st = large_step();
      if (st != TACAW_OK) break;
      more = true;
    }
    for (auto& r : runs) {
      if (r.done()) continue;
      st = r.step(nullptr);
      if (st != TACAW_OK) break;
      more = true;
    }
  }
  for (int i = 0; i < 4; ++i) {
    if (!used[i]) continue;
    hipEvent_t done;
    if (hipEventCreateWithFlags(&done, hipEventDisableTiming) != hipSuccess) continue;
    (void)hipEventRecord(done, c->batch_streams[i]);
    (void)hipStreamWaitEvent(user, done, 0);
    (void)hipEventDestroy(done);
  }
  (void)hipEventDestroy(start);
  if (st != TACAW_OK) return st;
  for (int i = 0; i < n_jobs; ++i) jobs[i]->last_stream = user;
  return TACAW_OK;
}

}  // namespace

// A captured batch: the whole batched launch sequence of a fixed set of jobs
// as one HIP graph, replayed on any stream.  The graph holds the jobs' device
// addresses at capture time.
struct tacaw_batch {
  tacaw_ctx* ctx = nullptr;
  std::vector<tacaw_job*> jobs;
  std::vector<std::vector<const void*>> buffers;   // per job: every device buffer at capture
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {
// every device buffer a job's kernels may touch
std::vector<const void*> job_buffers(const tacaw_job* j) {
  return {j->d_exit,    j->d_spec,   j->d_V,       j->d_pos,      j->d_species,  j->d_tile_start, j->d_tile_atoms,
          j->d_coef,    j->d_tw_x,   j->d_tw_y,    j->d_tw_t,     j->d_px,       j->d_py,         j->d_px_last,
          j->d_py_last, j->d_probe0, j->d_origin,  j->d_rloc,     j->d_count,    j->d_fslice,     j->d_W,
          j->d_ks_start, j->d_ks_atoms, j->d_kcoef, j->d_tw_px,  j->d_tw_py};
}
}  // namespace

extern "C" {

tacaw_status tacaw_run_batch(tacaw_job* const* jobs, int n_jobs, void* hip_stream) {
  clear_error();
  tacaw_status st = check_batch(jobs, n_jobs);
  if (st != TACAW_OK) return st;
  tacaw_ctx* c = jobs[0]->ctx;
  for (int i = 0; i < n_jobs; ++i) leave_serving_state(jobs[i]);
  if (hipSetDevice(c->device) != hipSuccess) {
    set_error("hipSetDevice failed");
    return TACAW_EDEVICE;
  }
  return enqueue_batch(c, jobs, n_jobs, (hipStream_t)hip_stream);
}

tacaw_status tacaw_batch_capture(tacaw_job* const* jobs, int32_t n_jobs, tacaw_batch** out) {
  clear_error();
  if (!out) {
    set_error("out is NULL");
    return TACAW_EINVAL;
  }
  *out = nullptr;
  tacaw_status st = check_batch(jobs, n_jobs);
  if (st != TACAW_OK) return st;
  tacaw_ctx* c = jobs[0]->ctx;
  if (hipSetDevice(c->device) != hipSuccess) {
    set_error("hipSetDevice failed");
    return TACAW_EDEVICE;
  }
  // allocation and uploads stay outside the graph
  for (int i = 0; i < n_jobs; ++i)
    if ((st = materialize(jobs[i], nullptr)) != TACAW_OK) return st;
  hipStream_t cap = nullptr;
  if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) {
    set_error("hipStreamCreate failed");
    return TACAW_EDEVICE;
  }
  bool timing = false;
  {
    std::lock_guard<std::mutex> lk(c->mu);
    timing = c->timing;
    c->timing = false;   // no timing events inside the graph
  }
  tacaw_batch* b = new tacaw_batch();
  b->ctx = c;
  hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    st = enqueue_batch(c, jobs, n_jobs, cap);
    e = hipStreamEndCapture(cap, &b->graph);
  }
  {
    std::lock_guard<std::mutex> lk(c->mu);
    c->timing = timing;
  }
  if (st == TACAW_OK && e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
  (void)hipStreamDestroy(cap);
  if (st != TACAW_OK || e != hipSuccess) {
    if (st == TACAW_OK) {
      set_error("batch capture failed: %s", hipGetErrorString(e));
      st = TACAW_EDEVICE;
    }
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    delete b;
    return st;
  }
  for (int i = 0; i < n_jobs; ++i) {
    b->jobs.push_back(jobs[i]);
    b->buffers.push_back(job_buffers(jobs[i]));
  }
  *out = b;
  return TACAW_OK;
}

tacaw_status tacaw_batch_launch(tacaw_batch* b, void* hip_stream) {
  clear_error();
  if (!b) {
    set_error("batch is NULL");
    return TACAW_EINVAL;
  }
  tacaw_status st = check_batch(b->jobs.data(), (int)b->jobs.size());
  if (st != TACAW_OK) return st;
  for (size_t i = 0; i < b->jobs.size(); ++i) {
    const tacaw_job* j = b->jobs[i];
    if (!j->materialized || job_buffers(j) != b->buffers[i]) {
      set_error("job %zu's device buffers changed since the capture: capture the batch again", i);
      return TACAW_EINVAL;
    }
  }
  if (hipSetDevice(b->ctx->device) != hipSuccess) {
    set_error("hipSetDevice failed");
    return TACAW_EDEVICE;
  }
  hipStream_t s = (hipStream_t)hip_stream;
  const hipError_t e = hipGraphLaunch(b->exec, s);
  if (e != hipSuccess) {
    set_error("hipGraphLaunch: %s", hipGetErrorString(e));
    return TACAW_EDEVICE;
  }
  for (tacaw_job* j : b->jobs) {
    leave_serving_state(j);
    mark_all_present(j);
    j->has_result = true;
    j->last_stream = s;
  }
  return TACAW_OK;
}

tacaw_status tacaw_batch_destroy(tacaw_batch* b) {
  clear_error();
  if (!b) return TACAW_OK;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  delete b;
  return TACAW_OK;
}

tacaw_status tacaw_autotune(tacaw_job* job, void* hip_stream, int* row_variant, int* col_variant) {
  clear_error();
  if (!job) {
    set_error("job is NULL");
    return TACAW_EINVAL;
  }
  tacaw_ctx* c = job->ctx;
  if (hipSetDevice(c->device) != hipSuccess) {
    set_error("hipSetDevice failed");
    return TACAW_EDEVICE;
  }
  load_tune_cache(c);
  tacaw_status st = materialize(job, nullptr);
  if (st != TACAW_OK) return st;
  hipStream_t s = (hipStream_t)hip_stream;
  const HostPlan& hp = job->hp;
  const int fb = std::min(hp.fb, hp.F);
  // row variants: 0, 1 (LDS rows), 2, 3 (register FFT with one or two rows
  // in flight, grids 64-1024), 4 (six-step rows, nx 384);
  // column variants: 0, 1 (LDS columns), 2 (register FFT on 8-32 column
  // tiles, ny 64-1024), 3 (16-column tiles, ny 256 and 512), 5 (six-step on
  // 8-column tiles, ny 512), 6 (six-step on 16-column tiles, ny 512, nx a
  // multiple of 16), 7 (six-step on 16-column tiles, ny 256, nx a multiple
  // of 16), 8 (six-step on 8-column tiles, ny 384, nx a multiple of 8)
  auto reg = [](int n) { return n == 64 || n == 128 || n == 256 || n == 384 || n == 512 || n == 768 || n == 1024; };
  const int row_cand[5] = {0, 1, 2, 3, 4};
  const int col_cand_512[6] = {0, 1, 2, 3, 5, 6};
  const int col_cand_256[5] = {0, 1, 2, 3, 7};
  const int col_cand_384[4] = {0, 1, 2, 8};
  const int col_cand_other[3] = {0, 1, 2};
  const int* col_cand = hp.ny == 512   ? col_cand_512
                        : hp.ny == 256 ? col_cand_256
                        : hp.ny == 384 ? col_cand_384
                                       : col_cand_other;
  const int n_row_var = hp.nx == 384 ? 5 : reg(hp.nx) ? 4 : 2;
  const int n_col_var = hp.ny == 512                       ? (hp.nx % 16 == 0 ? 6 : 5)
                        : hp.ny == 256 && hp.nx % 16 == 0 ? 5
                        : hp.ny == 384 && hp.nx % 8 == 0  ? 4
                        : reg(hp.ny)                      ? 3
                                                          : 2;
  const int n_var = std::max(n_row_var, n_col_var);
  double best_row[6] = {1e30, 1e30, 1e30, 1e30, 1e30, 1e30}, best_col[6] = {1e30, 1e30, 1e30, 1e30, 1e30, 1e30};
  const bool was_timing = c->timing;
  for (int v = 0; v < n_var; ++v) {
    c->row_variant[hp.nx] = row_cand[std::min(v, n_row_var - 1)] + 1;
    c->col_variant[hp.ny] = col_cand[std::min(v, n_col_var - 1)] + 1;
    for (int rep = 0; rep < 2; ++rep) {   // first repetition warms up
      {
        std::lock_guard<std::mutex> lk(c->mu);
        c->timing = true;
        for (int i = 0; i < TACAW_K_COUNT; ++i) {
          c->total_ms[i] = 0;
          c->launches[i] = 0;
        }
      }
      st = run_batch_range(job, s, 0, fb);
      if (st != TACAW_OK) break;
      double row_ms = 0, col_ms = 0;
      int64_t n = 0;
      tacaw_timing_get(c, TACAW_K_ROW, &row_ms, &n);
      tacaw_timing_get(c, TACAW_K_COL, &col_ms, &n);
      if (v < n_row_var) best_row[v] = row_ms;
      if (v < n_col_var) best_col[v] = col_ms;
    }
    if (st != TACAW_OK) break;
  }
  {
    std::lock_guard<std::mutex> lk(c->mu);
    c->timing = was_timing;
  }
  if (st != TACAW_OK) return st;
  int rv = 0, cv = 0;
  for (int v = 1; v < n_row_var; ++v)
    if (best_row[v] < best_row[rv]) rv = v;
  for (int v = 1; v < n_col_var; ++v)
    if (best_col[v] < best_col[cv]) cv = v;
  rv = row_cand[rv];
  cv = col_cand[cv];
  c->row_variant[hp.nx] = rv + 1;
  c->col_variant[hp.ny] = cv + 1;
  if (row_variant) *row_variant = rv;
  if (col_variant) *col_variant = cv;
  if (!c->tune_cache.empty()) {
    std::ofstream out(c->tune_cache, std::ios::app);
    out << "{\"nx\": " << hp.nx << ", \"ny\": " << hp.ny << ", \"row_variant\": " << rv
        << ", \"col_variant\": " << cv << "}\n";
  }
  return TACAW_OK;
}

}  // extern "C"
