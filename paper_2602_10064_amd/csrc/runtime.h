// Host runtime of libtacaw: context, job, planner.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <condition_variable>
#include <deque>
#include <functional>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "tacaw.h"
#include "tacaw_internal.h"

struct tacaw_ctx;
struct tacaw_job;

namespace tacaw {

void set_error(const char* fmt, ...);
void clear_error();

// Everything the planner derives on the host from a job description and its
// inputs (FP64), ready to upload.
struct HostPlan {
  int nx = 0, ny = 0, pnx = 0, pny = 0, ns = 0, F = 0, P = 0, A = 0, S = 0, M = 0;
  bool plane = true, windowed = false, two_sided = false;
  double lx = 0, ly = 0, lz = 0, dx = 0, dy = 0, dz = 0, lam = 0, sigma = 0, alpha = 0, rc = 0;
  float rcx = 0, rcy = 0;
  int img_x = 0, img_y = 0, tiles_x = 0, tiles_y = 0;
  int fb = 1;                          // frames per batch
  bool splat_per_slice = true;         // potentials built slice by slice
  bool overlap = true;                 // per-slice potentials built one slice ahead on a side stream
  int splat_group = 1;                 // slices per potential launch (all slices when !splat_per_slice)
  std::vector<int32_t> slice_of;       // per input atom (frame-mean z)
  bool instant_z = false;              // TACAW_SLICE_BY_INSTANT_Z
  std::vector<int16_t> fslice;         // [F][A] sorted order: each frame's own slice (instant_z)
  std::vector<int32_t> order;          // sorted position -> input atom
  std::vector<int32_t> tile_start;     // [ns * tiles + 1]
  std::vector<int32_t> tile_atoms;     // sorted-atom indices
  std::vector<float> coef;             // [S][5][3]
  std::vector<int32_t> sorted_species; // [A]
  std::vector<int32_t> origin;         // [P][2] wrapped window origin
  std::vector<double> rloc;            // [P][2] probe position relative to the window
  // reciprocal-space potential route (kspace_coef given)
  bool kspace = false;
  int kgroup = 0;                      // slices per structure-factor launch (even unless all slices)
  std::vector<int32_t> ks_start;       // [ns * S + 1] CSR offsets per (slice, species)
  std::vector<int32_t> ks_atoms;       // sorted-atom indices
  std::vector<float> kcoef;            // [S][12] (a, c times C/A; d times log2 e)
};

// Device bytes of each buffer of a job.
struct Footprint {
  size_t exit = 0, spec = 0, V = 0, W = 0, pos = 0, tiles = 0, probes = 0, tables = 0;
  size_t total() const { return exit + spec + V + W + pos + tiles + probes + tables; }
};

tacaw_status validate_desc(const tacaw_job_desc* d);
int choose_frame_batch(const tacaw_job_desc* d);
bool splat_per_slice();
bool overlap_splat();
int splat_group(int n_slices, int fb, int pnx, int pny);
int kspace_group(int n_slices, int fb, int pnx, int pny);
Footprint footprint_of(const tacaw_job_desc* d, int fb, size_t n_tile_atoms_estimate);
double wavelength_A(double volt);
double sigma_rad_per_VA(double volt);
tacaw_status plan_job(const tacaw_job_desc* d, const int32_t* atom_species, const double* positions,
                      HostPlan& hp);

struct TimingRecord {
  int cls;
  hipEvent_t start, stop;
};

struct JobState;

// Launch through the timing wrapper (HIP events around the launch when the
// context's timing is on).
tacaw_status timed_launch(tacaw_ctx* c, int cls, hipStream_t s, const std::function<hipError_t()>& launch);
PassArgs pass_args(tacaw_job* j);
bool resident_for(const tacaw_job* j);
ResLane res_lane(tacaw_job* j, int f0, int fb, int sl, int n, int v_slices, int v_slice0);
int row_variant_for(tacaw_ctx* c, int n);
int col_variant_for(tacaw_ctx* c, int n);
tacaw_status materialize(tacaw_job* j, hipStream_t s);
tacaw_status run_batch_range(tacaw_job* job, hipStream_t s, int f_begin, int f_end);
tacaw_status run_time_stage(tacaw_job* job, hipStream_t s);

// Continuous lane batching of same-grid jobs on one stream (batch.cpp): a
// lane is one frame batch of one job at its own slice; each step launches the
// potentials of lanes that start a slice group, then one row and one column
// pass over every active lane, and the time stage of each job whose last frame
// batch it finished.  Used by the batched executor and by the serving loop,
// which adds jobs as they are admitted.
struct LaneGroup {
  struct Lane {
    tacaw_job* job;
    int f0, fb, slice;
  };
  tacaw_ctx* c = nullptr;
  hipStream_t s = nullptr;
  bool serving = false;   // results are published by the serving loop, not here
  std::deque<Lane> pending;
  std::vector<Lane> active;
  std::map<tacaw_job*, int> left;   // frame batches not finished per job
  std::set<tacaw_job*> dropped;     // cancelled jobs whose lane is still in flight
  int rv = 0, cv = 0;
  int64_t shared_launches = 0;      // pass launches that served more than one job

  LaneGroup(tacaw_ctx* ctx, hipStream_t stream, int nx, int ny, bool serving);
  void add(tacaw_job* j);           // queue every frame batch of j
  bool has(const tacaw_job* j) const;
  // Remove j's queued frame batches.  True when nothing of j is in flight;
  // otherwise its lane ends with the batch in flight (no time stage) and
  // step() reports it among the finished jobs.
  bool drop(tacaw_job* j);
  bool done() const { return pending.empty() && active.empty(); }
  // One iteration; jobs whose work ended in it (time stage enqueued, or
  // dropped) are appended to *finished.
  tacaw_status step(std::vector<tacaw_job*>* finished);
};

// Whether a job shares pass launches with other jobs of its grid in the
// batched executor and the serving loop (else it runs as in the plain form).
bool shares_launches(const tacaw_job* j);
void load_tune_cache(tacaw_ctx* c);

struct tacaw_ctx_impl;

// Spectrum analysis helpers (analysis.cpp): the job must hold a spectrum; the
// kept frequency bin nearest to f; the unshifted kx then ky axes of the wave
// grid (fftfreq order).
tacaw_status check_ready(const tacaw_job* job);
tacaw_status nearest_bin(const tacaw_job* job, double f, int* m_out);
std::vector<double> k_axes(const HostPlan& hp);

// Device address of the allocation-free entry points' fixed scratch array on
// `device` (noalloc.hip); looked up once per device with that device current.
tacaw_status noalloc_init(int device);

}  // namespace tacaw

struct tacaw_ctx {
  int device = 0;
  size_t budget = 0;
  std::mutex mu;
  size_t resident = 0;           // bytes held by jobs admitted by the serving loop
  // timing
  bool timing = false;
  unsigned timing_mask = ~0u;    // kernel classes timed with events while timing
  int timing_every = 1;          // time one launch in this many of each selected class
  int64_t launch_seq[TACAW_K_COUNT] = {0};
  std::vector<tacaw::TimingRecord> records;
  std::vector<hipEvent_t> event_pool;
  double total_ms[TACAW_K_COUNT] = {0};
  int64_t launches[TACAW_K_COUNT] = {0};
  // serving loop
  std::thread server;
  std::condition_variable cv;
  std::deque<tacaw_job*> queue;  // submitted, not yet admitted
  std::vector<tacaw_job*> active;
  bool stop = false;
  bool server_started = false;
  hipStream_t serve_stream = nullptr;
  int64_t serve_shared_launches = 0;   // pass launches of the serving loop that served several jobs
  int64_t serve_grouped_jobs = 0;      // served jobs that shared at least one launch with another job
  // batched executor and autotuner
  hipStream_t batch_streams[4] = {nullptr, nullptr, nullptr, nullptr};
  int row_variant[2048] = {0};   // by grid size: 0 untuned (use 1), else variant + 1
  int col_variant[2048] = {0};
  std::string tune_cache;        // JSON-lines file of tuned variants ("" -> none)
  bool tune_loaded = false;
};

struct tacaw_job {
  tacaw_ctx* ctx = nullptr;
  tacaw_job_desc desc{};
  std::vector<double> probe_xy;
  std::vector<int32_t> species_Z;
  std::vector<double> gauss_a, gauss_b;
  std::vector<double> kspace_coef;   // n_species x 12, or empty
  tacaw::HostPlan hp;
  tacaw::Footprint fp;
  // device buffers
  float2* d_exit = nullptr;
  float* d_spec = nullptr;
  float* d_V = nullptr;
  tacaw::AtomPos* d_pos = nullptr;
  int32_t* d_species = nullptr;
  int32_t* d_tile_start = nullptr;
  int32_t* d_tile_atoms = nullptr;
  float* d_coef = nullptr;
  float2* d_tw_x = nullptr;
  float2* d_tw_y = nullptr;
  float2* d_tw_t = nullptr;
  float2* d_px = nullptr;        // regular slices
  float2* d_py = nullptr;
  float2* d_px_last = nullptr;   // last slice
  float2* d_py_last = nullptr;
  float2* d_probe0 = nullptr;
  tacaw::Aberrations aberr{};    // probe aberrations (off unless set)
  int32_t* d_origin = nullptr;
  int16_t* d_fslice = nullptr;   // [F][A] per-frame slices (instant-z binning only)
  // reciprocal-space potential route
  float2* d_W = nullptr;         // [fb][kgroup/2 rounded up][pny][pnx] structure factors of slice pairs
  int32_t* d_ks_start = nullptr;
  int32_t* d_ks_atoms = nullptr;
  float* d_kcoef = nullptr;
  float2* d_tw_px = nullptr;     // potential-grid twiddles (windowed jobs; else the wave grid's)
  float2* d_tw_py = nullptr;
  double* d_rloc = nullptr;
  int* d_count = nullptr;
  std::vector<tacaw::AtomPos> enc;   // encoded positions, kept until the device copy exists
  bool materialized = false;
  hipStream_t last_stream = nullptr;
  // side stream and events of the overlapped potential pipeline
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_splat[2] = {nullptr, nullptr}, ev_row[2] = {nullptr, nullptr};
  bool has_result = false;
  // frames whose exit waves the store holds from tacaw_run_frames or
  // tacaw_put_exit_frames (one flag per frame), for tacaw_finish
  std::vector<uint8_t> present;
  // HIP-graph replay of the whole launch sequence (TACAW_USE_GRAPH)
  hipStream_t capture_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  // serving state
  std::atomic<int> serve_state{0};   // 0 idle, 1 queued, 2 running, 3 done, 4 cancelled, 5 failed
  std::atomic<bool> cancel_req{false};
  int next_frame = 0;                // serving: next frame batch start
  int next_slice = 0;
  double t_submit = 0, t_admit = 0, t_done = 0;
  size_t retained = 0;               // bytes counted in ctx->resident after a served job ends
  bool served = false;
  // served: ran in at least one pass launch together with another job
  bool shared_launch = false;
  // the serving loop has published this job's end but its release thread
  // has not yet freed the working buffers (guarded by ctx->mu)
  bool release_pending = false;
};

// Wait until the serving loop's release thread is done with the job.
inline void wait_released(tacaw_job* j) {
  std::unique_lock<std::mutex> lk(j->ctx->mu);
  j->ctx->cv.wait(lk, [&] { return !j->release_pending; });
}

// A plain, batched or frame-range run takes a job back from a finished,
// cancelled or failed serving state to idle, so the results of that run are
// not reported as cancelled or failed.  Queued and running jobs are left alone
// (the callers refuse them first).
inline void leave_serving_state(tacaw_job* j) {
  wait_released(j);
  int s = j->serve_state.load();
  while (s >= 3 && !j->serve_state.compare_exchange_weak(s, 0)) {
  }
}
