// Serving loop: admission by device-memory footprint and continuous batching.
//
// Submitted jobs wait in a queue.  The loop admits the first queued job, in
// submission order, whose footprint fits the context budget next to the jobs
// already resident and for which there is room, so a small job can pass a
// large one that does not fit yet.  A job that has waited longer than
// TACAW_SERVE_AGE_MS (default 1000 ms) at the head of the queue stops that:
// then only the head is admitted, as soon as it fits.  An admitted job is
// materialised (allocation, upload, tables) by a housekeeping thread, so
// allocation never stalls the issue of other jobs' work.
//
// Jobs whose frame batches are small (the batched executor's rule) join the
// lane group of their grid size: one stream per group, where each launch
// advances one frame batch of every member job by one slice (potentials,
// then the row and column passes of all lanes together), a finished frame
// batch makes room for the next one of any member, and jobs join as they are
// admitted and leave when their time stage is queued.  So slice steps of
// different requests share launches.  A new group can hold its first launch
// for a batching window (TACAW_SERVE_BATCH_WINDOW_MS) so that requests
// arriving together start together.  Up to four groups (grid sizes) run at
// once, with two iterations in flight each.
//
// Large jobs take one of four stream slots: each keeps one frame batch
// (potentials + all slice passes of fb frames) in flight, so batches of
// different requests overlap on the device.  When a job's last batch is done
// its time stage runs.
//
// When a job is over, its state is published at once (tacaw_wait returns);
// a release thread of its own then frees the working buffers, and only the
// spectrum (and, if kept, the exit waves) stays resident until the job is
// destroyed.  Materialisation runs on another thread, so a release never
// waits behind a large job's setup.  A job's result is computed by the same per-row and
// per-column arithmetic on the same frame batches as in the plain form, so it
// is bitwise the same alone or in any mix.
#include <stdlib.h>

#include <chrono>
#include <map>
#include <memory>
#include <set>

#include "runtime.h"

namespace tacaw {
tacaw_status materialize(tacaw_job* j, hipStream_t s);
void mark_all_present(tacaw_job* j);
void release_working(tacaw_job* j);
size_t resident_bytes_after_done(const tacaw_job* j);
tacaw_status run_batch_range(tacaw_job* job, hipStream_t s, int f_begin, int f_end);
tacaw_status run_time_stage(tacaw_job* job, hipStream_t s);
}  // namespace tacaw

using namespace tacaw;

namespace {

constexpr int kSlots = 4;  // concurrently running jobs (one stream each)

enum { ST_IDLE = 0, ST_QUEUED = 1, ST_RUNNING = 2, ST_DONE = 3, ST_CANCELLED = 4, ST_FAILED = 5 };

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

struct Slot {
  tacaw_job* job = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr;
  bool inflight = false;
  bool time_issued = false;
  std::atomic<int> setup{0};   // 0 none, 1 materialising, 2 ready, 3 failed
};

// One background thread for the slow host-side steps: materialising admitted
// jobs and releasing finished ones.
struct Housekeeper {
  std::mutex mu;
  std::condition_variable cv;
  std::deque<std::function<void()>> tasks;
  bool stop = false;
  std::thread th;
  void start(int device) {
    th = std::thread([this, device] {
      (void)hipSetDevice(device);
      for (;;) {
        std::function<void()> t;
        {
          std::unique_lock<std::mutex> lk(mu);
          cv.wait(lk, [&] { return stop || !tasks.empty(); });
          if (tasks.empty()) return;   // stop requested and nothing left
          t = std::move(tasks.front());
          tasks.pop_front();
        }
        t();
      }
    });
  }
  void post(std::function<void()> t) {
    {
      std::lock_guard<std::mutex> lk(mu);
      tasks.push_back(std::move(t));
    }
    cv.notify_one();
  }
  void join() {
    {
      std::lock_guard<std::mutex> lk(mu);
      stop = true;
    }
    cv.notify_one();
    if (th.joinable()) th.join();
  }
};

double age_limit_ms() {
  const char* e = getenv("TACAW_SERVE_AGE_MS");
  return e ? atof(e) : 1000.0;
}

// Batching window: a lane group that has issued nothing yet waits this long
// (TACAW_SERVE_BATCH_WINDOW_MS, default 0) after its first member is ready
// before its first launch, so that requests arriving together share launches
// from the start.
double batch_window_ms() {
  const char* e = getenv("TACAW_SERVE_BATCH_WINDOW_MS");
  return e ? std::max(0.0, atof(e)) : 0.0;
}

// A job's work is over (its stream has passed it): publish its final state at
// once, so that tacaw_wait returns without waiting for the frees, then hand
// the release of its working buffers to the release thread.  Until that has
// run, release_pending holds the job (destroy, resubmission and other runs
// wait for it); the results themselves (spectrum, kept exit waves) are not
// touched by the release.
void publish(tacaw_ctx* c, Housekeeper& hk_release, tacaw_job* j, int state) {
  j->t_done = now_ms();
  // buffers that do not outlive the job's end leave the job's fields here,
  // before the state is published, and are freed by the release thread
  float2* exit_free = nullptr;
  float* spec_free = nullptr;
  if (state == ST_DONE) {
    mark_all_present(j);
    j->has_result = true;
    j->last_stream = nullptr;
    if (!(j->desc.flags & TACAW_KEEP_EXIT_WAVES)) {
      exit_free = j->d_exit;
      j->d_exit = nullptr;
      j->present.clear();
    }
  } else {
    j->has_result = false;
    exit_free = j->d_exit;
    spec_free = j->d_spec;
    j->d_exit = nullptr;
    j->d_spec = nullptr;
    j->present.clear();
  }
  {
    std::lock_guard<std::mutex> lk(c->mu);
    j->release_pending = true;
    j->serve_state.store(state);
  }
  c->cv.notify_all();
  hk_release.post([c, j, state, exit_free, spec_free] {
    release_working(j);   // the working buffers; the job's results stay
    if (exit_free) (void)hipFree(exit_free);
    if (spec_free) (void)hipFree(spec_free);
    const size_t keep = state == ST_DONE ? resident_bytes_after_done(j) : 0;
    {
      std::lock_guard<std::mutex> lk(c->mu);
      c->resident -= j->fp.total();
      c->resident += keep;
      j->retained = keep;
      j->release_pending = false;
    }
    c->cv.notify_all();
  });
}

// The slot's job is over: wait for its stream, publish it and free the slot.
void finish(tacaw_ctx* c, Housekeeper& hk_release, Slot& s, int state) {
  tacaw_job* j = s.job;
  (void)hipStreamSynchronize(s.stream);
  publish(c, hk_release, j, state);
  s.job = nullptr;
  s.inflight = false;
  s.time_issued = false;
  s.setup.store(0);
}

// A lane group of the serving loop: its stream, the iterations in flight
// (each with the jobs whose work ended in it) and the admitted jobs still
// being materialised.
struct ServeGroup {
  struct Joining {
    tacaw_job* job;
    std::shared_ptr<std::atomic<int>> setup;   // 1 materialising, 2 ready, 3 failed
  };
  struct Iter {
    hipEvent_t ev;
    std::vector<tacaw_job*> ended;
  };
  LaneGroup lg;
  std::deque<Iter> inflight;
  std::vector<Joining> joining;
  std::set<tacaw_job*> cancelled;   // dropped members
  int64_t shared_seen = 0;
  double first_ready_ms = 0;        // when the group's first member became ready
  bool stepped = false;             // an iteration has been issued
  ServeGroup(tacaw_ctx* c, hipStream_t s, int nx, int ny) : lg(c, s, nx, ny, true) {}
  bool idle() const { return lg.left.empty() && inflight.empty() && joining.empty(); }
};

constexpr int kGroups = 4;   // grid sizes served in shared launches at once
constexpr int kGroupDepth = 2;   // iterations in flight per group

void server_main(tacaw_ctx* c) {
  (void)hipSetDevice(c->device);
  Slot slots[kSlots];
  for (auto& s : slots) {
    (void)hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking);
    (void)hipEventCreateWithFlags(&s.ev, hipEventDisableTiming);
  }
  std::vector<hipStream_t> free_group_streams;
  for (int i = 0; i < kGroups; ++i) {
    hipStream_t st = nullptr;
    (void)hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    free_group_streams.push_back(st);
  }
  std::map<std::pair<int, int>, std::unique_ptr<ServeGroup>> groups;
  // materialisation (slow for large jobs) and release run on threads of
  // their own, so a release never waits behind a large job's setup
  Housekeeper hk, hk_release;
  hk.start(c->device);
  hk_release.start(c->device);
  const double age_ms = age_limit_ms();
  const double window_ms = batch_window_ms();
  // a grouped job's work is over (its stream has passed it): publish it
  auto end_grouped = [&](tacaw_job* j, int state) {
    if (j->shared_launch) {
      std::lock_guard<std::mutex> lk(c->mu);
      c->serve_grouped_jobs += 1;
    }
    publish(c, hk_release, j, state);
  };
  for (;;) {
    bool progressed = false;
    {
      std::unique_lock<std::mutex> lk(c->mu);
      int busy = 0;
      for (auto& s : slots) busy += s.job != nullptr;
      busy += (int)groups.size();
      if (busy == 0 && c->queue.empty()) {
        if (c->stop) break;
        c->cv.wait(lk, [&] { return c->stop || !c->queue.empty(); });
        if (c->stop && c->queue.empty()) break;
      }
      // drop cancelled jobs that were never admitted
      for (auto it = c->queue.begin(); it != c->queue.end();) {
        if ((*it)->cancel_req.load() || c->stop) {
          (*it)->t_done = now_ms();
          (*it)->serve_state.store(ST_CANCELLED);
          it = c->queue.erase(it);
          progressed = true;
        } else {
          ++it;
        }
      }
    }
    if (progressed) c->cv.notify_all();
    // admission: the first queued job that fits and has room (its grid's
    // group, a free group stream, or a free slot), unless the head has aged
    // past the limit, in which case only the head
    for (;;) {
      tacaw_job* j = nullptr;
      bool grouped = false;
      Slot* slot = nullptr;
      for (auto& s : slots)
        if (!s.job) {
          slot = &s;
          break;
        }
      {
        std::lock_guard<std::mutex> lk(c->mu);
        if (c->queue.empty()) break;
        const bool head_only = now_ms() - c->queue.front()->t_submit > age_ms;
        for (auto it = c->queue.begin(); it != c->queue.end(); ++it) {
          tacaw_job* cand = *it;
          const bool small = shares_launches(cand);
          const bool room = small ? (groups.count({cand->hp.nx, cand->hp.ny}) > 0 || !free_group_streams.empty())
                                  : slot != nullptr;
          if (room && c->resident + cand->fp.total() <= c->budget) {
            j = cand;
            grouped = small;
            c->queue.erase(it);
            break;
          }
          if (head_only) break;
        }
        if (!j) break;
        c->resident += j->fp.total();
      }
      j->t_admit = now_ms();
      j->next_frame = 0;
      progressed = true;
      if (grouped) {
        auto key = std::make_pair(j->hp.nx, j->hp.ny);
        auto g = groups.find(key);
        if (g == groups.end()) {
          hipStream_t st = free_group_streams.back();
          free_group_streams.pop_back();
          g = groups.emplace(key, std::make_unique<ServeGroup>(c, st, j->hp.nx, j->hp.ny)).first;
        }
        auto setup = std::make_shared<std::atomic<int>>(1);
        g->second->joining.push_back({j, setup});
        // materialised on the housekeeper's own (null) stream, synchronously
        hk.post([j, setup] { setup->store(materialize(j, nullptr) == TACAW_OK ? 2 : 3); });
      } else {
        slot->job = j;
        slot->setup.store(1);
        hk.post([j, slot] { slot->setup.store(materialize(j, slot->stream) == TACAW_OK ? 2 : 3); });
      }
    }
    // lane groups: join ready jobs, drop cancelled ones, retire finished
    // iterations, issue the next
    for (auto it = groups.begin(); it != groups.end();) {
      ServeGroup& g = *it->second;
      for (size_t k = 0; k < g.joining.size();) {
        const int st = g.joining[k].setup->load();
        tacaw_job* j = g.joining[k].job;
        if (st == 1) {
          ++k;
          continue;
        }
        g.joining.erase(g.joining.begin() + k);
        if (st == 3) {
          end_grouped(j, ST_FAILED);
        } else {
          j->serve_state.store(ST_RUNNING);
          if (!g.stepped && g.lg.left.empty()) g.first_ready_ms = now_ms();
          g.lg.add(j);
        }
        progressed = true;
      }
      std::vector<tacaw_job*> members;
      for (auto& kv : g.lg.left) members.push_back(kv.first);
      for (tacaw_job* j : members) {
        if (!(j->cancel_req.load() || c->stop) || g.cancelled.count(j)) continue;
        g.cancelled.insert(j);
        if (g.lg.drop(j)) {
          // nothing of it in flight beyond what the stream already holds
          hipEvent_t ev = nullptr;
          (void)hipEventCreateWithFlags(&ev, hipEventDisableTiming);
          (void)hipEventRecord(ev, g.lg.s);
          g.inflight.push_back({ev, {j}});
        }
        progressed = true;
      }
      while (!g.inflight.empty() && hipEventQuery(g.inflight.front().ev) == hipSuccess) {
        for (tacaw_job* j : g.inflight.front().ended) {
          const bool cancelled = g.cancelled.erase(j) > 0;
          end_grouped(j, cancelled ? ST_CANCELLED : ST_DONE);
        }
        (void)hipEventDestroy(g.inflight.front().ev);
        g.inflight.pop_front();
        progressed = true;
      }
      // a new group waits up to the batching window after its first member
      // is ready, so that requests arriving together start together
      const bool window_open = !g.stepped && !c->stop && now_ms() - g.first_ready_ms < window_ms;
      if (!g.lg.done() && (int)g.inflight.size() < kGroupDepth && !window_open) {
        g.stepped = true;
        std::vector<tacaw_job*> ended;
        tacaw_status st = g.lg.step(&ended);
        if (st != TACAW_OK) {
          // the group's stream state is unknown: wait for it, fail its jobs
          (void)hipStreamSynchronize(g.lg.s);
          for (auto& f : g.inflight) {
            for (tacaw_job* j : f.ended) end_grouped(j, ST_FAILED);
            (void)hipEventDestroy(f.ev);
          }
          g.inflight.clear();
          for (auto& kv : g.lg.left) end_grouped(kv.first, ST_FAILED);
          for (tacaw_job* j : ended) end_grouped(j, ST_FAILED);
          g.lg.left.clear();
          g.lg.pending.clear();
          g.lg.active.clear();
        } else {
          hipEvent_t ev = nullptr;
          (void)hipEventCreateWithFlags(&ev, hipEventDisableTiming);
          (void)hipEventRecord(ev, g.lg.s);
          g.inflight.push_back({ev, std::move(ended)});
          std::lock_guard<std::mutex> lk(c->mu);
          c->serve_shared_launches += g.lg.shared_launches - g.shared_seen;
          g.shared_seen = g.lg.shared_launches;
        }
        progressed = true;
      }
      if (g.idle()) {
        free_group_streams.push_back(g.lg.s);
        it = groups.erase(it);
        progressed = true;
      } else {
        ++it;
      }
    }
    // stream slots: issue / retire work
    for (auto& s : slots) {
      tacaw_job* j = s.job;
      if (!j) continue;
      const int setup = s.setup.load();
      if (setup == 1) continue;   // still being materialised
      if (setup == 3) {
        finish(c, hk_release, s, ST_FAILED);
        progressed = true;
        continue;
      }
      if (j->serve_state.load() == ST_QUEUED) j->serve_state.store(ST_RUNNING);
      if (s.inflight) {
        if (hipEventQuery(s.ev) != hipSuccess) continue;
        s.inflight = false;
        progressed = true;
      }
      if (j->cancel_req.load() || c->stop) {
        finish(c, hk_release, s, ST_CANCELLED);
        progressed = true;
        continue;
      }
      tacaw_status st = TACAW_OK;
      if (j->next_frame < j->hp.F) {
        const int f1 = std::min(j->hp.F, j->next_frame + j->hp.fb);
        st = run_batch_range(j, s.stream, j->next_frame, f1);
        j->next_frame = f1;
      } else if (!s.time_issued) {
        st = run_time_stage(j, s.stream);
        s.time_issued = true;
      } else {
        finish(c, hk_release, s, ST_DONE);
        progressed = true;
        continue;
      }
      if (st != TACAW_OK) {
        finish(c, hk_release, s, ST_FAILED);
        continue;
      }
      (void)hipEventRecord(s.ev, s.stream);
      s.inflight = true;
      progressed = true;
    }
    if (!progressed) std::this_thread::sleep_for(std::chrono::microseconds(50));
  }
  for (auto& s : slots) {
    if (s.job) {
      while (s.setup.load() == 1) std::this_thread::sleep_for(std::chrono::microseconds(50));
      finish(c, hk_release, s, ST_CANCELLED);
    }
  }
  hk.join();           // every posted setup has run
  hk_release.join();   // and every release
  for (auto& s : slots) {
    (void)hipEventDestroy(s.ev);
    (void)hipStreamDestroy(s.stream);
  }
  for (hipStream_t st : free_group_streams) (void)hipStreamDestroy(st);
}

}  // namespace

extern "C" {

void tacaw_serve_shutdown(tacaw_ctx* c) {
  {
    std::lock_guard<std::mutex> lk(c->mu);
    if (!c->server_started) return;
    c->stop = true;
  }
  c->cv.notify_all();
  if (c->server.joinable()) c->server.join();
  c->server_started = false;
}

tacaw_status tacaw_submit(tacaw_ctx* c, tacaw_job* j) {
  clear_error();
  if (!c || !j) {
    set_error("ctx and job must not be NULL");
    return TACAW_EINVAL;
  }
  if (j->ctx != c) {
    set_error("job belongs to another context");
    return TACAW_EINVAL;
  }
  const int st = j->serve_state.load();
  if (st == ST_QUEUED || st == ST_RUNNING) {
    set_error("job is already in the serving loop");
    return TACAW_EBUSY;
  }
  if (j->fp.total() > c->budget) {
    set_error("job footprint %.3f GiB can never fit the budget %.3f GiB", j->fp.total() / 1073741824.0,
              c->budget / 1073741824.0);
    return TACAW_ENOMEM;
  }
  wait_released(j);   // a job served before is fully released first
  std::lock_guard<std::mutex> lk(c->mu);
  if (c->stop) {
    set_error("context is shutting down");
    return TACAW_EINVAL;
  }
  // a job that was run or served before gives its retained memory back first
  if (j->retained) {
    c->resident -= j->retained;
    j->retained = 0;
  }
  if (j->materialized || j->d_exit || j->d_spec) {
    // plain-form buffers are not accounted; release them so admission allocates
    (void)hipDeviceSynchronize();
    release_working(j);
    if (j->d_exit) (void)hipFree(j->d_exit);
    if (j->d_spec) (void)hipFree(j->d_spec);
    j->d_exit = nullptr;
    j->d_spec = nullptr;
  }
  j->has_result = false;
  j->cancel_req.store(false);
  j->t_submit = now_ms();
  j->t_admit = j->t_done = 0;
  j->served = true;
  j->shared_launch = false;
  j->serve_state.store(ST_QUEUED);
  c->queue.push_back(j);
  if (!c->server_started) {
    c->stop = false;
    c->server = std::thread(server_main, c);
    c->server_started = true;
  }
  c->cv.notify_all();
  return TACAW_OK;
}

tacaw_status tacaw_poll(tacaw_job* j, int* done) {
  clear_error();
  if (!j || !done) {
    set_error("job and done must not be NULL");
    return TACAW_EINVAL;
  }
  const int st = j->serve_state.load();
  *done = (st == ST_DONE || st == ST_CANCELLED || st == ST_FAILED) ? 1 : 0;
  return TACAW_OK;
}

tacaw_status tacaw_wait(tacaw_job* j) {
  clear_error();
  if (!j) {
    set_error("job is NULL");
    return TACAW_EINVAL;
  }
  tacaw_ctx* c = j->ctx;
  std::unique_lock<std::mutex> lk(c->mu);
  c->cv.wait(lk, [&] {
    const int st = j->serve_state.load();
    return st != ST_QUEUED && st != ST_RUNNING;
  });
  const int st = j->serve_state.load();
  if (st == ST_CANCELLED) {
    set_error("job was cancelled");
    return TACAW_ECANCELLED;
  }
  if (st == ST_FAILED) {
    set_error("job failed on the device");
    return TACAW_EDEVICE;
  }
  if (st == ST_IDLE) {
    set_error("job was never submitted");
    return TACAW_EINVAL;
  }
  return TACAW_OK;
}

tacaw_status tacaw_cancel(tacaw_job* j) {
  clear_error();
  if (!j) {
    set_error("job is NULL");
    return TACAW_EINVAL;
  }
  j->cancel_req.store(true);
  j->ctx->cv.notify_all();
  return TACAW_OK;
}

tacaw_status tacaw_serve_stats(tacaw_ctx* c, int64_t* shared_launches, int64_t* grouped_jobs) {
  clear_error();
  if (!c) {
    set_error("ctx is NULL");
    return TACAW_EINVAL;
  }
  std::lock_guard<std::mutex> lk(c->mu);
  if (shared_launches) *shared_launches = c->serve_shared_launches;
  if (grouped_jobs) *grouped_jobs = c->serve_grouped_jobs;
  return TACAW_OK;
}

tacaw_status tacaw_job_latency(const tacaw_job* j, double* queued_ms, double* total_ms) {
  clear_error();
  if (!j) {
    set_error("job is NULL");
    return TACAW_EINVAL;
  }
  const int st = j->serve_state.load();
  if (st != ST_DONE && st != ST_CANCELLED && st != ST_FAILED) {
    set_error("job has not finished in the serving loop");
    return TACAW_ENOTREADY;
  }
  if (queued_ms) *queued_ms = (j->t_admit > 0 ? j->t_admit : j->t_done) - j->t_submit;
  if (total_ms) *total_ms = j->t_done - j->t_submit;
  return TACAW_OK;
}

}  // extern "C"
