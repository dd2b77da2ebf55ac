// Serving loop: admission by device-memory footprint and continuous batching.
//
// Submitted jobs wait in a queue.  When a stream slot is free, the loop
// admits the first queued job, in submission order, whose footprint fits the
// context budget next to the jobs already resident, so a small job can pass a
// large one that does not fit yet.  A job that has waited longer than
// TACAW_SERVE_AGE_MS (default 1000 ms) at the head of the queue stops that:
// then only the head is admitted, as soon as it fits.  An admitted job is
// materialised (allocation, upload, tables) by a housekeeping thread on its
// slot's stream, so allocation never stalls the issue of other jobs' work;
// from then on the loop interleaves frame batches of every running job: each
// running job owns a non-blocking stream and keeps one frame batch
// (potentials + all slice passes of fb frames) in flight, so batches of
// different requests overlap on the device.  When a job's last batch is done
// its time stage runs; then the housekeeping thread frees its working buffers
// and only the spectrum (and, if kept, the exit waves) stays resident until
// the job is destroyed.  A job's result is computed by the same kernels on the
// same frame batches as in the plain form, so it is bitwise the same alone or
// in any mix.
#include <stdlib.h>

#include <chrono>

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

// Release a finished, cancelled or failed job's device memory and publish its
// final state (runs on the housekeeping thread; the job's stream is idle).
void release(tacaw_ctx* c, tacaw_job* j, int state) {
  size_t keep = 0;
  if (state == ST_DONE) {
    mark_all_present(j);
    j->has_result = true;
    j->last_stream = nullptr;
    release_working(j);
    keep = resident_bytes_after_done(j);
  } else {
    release_working(j);
    if (j->d_exit) (void)hipFree(j->d_exit);
    if (j->d_spec) (void)hipFree(j->d_spec);
    j->d_exit = nullptr;
    j->d_spec = nullptr;
    j->has_result = false;
  }
  {
    std::lock_guard<std::mutex> lk(c->mu);
    c->resident -= j->fp.total();
    c->resident += keep;
    j->retained = keep;
    j->serve_state.store(state);
  }
  c->cv.notify_all();
}

// The slot's job is over: wait for its stream, stamp the end, hand the
// release to the housekeeper and free the slot.
void finish(tacaw_ctx* c, Housekeeper& hk, Slot& s, int state) {
  tacaw_job* j = s.job;
  (void)hipStreamSynchronize(s.stream);
  j->t_done = now_ms();
  hk.post([c, j, state] { release(c, j, state); });
  s.job = nullptr;
  s.inflight = false;
  s.time_issued = false;
  s.setup.store(0);
}

void server_main(tacaw_ctx* c) {
  (void)hipSetDevice(c->device);
  Slot slots[kSlots];
  for (auto& s : slots) {
    (void)hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking);
    (void)hipEventCreateWithFlags(&s.ev, hipEventDisableTiming);
  }
  Housekeeper hk;
  hk.start(c->device);
  const double age_ms = age_limit_ms();
  for (;;) {
    bool progressed = false;
    {
      std::unique_lock<std::mutex> lk(c->mu);
      int busy = 0;
      for (auto& s : slots) busy += s.job != nullptr;
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
    // admission: the first queued job that fits, unless the head has aged
    // past the limit, in which case only the head
    for (auto& s : slots) {
      if (s.job) continue;
      tacaw_job* j = nullptr;
      {
        std::lock_guard<std::mutex> lk(c->mu);
        if (c->queue.empty()) break;
        const bool head_only = now_ms() - c->queue.front()->t_submit > age_ms;
        for (auto it = c->queue.begin(); it != c->queue.end(); ++it) {
          if (c->resident + (*it)->fp.total() <= c->budget) {
            j = *it;
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
      s.job = j;
      s.setup.store(1);
      Slot* sp = &s;
      hk.post([j, sp] { sp->setup.store(materialize(j, sp->stream) == TACAW_OK ? 2 : 3); });
      progressed = true;
    }
    // issue / retire work
    for (auto& s : slots) {
      tacaw_job* j = s.job;
      if (!j) continue;
      const int setup = s.setup.load();
      if (setup == 1) continue;   // still being materialised
      if (setup == 3) {
        finish(c, hk, s, ST_FAILED);
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
        finish(c, hk, s, ST_CANCELLED);
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
        finish(c, hk, s, ST_DONE);
        progressed = true;
        continue;
      }
      if (st != TACAW_OK) {
        finish(c, hk, s, ST_FAILED);
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
      finish(c, hk, s, ST_CANCELLED);
    }
  }
  hk.join();   // every posted setup and release has run
  for (auto& s : slots) {
    (void)hipEventDestroy(s.ev);
    (void)hipStreamDestroy(s.stream);
  }
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
