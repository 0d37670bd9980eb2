// The serving scheduler, independent of the device: requests (jobs) are
// queued in FIFO order, admitted while their device-memory share fits the
// budget (first-fit ranges of an arena of exactly that size) and a request
// slot is free, and handed to an executor in steps of up to max_step_jobs
// jobs, one step per executor stream at a time.  A completion thread polls
// the executor's streams, delivers each finished job's results, releases its
// memory and wakes the scheduler.  Completed tickets stay queryable up to
// keep_done of them; latency percentiles cover the last lat_window
// completions.
//
// The executor interface is what the library's device executor (HIP streams,
// staging and persistent kernels) implements; host tests drive the same
// scheduler with a CPU executor, so admission, memory accounting, slot
// reuse, ordering and failure handling are checked without a device.  Plain
// C++17: no device code, no HIP headers.
#pragma once

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <cstdio>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "tsqbx.h"
#include "tsqbx_arena.h"

namespace tsqbx {

inline double sched_now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// One request as the scheduler sees it; executors derive their request type
// from it.
struct Job {
  virtual ~Job() = default;
  uint64_t ticket = 0;
  size_t bytes = 0;        // device-memory share reserved while admitted
  size_t arena_off = 0;    // its range in the arena: [arena_off, arena_off + bytes)
  int64_t pair_terms = 0;  // credited to the statistics on success
  double t_submit = 0, t_launch = 0, t_done = 0;
  int status = TSQBX_OK;
  bool done = false;
  int waiters = 0;  // threads blocked in wait() on it
};

class Executor {
 public:
  virtual ~Executor() = default;
  // Steps that can be in flight at once (one per stream).
  virtual int streams() const = 0;
  // Called first on the scheduler's and the completion thread.
  virtual void thread_start() {}
  // Start a step of jobs on a free stream; TSQBX_OK, or an error status (err
  // says why) after which the step's jobs fail.
  virtual int launch(int stream, const std::vector<Job *> &jobs, std::string &err) = 0;
  // A launched step: 1 finished, 0 still running, an error status if failed.
  virtual int query(int stream) = 0;
  // Block until whatever a failed launch left running on the stream ends.
  virtual void sync(int stream) = 0;
  // Deliver a job of a finished step (step_status: TSQBX_OK or the step's
  // error); returns the job's final status.
  virtual int finish(Job *job, int step_status) = 0;
  // Drop the job's host-side data; called once for every job that ends
  // (completed, failed, refused or cancelled), before it is forgotten.
  virtual void release(Job *job) = 0;
};

struct SchedLimits {
  size_t budget = 0;
  int max_slots = 1;
  int max_step_jobs = 32;
  size_t keep_done = 4096;
  size_t lat_window = 65536;
};

class Scheduler {
 public:
  Scheduler(Executor *ex, const SchedLimits &lim) : ex_(ex), lim_(lim) {
    arena_.init(lim.budget);
    busy_stream_.assign(std::max(ex->streams(), 1), 0);
    st_.budget_bytes = lim.budget;
  }
  Scheduler(const Scheduler &) = delete;
  Scheduler &operator=(const Scheduler &) = delete;
  ~Scheduler() {
    stop();
    for (auto &kv : all_) delete kv.second;
  }

  void start() {
    sched_ = std::thread([this] { scheduler(); });
    comp_ = std::thread([this] { completer(); });
  }

  // Queue a job (the scheduler owns it from here on).  TSQBX_E_STATE once
  // stopping, TSQBX_E_BUDGET when it can never fit; the job is then released
  // and deleted.
  int submit(Job *j, uint64_t *ticket) {
    std::lock_guard<std::mutex> lk(mu_);
    ++st_.submitted;
    int rc = TSQBX_OK;
    if (stopping_) {
      rc = TSQBX_E_STATE;
    } else if (j->bytes > lim_.budget) {
      ++st_.rejected;
      rc = TSQBX_E_BUDGET;
    }
    if (rc != TSQBX_OK) {
      ex_->release(j);
      delete j;
      return rc;
    }
    j->ticket = next_ticket_++;
    j->t_submit = sched_now_s();
    all_[j->ticket] = j;
    queue_.push_back(j);
    *ticket = j->ticket;
    cv_sched_.notify_all();
    return TSQBX_OK;
  }

  // Withdraw a queued job: it ends with TSQBX_E_CANCELED.  TSQBX_E_INVALID
  // for an unknown ticket, TSQBX_E_STATE once it has been admitted.
  int cancel(uint64_t ticket) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = all_.find(ticket);
    if (it == all_.end()) return TSQBX_E_INVALID;
    Job *j = it->second;
    auto q = std::find(queue_.begin(), queue_.end(), j);
    if (q == queue_.end()) return TSQBX_E_STATE;
    queue_.erase(q);
    j->status = TSQBX_E_CANCELED;
    j->done = true;
    j->t_launch = j->t_done = sched_now_s();
    ++st_.failed;
    ex_->release(j);
    retire(j, false);
    cv_done_.notify_all();
    cv_sched_.notify_all();
    return TSQBX_OK;
  }

  // *done and the job's *status; TSQBX_E_INVALID for an unknown ticket.
  int poll(uint64_t ticket, int *done, int *status) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = all_.find(ticket);
    if (it == all_.end()) return TSQBX_E_INVALID;
    *done = it->second->done ? 1 : 0;
    *status = it->second->done ? it->second->status : TSQBX_OK;
    return TSQBX_OK;
  }

  // TSQBX_E_INVALID for an unknown ticket, TSQBX_E_TIMEOUT if not done in
  // time; else TSQBX_OK with the job's *status.
  int wait(uint64_t ticket, double timeout_s, int *status) {
    std::unique_lock<std::mutex> lk(mu_);
    auto it = all_.find(ticket);
    if (it == all_.end()) return TSQBX_E_INVALID;
    Job *j = it->second;
    ++j->waiters;  // keeps j from being forgotten while this thread waits
    const bool ok =
        cv_done_.wait_for(lk, std::chrono::duration<double>(timeout_s), [&] { return j->done; });
    --j->waiters;
    if (!ok) return TSQBX_E_TIMEOUT;
    *status = j->status;
    return TSQBX_OK;
  }

  int drain(double timeout_s) {
    std::unique_lock<std::mutex> lk(mu_);
    return cv_done_.wait_for(lk, std::chrono::duration<double>(timeout_s),
                             [&] { return queue_.empty() && jobs_in_flight_ == 0; })
               ? TSQBX_OK
               : TSQBX_E_TIMEOUT;
  }

  void stats(tsqbx_server_stats *out) {
    std::lock_guard<std::mutex> lk(mu_);
    *out = st_;
    out->bytes_in_flight = bytes_in_flight_;
    out->peak_bytes_in_flight = peak_bytes_;
    out->latency_p50_ms = percentile(lat_ms_, 0.50);
    out->latency_p90_ms = percentile(lat_ms_, 0.90);
    out->latency_p99_ms = percentile(lat_ms_, 0.99);
    out->latency_max_ms = lat_ms_.empty() ? 0.0 : *std::max_element(lat_ms_.begin(), lat_ms_.end());
    out->queue_p50_ms = percentile(queue_ms_, 0.50);
    out->queue_p99_ms = percentile(queue_ms_, 0.99);
    out->busy_s = busy_acc_ + (busy_since_ >= 0 ? sched_now_s() - busy_since_ : 0.0);
    out->host_launch_s = host_launch_s_;
  }

  // Refuse new jobs, run the queued and in-flight ones to completion, end
  // the threads.  Idempotent.
  void stop() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stopping_ = true;
    }
    cv_sched_.notify_all();
    cv_comp_.notify_all();
    if (sched_.joinable()) sched_.join();
    {
      std::unique_lock<std::mutex> lk(mu_);
      cv_done_.wait(lk, [&] { return jobs_in_flight_ == 0; });
    }
    cv_comp_.notify_all();
    if (comp_.joinable()) comp_.join();
  }

  size_t budget() const { return lim_.budget; }

 private:
  struct Step {
    int stream = -1;
    std::vector<Job *> jobs;
  };

  static double percentile(std::vector<double> v, double q) {
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    const double pos = q * (v.size() - 1);
    const size_t i = (size_t)pos;
    const double f = pos - i;
    return i + 1 < v.size() ? v[i] * (1 - f) + v[i + 1] * f : v[i];
  }

  // A job has ended (caller holds mu_): latency rings (admitted jobs only),
  // then forget the oldest ended jobs beyond keep_done, except those a
  // waiter still holds.
  void retire(Job *j, bool admitted) {
    if (admitted) {
      const double lat = (j->t_done - j->t_submit) * 1e3, qu = (j->t_launch - j->t_submit) * 1e3;
      if (lat_ms_.size() < lim_.lat_window) {
        lat_ms_.push_back(lat);
        queue_ms_.push_back(qu);
      } else {
        lat_ms_[lat_next_] = lat;
        queue_ms_[lat_next_] = qu;
      }
      lat_next_ = (lat_next_ + 1) % lim_.lat_window;
    }
    retired_.push_back(j->ticket);
    while (retired_.size() > lim_.keep_done) {
      auto it = all_.find(retired_.front());
      if (it != all_.end()) {
        if (it->second->waiters > 0) break;
        delete it->second;
        all_.erase(it);
      }
      retired_.pop_front();
    }
  }

  // An admitted job has ended (caller holds mu_).
  void end_admitted(Job *j) {
    arena_.release(j->arena_off, j->bytes);
    bytes_in_flight_ -= j->bytes;
    --jobs_in_flight_;
    ex_->release(j);
    retire(j, true);
  }

  int free_stream() const {
    for (size_t k = 0; k < busy_stream_.size(); ++k)
      if (!busy_stream_[k]) return (int)k;
    return -1;
  }

  void scheduler() {
    ex_->thread_start();
    std::unique_lock<std::mutex> lk(mu_);
    for (;;) {
      cv_sched_.wait(lk, [&] {
        if (stopping_ && queue_.empty()) return true;
        if (queue_.empty()) return false;
        return free_stream() >= 0 && jobs_in_flight_ < lim_.max_slots &&
               bytes_in_flight_ + queue_.front()->bytes <= lim_.budget;
      });
      if (stopping_ && queue_.empty()) break;
      // admit in FIFO order while memory and slots allow
      Step step;
      step.stream = free_stream();
      while (!queue_.empty() && jobs_in_flight_ < lim_.max_slots &&
             step.jobs.size() < (size_t)lim_.max_step_jobs) {
        Job *j = queue_.front();
        size_t off = 0;
        if (bytes_in_flight_ + j->bytes > lim_.budget || !arena_.alloc(j->bytes, &off)) break;
        queue_.pop_front();
        j->arena_off = off;
        bytes_in_flight_ += j->bytes;
        peak_bytes_ = std::max(peak_bytes_, bytes_in_flight_);
        ++jobs_in_flight_;
        ++st_.admitted;
        step.jobs.push_back(j);
      }
      if (step.jobs.empty()) {
        // the head fits the budget but not the fragmented arena: wait for a release
        cv_sched_.wait_for(lk, std::chrono::milliseconds(1));
        continue;
      }
      busy_stream_[step.stream] = 1;
      const double t0 = sched_now_s();
      for (Job *j : step.jobs) j->t_launch = t0;
      if (busy_since_ < 0) busy_since_ = t0;
      lk.unlock();
      std::string err;
      const int rc = ex_->launch(step.stream, step.jobs, err);
      const double t1 = sched_now_s();
      if (rc != TSQBX_OK) {
        ex_->sync(step.stream);  // the stream may hold partial work
        fprintf(stderr, "tsqbx server: step failed: %s\n", err.c_str());
      }
      lk.lock();
      host_launch_s_ += t1 - t0;
      if (rc != TSQBX_OK) {
        const double td = sched_now_s();
        for (Job *j : step.jobs) {
          j->status = rc;
          j->done = true;
          j->t_done = td;
          ++st_.failed;
          end_admitted(j);
        }
        busy_stream_[step.stream] = 0;
        if (inflight_.empty() && busy_since_ >= 0) {
          busy_acc_ += td - busy_since_;
          busy_since_ = -1;
        }
        cv_done_.notify_all();
        continue;
      }
      ++st_.steps;
      inflight_.push_back(std::move(step));
      cv_comp_.notify_all();
    }
  }

  void completer() {
    ex_->thread_start();
    std::unique_lock<std::mutex> lk(mu_);
    for (;;) {
      cv_comp_.wait(lk, [&] {
        return !inflight_.empty() || (stopping_ && queue_.empty() && jobs_in_flight_ == 0);
      });
      if (inflight_.empty()) break;
      // find a finished step, polling without the lock
      std::vector<int> streams;
      for (auto &s : inflight_) streams.push_back(s.stream);
      lk.unlock();
      int found = -1, q = 0;
      for (int spin = 0; found < 0; ++spin) {
        for (size_t i = 0; i < streams.size(); ++i) {
          q = ex_->query(streams[i]);
          if (q != 0) {
            found = (int)i;
            break;
          }
        }
        if (found < 0) {
          if (spin < 200)
            std::this_thread::yield();
          else
            std::this_thread::sleep_for(std::chrono::microseconds(20));
        }
        if (spin > 0 && spin % 64 == 0) {
          // new steps may have been launched meanwhile
          std::lock_guard<std::mutex> g(mu_);
          if (inflight_.size() != streams.size()) break;
        }
      }
      if (found < 0) {
        lk.lock();
        continue;
      }
      const int step_status = q == 1 ? TSQBX_OK : q;
      lk.lock();
      Step step = std::move(inflight_[found]);  // steps are only appended meanwhile
      inflight_.erase(inflight_.begin() + found);
      lk.unlock();
      // deliver the results without the lock (the jobs still count as in flight)
      std::vector<int> status;
      for (Job *j : step.jobs) status.push_back(ex_->finish(j, step_status));
      lk.lock();
      const double t1 = sched_now_s();
      for (size_t i = 0; i < step.jobs.size(); ++i) {
        Job *j = step.jobs[i];
        j->status = status[i];
        if (status[i] == TSQBX_OK) {
          ++st_.completed;
          st_.pair_terms_completed += j->pair_terms;
        } else {
          ++st_.failed;
        }
        j->t_done = t1;
        j->done = true;
        end_admitted(j);
      }
      busy_stream_[step.stream] = 0;
      if (inflight_.empty() && busy_since_ >= 0) {
        busy_acc_ += t1 - busy_since_;
        busy_since_ = -1;
      }
      cv_done_.notify_all();
      cv_sched_.notify_all();
    }
  }

  Executor *ex_;
  SchedLimits lim_;
  Arena arena_;
  std::mutex mu_;
  std::condition_variable cv_sched_, cv_done_, cv_comp_;
  std::deque<Job *> queue_;
  std::map<uint64_t, Job *> all_;
  std::vector<Step> inflight_;
  std::vector<char> busy_stream_;
  uint64_t next_ticket_ = 1;
  bool stopping_ = false;
  size_t bytes_in_flight_ = 0, peak_bytes_ = 0;
  int jobs_in_flight_ = 0;
  tsqbx_server_stats st_{};
  std::vector<double> lat_ms_, queue_ms_;  // rings of the last lat_window completions
  size_t lat_next_ = 0;
  std::deque<uint64_t> retired_;           // ended tickets, oldest first
  double busy_since_ = -1, busy_acc_ = 0;
  double host_launch_s_ = 0;               // scheduler time spent issuing steps
  std::thread sched_, comp_;
};

}  // namespace tsqbx
