// The serving scheduler (paper_1811_01110_amd/csrc/tsqbx_sched.h) driven on
// the CPU by a fake executor: steps "run" for a set time on a host clock and
// deliver outputs computed by the CPU oracle, so admission under the memory
// budget, FIFO order, slot limits, arena fragmentation, failures of a launch,
// of a step and of one job, cancellation, time-outs, shutdown with work in
// flight and the bounded ticket history are checked without a device.  The
// fake checks its own invariants on every launch (ranges inside the budget
// and disjoint, tickets admitted in increasing order, at most max_slots jobs
// and max_step_jobs per step, one step per stream) and counts releases.
// Built with AddressSanitizer/UBSan and, separately, ThreadSanitizer.
//
// Usage: server_fake_driver <scenario>; prints "<scenario> ok".
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <random>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "tsqbx_oracle.h"
#include "tsqbx_sched.h"

using namespace tsqbx;

#define CHECK(c)                                                     \
  do {                                                               \
    if (!(c)) {                                                      \
      std::fprintf(stderr, "CHECK failed %s:%d: %s\n", __FILE__, __LINE__, #c); \
      std::exit(1);                                                  \
    }                                                                \
  } while (0)

namespace {

double now_ms() { return sched_now_s() * 1e3; }
void sleep_ms(double ms) { std::this_thread::sleep_for(std::chrono::duration<double, std::milli>(ms)); }

// A small single-layer problem for the oracle: sources on a sphere, one
// center per target inside it, every source in every list.
struct Problem {
  int64_t N = 48, M = 6;
  std::vector<double> src, w, ctr, tgt;
  std::vector<int64_t> off;
  std::vector<int32_t> list;
  tsqbx_oracle_problem op{};
  Problem() {
    std::mt19937_64 rng(7);
    std::uniform_real_distribution<double> u(-1.0, 1.0);
    for (int64_t i = 0; i < N; ++i) {
      double v[3], r = 0;
      for (double &x : v) {
        x = u(rng);
        r += x * x;
      }
      r = std::sqrt(r);
      for (double x : v) src.push_back(x / r);
      w.push_back(0.5 + 0.25 * u(rng));
    }
    off.push_back(0);
    for (int64_t c = 0; c < M; ++c) {
      for (int a = 0; a < 3; ++a) ctr.push_back(0.2 * u(rng));
      for (int a = 0; a < 3; ++a) tgt.push_back(ctr[3 * c + a] + 0.05 * u(rng));
      for (int64_t i = 0; i < N; ++i) list.push_back((int32_t)i);
      off.push_back((int64_t)list.size());
    }
    op.n_sources = N;
    op.sources = src.data();
    op.weights = w.data();
    op.n_centers = M;
    op.centers = ctr.data();
    op.list_offsets = off.data();
    op.list_sources = list.data();
    op.n_targets = M;
    op.targets = tgt.data();
  }
  void eval(const std::vector<double> &sigma, double *out) const {
    double *const outs[3] = {out, nullptr, nullptr};
    double *const abs[3] = {nullptr, nullptr, nullptr};
    CHECK(tsqbx_oracle_eval(&op, 6, TSQBX_ORACLE_SLP, sigma.data(), 0, nullptr, outs, abs, 1) == 0);
  }
};

const Problem &problem() {
  static Problem P;
  return P;
}

struct FakeJob : Job {
  int id = 0;
  std::vector<double> sigma;
  double *out = nullptr;     // the caller's buffer (problem().M entries)
  double work_ms = 0;        // time its step runs, summed over the step
  bool fail_launch = false;  // its step's launch fails
  bool fail_step = false;    // its step fails on the device
  bool fail_finish = false;  // only its own delivery fails
  int stream = -1;
  double t_launched = -1, t_finished = -1;
  std::atomic<int> *released = nullptr;  // counter in the test's record
};

class FakeExec : public Executor {
 public:
  FakeExec(int streams, const SchedLimits &lim) : lim_(lim), slots_(streams) {}
  int streams() const override { return (int)slots_.size(); }

  int launch(int stream, const std::vector<Job *> &jobs, std::string &err) override {
    std::lock_guard<std::mutex> g(m_);
    CHECK(stream >= 0 && stream < (int)slots_.size());
    Slot &sl = slots_[stream];
    CHECK(!sl.active);  // one step per stream
    CHECK(!jobs.empty() && (int)jobs.size() <= lim_.max_step_jobs);
    bool fail = false, fail_step = false;
    double work = 0;
    for (Job *j0 : jobs) {
      auto *j = static_cast<FakeJob *>(j0);
      CHECK(j->ticket > last_ticket_);  // FIFO admission
      last_ticket_ = j->ticket;
      CHECK(j->bytes <= lim_.budget && j->arena_off + j->bytes <= lim_.budget);
      for (auto &kv : ranges_) {  // disjoint from every range in flight
        const size_t a = kv.second.first, b = a + kv.second.second;
        CHECK(j->bytes == 0 || kv.second.second == 0 || j->arena_off >= b ||
              j->arena_off + j->bytes <= a);
      }
      ranges_[j->ticket] = {j->arena_off, j->bytes};
      bytes_ += j->bytes;
      fail |= j->fail_launch;
      fail_step |= j->fail_step;
      work += j->work_ms;
      j->stream = stream;
      j->t_launched = now_ms();
      launched_.push_back(j->id);
    }
    CHECK(bytes_ <= lim_.budget);
    CHECK((int)ranges_.size() <= lim_.max_slots);
    peak_jobs_ = std::max(peak_jobs_, (int)ranges_.size());
    peak_bytes_ = std::max(peak_bytes_, bytes_);
    ++launches_;
    if (fail) {
      for (Job *j : jobs) {
        bytes_ -= j->bytes;
        ranges_.erase(j->ticket);
      }
      err = "launch failure planted by the test";
      return TSQBX_E_DEVICE;
    }
    sl.active = true;
    sl.left = (int)jobs.size();
    sl.ready_at = now_ms() + work;
    sl.status = fail_step ? TSQBX_E_DEVICE : TSQBX_OK;
    return TSQBX_OK;
  }

  int query(int stream) override {
    std::lock_guard<std::mutex> g(m_);
    Slot &sl = slots_[stream];
    CHECK(sl.active);
    if (now_ms() < sl.ready_at) return 0;
    return sl.status == TSQBX_OK ? 1 : sl.status;
  }

  void sync(int) override {}

  int finish(Job *j0, int step_status) override {
    auto *j = static_cast<FakeJob *>(j0);
    int rc = step_status;
    if (rc == TSQBX_OK && j->fail_finish) rc = TSQBX_E_DEVICE;
    if (rc == TSQBX_OK) problem().eval(j->sigma, j->out);
    std::lock_guard<std::mutex> g(m_);
    Slot &sl = slots_[j->stream];
    CHECK(sl.active && sl.left > 0);
    if (--sl.left == 0) sl.active = false;
    auto it = ranges_.find(j->ticket);
    CHECK(it != ranges_.end());
    bytes_ -= it->second.second;
    ranges_.erase(it);
    j->t_finished = now_ms();
    return rc;
  }

  void release(Job *j0) override {
    auto *j = static_cast<FakeJob *>(j0);
    if (j->released) j->released->fetch_add(1);
    std::vector<double>().swap(j->sigma);
  }

  std::vector<int> launched() {
    std::lock_guard<std::mutex> g(m_);
    return launched_;
  }
  int peak_jobs() {
    std::lock_guard<std::mutex> g(m_);
    return peak_jobs_;
  }
  size_t peak_bytes() {
    std::lock_guard<std::mutex> g(m_);
    return peak_bytes_;
  }

 private:
  struct Slot {
    bool active = false;
    int left = 0;
    double ready_at = 0;
    int status = TSQBX_OK;
  };
  SchedLimits lim_;
  std::mutex m_;
  std::vector<Slot> slots_;
  std::map<uint64_t, std::pair<size_t, size_t>> ranges_;  // ticket -> (offset, bytes)
  size_t bytes_ = 0, peak_bytes_ = 0;
  int peak_jobs_ = 0, launches_ = 0;
  uint64_t last_ticket_ = 0;
  std::vector<int> launched_;
};

// One scenario's server: the fake executor, the scheduler, the callers'
// output buffers and the jobs' observation records.
struct Rig {
  SchedLimits lim;
  std::unique_ptr<FakeExec> ex;
  std::unique_ptr<Scheduler> sc;
  std::atomic<int> released{0};
  std::atomic<int> submitted{0};
  std::mutex m;
  std::vector<std::unique_ptr<std::vector<double>>> outs;
  std::map<int, FakeJob *> by_id;  // valid while the scheduler keeps the job

  Rig(size_t budget, int max_slots, int max_step, int streams, size_t keep_done = 4096) {
    lim.budget = budget;
    lim.max_slots = max_slots;
    lim.max_step_jobs = max_step;
    lim.keep_done = keep_done;
    lim.lat_window = 1024;
    ex = std::make_unique<FakeExec>(streams, lim);
    sc = std::make_unique<Scheduler>(ex.get(), lim);
    sc->start();
  }
  ~Rig() { sc.reset(); }

  // Submit job id with these bytes; returns the status and the ticket.
  int submit(int id, size_t bytes, double work_ms, uint64_t *ticket, double **out_buf = nullptr,
             std::vector<double> *sigma_out = nullptr, bool fail_launch = false,
             bool fail_step = false, bool fail_finish = false) {
    auto *j = new FakeJob;
    j->id = id;
    j->bytes = bytes;
    j->work_ms = work_ms;
    j->fail_launch = fail_launch;
    j->fail_step = fail_step;
    j->fail_finish = fail_finish;
    j->released = &released;
    std::mt19937_64 rng(1000 + id);
    std::normal_distribution<double> nd;
    for (int64_t i = 0; i < problem().N; ++i) j->sigma.push_back(nd(rng));
    if (sigma_out) *sigma_out = j->sigma;
    {
      std::lock_guard<std::mutex> g(m);
      outs.push_back(std::make_unique<std::vector<double>>(problem().M, -1.0));
      j->out = outs.back()->data();
      by_id[id] = j;
    }
    if (out_buf) *out_buf = j->out;
    ++submitted;
    return sc->submit(j, ticket);
  }
};

void scenario_mix() {
  // many jobs of random sizes (some the whole budget) from four threads
  const size_t B = 1 << 20;
  Rig rig(B, 8, 4, 3);
  const int per_thread = 100;
  struct Rec {
    uint64_t ticket;
    double *out;
    std::vector<double> sigma;
  };
  std::vector<std::vector<Rec>> recs(4);
  std::vector<std::thread> th;
  for (int t = 0; t < 4; ++t)
    th.emplace_back([&, t] {
      std::mt19937_64 rng(t);
      for (int k = 0; k < per_thread; ++k) {
        const int id = t * per_thread + k;
        const size_t bytes = (k % 37 == 5) ? B : 1 + rng() % (B / 3);
        Rec r;
        CHECK(rig.submit(id, bytes, 0.02 * (rng() % 10), &r.ticket, &r.out, &r.sigma) == TSQBX_OK);
        recs[t].push_back(std::move(r));
        if (k % 16 == 0) sleep_ms(0.2);
      }
    });
  for (auto &t : th) t.join();
  CHECK(rig.sc->drain(60.0) == TSQBX_OK);
  std::vector<double> want(problem().M);
  for (auto &v : recs)
    for (auto &r : v) {
      int st = -99;
      CHECK(rig.sc->wait(r.ticket, 1.0, &st) == TSQBX_OK && st == TSQBX_OK);
      problem().eval(r.sigma, want.data());
      CHECK(std::memcmp(want.data(), r.out, want.size() * sizeof(double)) == 0);
    }
  tsqbx_server_stats s;
  rig.sc->stats(&s);
  CHECK(s.submitted == 4 * per_thread && s.completed == 4 * per_thread && s.failed == 0);
  CHECK(s.admitted == 4 * per_thread && s.bytes_in_flight == 0);
  CHECK(s.peak_bytes_in_flight <= B && rig.ex->peak_bytes() <= B);
  CHECK(rig.ex->peak_jobs() <= 8 && s.steps >= 4 * per_thread / 4);
  CHECK(s.latency_p50_ms > 0 && s.latency_p99_ms >= s.latency_p50_ms);
  CHECK(rig.released.load() == 4 * per_thread);
}

void scenario_budget() {
  Rig rig(4096, 4, 4, 2);
  uint64_t t = 0;
  CHECK(rig.submit(1, 4097, 0, &t) == TSQBX_E_BUDGET);
  CHECK(rig.submit(2, 4096, 0.5, &t) == TSQBX_OK);
  int st = -99;
  CHECK(rig.sc->wait(t, 5.0, &st) == TSQBX_OK && st == TSQBX_OK);
  tsqbx_server_stats s;
  rig.sc->stats(&s);
  CHECK(s.rejected == 1 && s.submitted == 2 && s.completed == 1);
  CHECK(rig.released.load() == 2);  // the refused job was released too
}

void scenario_failures() {
  // a failed launch, a failed step and one failed delivery; the rest complete
  Rig rig(1 << 16, 16, 1, 2);  // one job per step
  std::vector<uint64_t> tk(12);
  for (int i = 0; i < 12; ++i)
    CHECK(rig.submit(i, 1024, 0.3, &tk[i], nullptr, nullptr, i == 3, i == 6, i == 9) == TSQBX_OK);
  CHECK(rig.sc->drain(10.0) == TSQBX_OK);
  for (int i = 0; i < 12; ++i) {
    int st = -99;
    CHECK(rig.sc->wait(tk[i], 1.0, &st) == TSQBX_OK);
    CHECK(st == ((i == 3 || i == 6 || i == 9) ? TSQBX_E_DEVICE : TSQBX_OK));
  }
  // a step of several jobs where one delivery fails: only that job fails
  Rig r2(1 << 16, 16, 8, 1);
  std::vector<uint64_t> t2(8);
  uint64_t blocker = 0;
  CHECK(r2.submit(100, 1024, 30.0, &blocker) == TSQBX_OK);  // holds the one stream
  sleep_ms(2);
  for (int i = 0; i < 8; ++i)
    CHECK(r2.submit(i, 1024, 0.1, &t2[i], nullptr, nullptr, false, false, i == 5) == TSQBX_OK);
  CHECK(r2.sc->drain(10.0) == TSQBX_OK);
  for (int i = 0; i < 8; ++i) {
    int st = -99;
    CHECK(r2.sc->wait(t2[i], 1.0, &st) == TSQBX_OK);
    CHECK(st == (i == 5 ? TSQBX_E_DEVICE : TSQBX_OK));
  }
  tsqbx_server_stats s;
  r2.sc->stats(&s);
  CHECK(s.completed == 8 && s.failed == 1 && s.steps == 2);
}

void scenario_cancel_timeout() {
  Rig rig(1 << 16, 1, 1, 1);  // one job at a time
  uint64_t a = 0, b = 0, c = 0;
  CHECK(rig.submit(0, 1024, 60.0, &a) == TSQBX_OK);
  CHECK(rig.submit(1, 1024, 0.1, &b) == TSQBX_OK);
  CHECK(rig.submit(2, 1024, 0.1, &c) == TSQBX_OK);
  sleep_ms(5);
  int st = -99;
  CHECK(rig.sc->wait(b, 0.001, &st) == TSQBX_E_TIMEOUT);
  CHECK(rig.sc->cancel(b) == TSQBX_OK);
  CHECK(rig.sc->cancel(b) == TSQBX_E_STATE);     // ended
  CHECK(rig.sc->cancel(a) == TSQBX_E_STATE);     // admitted
  CHECK(rig.sc->cancel(999) == TSQBX_E_INVALID);  // unknown
  CHECK(rig.sc->wait(b, 1.0, &st) == TSQBX_OK && st == TSQBX_E_CANCELED);
  int done = 0;
  CHECK(rig.sc->poll(c, &done, &st) == TSQBX_OK && done == 0);
  CHECK(rig.sc->wait(c, 10.0, &st) == TSQBX_OK && st == TSQBX_OK);
  const auto l = rig.ex->launched();
  CHECK(l.size() == 2 && l[0] == 0 && l[1] == 2);  // the cancelled job never ran
  tsqbx_server_stats s;
  rig.sc->stats(&s);
  CHECK(s.completed == 2 && s.failed == 1 && rig.released.load() == 3);
}

void scenario_fragmentation() {
  // four 1 KiB jobs fill a 4 KiB arena; the 1st and 3rd end first, leaving
  // 2 KiB free in two pieces: the next 2 KiB job fits the budget but not the
  // arena and waits for the 2nd, and the 1 KiB job queued behind it waits too
  Rig rig(4096, 16, 1, 4);
  uint64_t t[6];
  const double work[4] = {10, 150, 10, 150};
  for (int i = 0; i < 4; ++i) CHECK(rig.submit(i, 1024, work[i], &t[i]) == TSQBX_OK);
  sleep_ms(5);
  CHECK(rig.submit(4, 2048, 1, &t[4]) == TSQBX_OK);
  CHECK(rig.submit(5, 1024, 1, &t[5]) == TSQBX_OK);
  int st = -99;
  for (int i = 0; i < 6; ++i) CHECK(rig.sc->wait(t[i], 10.0, &st) == TSQBX_OK && st == TSQBX_OK);
  FakeJob *j1 = rig.by_id[1], *j3 = rig.by_id[3], *j4 = rig.by_id[4], *j5 = rig.by_id[5];
  CHECK(j4->arena_off == 0);  // the coalesced range of jobs 0 and 1
  CHECK(j4->t_launched >= std::min(j1->t_finished, j3->t_finished));
  CHECK(j5->t_launched >= j4->t_launched);  // FIFO: no overtaking
  const auto l = rig.ex->launched();
  CHECK(l.size() == 6 && l[4] == 4 && l[5] == 5);
}

void scenario_stop_in_flight() {
  // shutdown with work queued and running: everything finishes, later
  // submissions are refused, every job is released once
  auto rig = std::make_unique<Rig>(1 << 14, 4, 2, 2);
  std::vector<uint64_t> tk(40);
  for (int i = 0; i < 40; ++i) CHECK(rig->submit(i, 1000 + 37 * i, 0.5, &tk[i]) == TSQBX_OK);
  rig->sc->stop();
  tsqbx_server_stats s;
  rig->sc->stats(&s);
  CHECK(s.completed == 40 && s.bytes_in_flight == 0);
  uint64_t t = 0;
  CHECK(rig->submit(99, 10, 0, &t) == TSQBX_E_STATE);
  CHECK(rig->released.load() == 41);
  rig.reset();
}

void scenario_history() {
  // only keep_done ended tickets stay queryable; waiters keep theirs
  Rig rig(1 << 16, 16, 8, 1, /*keep_done=*/1);
  uint64_t blocker = 0;
  CHECK(rig.submit(100, 64, 40.0, &blocker) == TSQBX_OK);
  sleep_ms(2);
  std::vector<uint64_t> tk(8);
  for (int i = 0; i < 8; ++i) CHECK(rig.submit(i, 64, 0.1, &tk[i]) == TSQBX_OK);
  std::vector<std::thread> waiters;
  std::atomic<int> ok{0};
  for (int i = 0; i < 8; ++i)
    waiters.emplace_back([&, i] {
      int st = -99;
      if (rig.sc->wait(tk[i], 10.0, &st) == TSQBX_OK && st == TSQBX_OK) ++ok;
    });
  for (auto &w : waiters) w.join();
  CHECK(ok.load() == 8);
  CHECK(rig.sc->drain(5.0) == TSQBX_OK);
  uint64_t more[20];
  for (int i = 0; i < 20; ++i) CHECK(rig.submit(200 + i, 64, 0.0, &more[i]) == TSQBX_OK);
  CHECK(rig.sc->drain(5.0) == TSQBX_OK);
  int done = 0, st = 0;
  CHECK(rig.sc->poll(tk[0], &done, &st) == TSQBX_E_INVALID);  // forgotten
  CHECK(rig.sc->poll(more[19], &done, &st) == TSQBX_OK && done == 1 && st == TSQBX_OK);
}

}  // namespace

int main(int argc, char **argv) {
  const std::string which = argc > 1 ? argv[1] : "all";
  const std::pair<const char *, void (*)()> all[] = {
      {"mix", scenario_mix},
      {"budget", scenario_budget},
      {"failures", scenario_failures},
      {"cancel_timeout", scenario_cancel_timeout},
      {"fragmentation", scenario_fragmentation},
      {"stop_in_flight", scenario_stop_in_flight},
      {"history", scenario_history},
  };
  int ran = 0;
  for (auto &s : all)
    if (which == "all" || which == s.first) {
      s.second();
      std::printf("%s ok\n", s.first);
      std::fflush(stdout);
      ++ran;
    }
  return ran > 0 ? 0 : 2;
}
