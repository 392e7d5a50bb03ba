// Scheduler core of the request loop (fhe_server_*): continuous batching of requests
// that arrive over time, admission by a device-memory budget, completion records.
// Host-only C++17 with no HIP types: the device side is an executor policy class, so
// that the same core runs against the HIP executor in the library and against a mock
// executor in CPU tests (and under a thread sanitizer there).
//
// Executor interface (a class E):
//   using Job = ...;                        // the request payload
//   using Cell = ...;                       // requests of one cell can share a batch
//   Cell cell_of(const Job&) const;         // (ordered: used as a map key)
//   size_t unit_bytes(const Job&) const;    // scratch bytes per request of the job's cell
//   int launch(int slot, const std::vector<const Job*>& batch, size_t offset);
//       // queue the batch on the slot's stream with scratch at arena offset `offset`;
//       // FHE status (a failure completes the batch's requests with that status)
//   int poll(int slot);                     // 1 done, 0 running, < 0 failed (status)
//   void discard(const Job&);               // a request completed without a launch
//   uint64_t now();                         // monotonic nanoseconds
//
// Policy (one scheduler thread):
//   - A request with an arrival time in the future waits in a min-heap until then;
//     arrived requests wait in one FIFO per cell.
//   - Whenever a slot is idle, the cell whose front request arrived first is served:
//     up to max_batch of its requests form one batch (continuous batching: whatever
//     arrived while other batches ran joins the next batch).
//   - Admission by footprint: a batch of n requests needs n * unit bytes of scratch,
//     taken from an arena of `budget` bytes (first fit, 256-byte granules, released
//     when the batch completes).  The batch is cut to what the budget allows; if the
//     arena has no room now, the batch waits for completions; a request that needs more
//     than the whole budget alone completes with FHE_E_NOMEM.
//   - cancel(): requests not yet launched complete with FHE_E_STATE.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <queue>
#include <thread>
#include <vector>

namespace fhe {

// Completion record (the layout of fhe_done).
struct SrvDone {
  uint64_t ticket;
  int status;
  int batch;
  uint64_t t_arrive;
  uint64_t t_start;
  uint64_t t_done;
};

// First-fit allocator of byte ranges of one arena; ranges are 256-byte aligned.
class SrvArena {
 public:
  explicit SrvArena(size_t cap = 0) { reset(cap); }
  void reset(size_t cap) {
    cap_ = cap & ~(size_t)255;
    free_.clear();
    if (cap_) free_[0] = cap_;
  }
  size_t capacity() const { return cap_; }
  static size_t round(size_t bytes) { return (bytes + 255) & ~(size_t)255; }
  // Offset of a free range of `bytes` (rounded up), or false.
  bool alloc(size_t bytes, size_t* off) {
    const size_t b = round(std::max<size_t>(bytes, 1));
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < b) continue;
      *off = it->first;
      const size_t rest = it->second - b, at = it->first + b;
      free_.erase(it);
      if (rest) free_[at] = rest;
      return true;
    }
    return false;
  }
  // Returns a range taken by alloc (same `bytes`); neighbours are merged.
  void release(size_t off, size_t bytes) {
    const size_t b = round(std::max<size_t>(bytes, 1));
    auto it = free_.emplace(off, b).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t free_bytes() const {
    size_t s = 0;
    for (auto& kv : free_) s += kv.second;
    return s;
  }

 private:
  size_t cap_ = 0;
  std::map<size_t, size_t> free_;  // offset -> bytes
};

template <class E>
class SrvCore {
 public:
  using Job = typename E::Job;
  using Cell = typename E::Cell;

  // Status codes (the C ABI's): ok, out of memory, cancelled / bad state.
  static constexpr int kOk = 0, kNoMem = -4, kState = -6;

  SrvCore(E& exec, size_t budget, int nslots, int max_batch)
      : ex_(exec), arena_(budget), budget_(arena_.capacity()), max_batch_(max_batch), slots_(nslots) {}
  ~SrvCore() { stop(); }

  void start() { th_ = std::thread([this] { loop(); }); }

  // Stops the scheduler once every submitted request has completed.
  void stop() {
    {
      std::lock_guard<std::mutex> lk(m_);
      stop_ = true;
      cv_.notify_all();
    }
    if (th_.joinable()) th_.join();
  }

  // Queue one request; arrival 0 means now.  Returns the ticket, or 0 after stop.
  uint64_t submit(const Job& j, uint64_t arrival) {
    std::lock_guard<std::mutex> lk(m_);
    if (stop_) return 0;
    Req r;
    r.ticket = next_ticket_++;
    const uint64_t now = ex_.now();
    r.t_arrive = arrival ? arrival : now;
    r.job = j;
    ++submitted_;
    if (r.t_arrive > now)
      future_.push(r);
    else
      arrive(r);
    cv_.notify_all();
    return r.ticket;
  }

  // Moves up to `max` completion records to `out`; returns how many.
  int poll(SrvDone* out, int max) {
    std::lock_guard<std::mutex> lk(m_);
    const int n = (int)std::min<size_t>(done_.size(), (size_t)std::max(max, 0));
    for (int i = 0; i < n; ++i) out[i] = done_[i];
    done_.erase(done_.begin(), done_.begin() + n);
    return n;
  }

  void drain() {
    std::unique_lock<std::mutex> lk(m_);
    cv_.wait(lk, [&] { return finished_ == submitted_; });
  }

  // Requests not yet launched (queued or scheduled) complete with FHE_E_STATE.
  void cancel() {
    std::lock_guard<std::mutex> lk(m_);
    const uint64_t t = ex_.now();
    for (auto& kv : queues_)
      for (const Req& r : kv.second) {
        ex_.discard(r.job);
        finish_one(r, kState, 0, t, t);
      }
    queues_.clear();
    npending_ = 0;
    while (!future_.empty()) {
      ex_.discard(future_.top().job);
      finish_one(future_.top(), kState, 0, t, t);
      future_.pop();
    }
    cv_.notify_all();
  }

  size_t arena_free() {
    std::lock_guard<std::mutex> lk(m_);
    return arena_.free_bytes();
  }

 private:
  struct Req {
    uint64_t ticket = 0, t_arrive = 0;
    Job job{};
  };
  struct Later {
    bool operator()(const Req& a, const Req& b) const {
      return a.t_arrive != b.t_arrive ? a.t_arrive > b.t_arrive : a.ticket > b.ticket;
    }
  };
  struct Slot {
    bool busy = false;
    std::vector<Req> reqs;
    uint64_t t_start = 0;
    size_t off = 0, bytes = 0;
  };

  void arrive(const Req& r) {
    queues_[ex_.cell_of(r.job)].push_back(r);
    ++npending_;
  }

  void finish_one(const Req& r, int status, int batch, uint64_t t0, uint64_t t1) {
    done_.push_back(SrvDone{r.ticket, status, batch, r.t_arrive, t0, t1});
    ++finished_;
  }

  void finish(const std::vector<Req>& reqs, int status, uint64_t t0, uint64_t t1) {
    for (const Req& r : reqs) finish_one(r, status, (int)reqs.size(), t0, t1);
  }

  void loop() {
    std::unique_lock<std::mutex> lk(m_);
    for (;;) {
      bool progress = false;
      // completions (their scratch goes back to the arena)
      for (int s = 0; s < (int)slots_.size(); ++s) {
        Slot& sl = slots_[s];
        if (!sl.busy) continue;
        const int p = ex_.poll(s);
        if (p == 0) continue;
        finish(sl.reqs, p > 0 ? kOk : p, sl.t_start, ex_.now());
        arena_.release(sl.off, sl.bytes);
        sl.busy = false;
        sl.reqs.clear();
        progress = true;
      }
      // scheduled arrivals that are due join the queues in arrival order
      uint64_t now = ex_.now();
      while (!future_.empty() && future_.top().t_arrive <= now) {
        arrive(future_.top());
        future_.pop();
      }
      const uint64_t next_arrival = future_.empty() ? UINT64_MAX : future_.top().t_arrive;
      // admissions: the oldest request first, batched with the requests of its cell
      while (npending_ > 0) {
        std::deque<Req>* q = nullptr;
        for (auto& kv : queues_) {
          if (kv.second.empty()) continue;
          const Req& f = kv.second.front();
          if (!q || f.t_arrive < q->front().t_arrive ||
              (f.t_arrive == q->front().t_arrive && f.ticket < q->front().ticket))
            q = &kv.second;
        }
        const size_t unit = ex_.unit_bytes(q->front().job);
        if (SrvArena::round(unit) > budget_) {  // cannot run even alone
          const Req r = q->front();
          q->pop_front();
          --npending_;
          const uint64_t t = ex_.now();
          ex_.discard(r.job);
          finish_one(r, kNoMem, 0, t, t);
          progress = true;
          continue;
        }
        int slot = -1;
        for (int s = 0; s < (int)slots_.size(); ++s)
          if (!slots_[s].busy) {
            slot = s;
            break;
          }
        if (slot < 0) break;  // every slot is running a batch
        int take = std::min((int)q->size(), max_batch_);
        while (take > 1 && SrvArena::round((size_t)take * unit) > budget_) --take;
        size_t off = 0;
        while (take >= 1 && !arena_.alloc((size_t)take * unit, &off)) --take;
        if (take < 1) break;  // wait for running batches to give memory back
        Slot& sl = slots_[slot];
        sl.reqs.assign(q->begin(), q->begin() + take);
        q->erase(q->begin(), q->begin() + take);
        npending_ -= take;
        sl.busy = true;
        sl.off = off;
        sl.bytes = (size_t)take * unit;
        sl.t_start = ex_.now();
        std::vector<const Job*> jobs;
        for (const Req& r : sl.reqs) jobs.push_back(&r.job);
        lk.unlock();
        const int rc = ex_.launch(slot, jobs, off);
        lk.lock();
        if (rc != kOk) {
          finish(sl.reqs, rc, sl.t_start, ex_.now());
          arena_.release(sl.off, sl.bytes);
          sl.busy = false;
          sl.reqs.clear();
        }
        progress = true;
        now = ex_.now();
      }
      bool busy = false;
      for (const Slot& sl : slots_) busy = busy || sl.busy;
      if (stop_ && npending_ == 0 && future_.empty() && !busy) break;
      if (progress) {
        cv_.notify_all();
      } else {
        // sleep until a completion may be due, the next scheduled arrival, or a submit
        uint64_t wait = busy ? 20000 : 500000;
        if (next_arrival != UINT64_MAX) wait = std::min(wait, next_arrival > now ? next_arrival - now : 0);
        if (wait > 0) timed_wait(lk, wait);
      }
    }
    cv_.notify_all();
  }

  // Bounded sleep on the condition variable.  The steady clock normally; builds under
  // GCC 11's ThreadSanitizer define FHE_SRV_SYSTEM_CLOCK_WAIT, since its runtime does
  // not intercept the steady-clock wait (pthread_cond_clockwait) and then misreads the
  // mutex's state.
  void timed_wait(std::unique_lock<std::mutex>& lk, uint64_t ns) {
#ifdef FHE_SRV_SYSTEM_CLOCK_WAIT
    cv_.wait_until(lk, std::chrono::system_clock::now() + std::chrono::nanoseconds(ns));
#else
    cv_.wait_for(lk, std::chrono::nanoseconds(ns));
#endif
  }

  E& ex_;
  SrvArena arena_;
  size_t budget_;
  int max_batch_;
  std::vector<Slot> slots_;
  std::map<Cell, std::deque<Req>> queues_;
  size_t npending_ = 0;
  std::priority_queue<Req, std::vector<Req>, Later> future_;
  std::vector<SrvDone> done_;
  std::mutex m_;
  std::condition_variable cv_;
  std::thread th_;
  bool stop_ = false;
  uint64_t next_ticket_ = 1, submitted_ = 0, finished_ = 0;
};

}  // namespace fhe
