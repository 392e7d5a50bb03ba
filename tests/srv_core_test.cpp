// CPU tests of the request loop's scheduler core (paper_2607_05920_amd/csrc/srv_core.h)
// against a mock executor: a fake device whose batches "complete" after a set delay,
// with injectable launch and completion errors.  Built and run by tests/test_srv_core.py
// (also under -fsanitize=thread).  Prints one line per test; exits non-zero on failure.
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <set>
#include <string>
#include <thread>

#include "srv_core.h"

using namespace fhe;

namespace {

int g_failures = 0;
#define CHECK(c)                                                     \
  do {                                                               \
    if (!(c)) {                                                      \
      std::printf("  FAILED %s:%d: %s\n", __FILE__, __LINE__, #c);   \
      ++g_failures;                                                  \
    }                                                                \
  } while (0)

uint64_t steady_ns() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct MockJob {
  int cell = 0;
  size_t unit = 1000;
  int launch_status = 0;  // injected launch error (FHE status)
  int done_status = 1;    // 1: completes fine; < 0: the device reports this error
  uint64_t delay_ns = 200000;
};

// A fake device: every slot runs one batch at a time; a batch completes `delay` after
// its launch (the largest delay of its jobs).  Records what it was asked to run.
struct MockExec {
  using Job = MockJob;
  using Cell = int;
  struct Run {
    int slot;
    std::vector<MockJob> jobs;
    size_t off;
    uint64_t t_launch, t_ready;
  };
  std::mutex m;
  std::vector<Run> runs;           // every launch, in order
  std::map<int, size_t> current;   // slot -> index into runs
  std::atomic<int> concurrent{0}, max_concurrent{0};
  size_t max_arena_end = 0;

  Cell cell_of(const Job& j) const { return j.cell; }
  size_t unit_bytes(const Job& j) const { return j.unit; }
  uint64_t now() { return steady_ns(); }
  int launch(int slot, const std::vector<const Job*>& batch, size_t off) {
    std::lock_guard<std::mutex> lk(m);
    Run r{slot, {}, off, now(), 0};
    uint64_t d = 0;
    size_t bytes = 0;
    for (const Job* j : batch) {
      r.jobs.push_back(*j);
      d = std::max(d, j->delay_ns);
      bytes += j->unit;
      if (j->launch_status != 0) return j->launch_status;
    }
    r.t_ready = r.t_launch + d;
    max_arena_end = std::max(max_arena_end, off + bytes);
    current[slot] = runs.size();
    runs.push_back(r);
    const int c = ++concurrent;
    int m0 = max_concurrent.load();
    while (c > m0 && !max_concurrent.compare_exchange_weak(m0, c)) {
    }
    return 0;
  }
  std::atomic<int> discarded{0};
  void discard(const Job&) { ++discarded; }
  int poll(int slot) {
    std::lock_guard<std::mutex> lk(m);
    const Run& r = runs[current.at(slot)];
    if (now() < r.t_ready) return 0;
    --concurrent;
    for (const MockJob& j : r.jobs)
      if (j.done_status < 0) return j.done_status;
    return 1;
  }
};

std::vector<SrvDone> all_done(SrvCore<MockExec>& core, size_t n) {
  std::vector<SrvDone> out(n + 8);
  const int k = core.poll(out.data(), (int)out.size());
  out.resize(k);
  return out;
}

void test_burst_batches_by_cell() {
  std::printf("burst_batches_by_cell\n");
  MockExec ex;
  SrvCore<MockExec> core(ex, 1 << 20, 2, 4);
  // 10 requests of cell 0 and 5 of cell 1, all arriving now; the first batch launches
  // at once, the rest queue behind it and are merged
  std::vector<uint64_t> t;
  const uint64_t t0 = steady_ns() + 2000000;  // all arrive together, after the submits
  for (int i = 0; i < 15; ++i) {
    MockJob j;
    j.cell = i < 10 ? 0 : 1;
    j.delay_ns = 1000000;
    t.push_back(core.submit(j, t0));
  }
  core.start();
  core.drain();
  auto d = all_done(core, 15);
  CHECK(d.size() == 15);
  int maxb = 0;
  for (auto& x : d) {
    CHECK(x.status == 0);
    maxb = std::max(maxb, x.batch);
    CHECK(x.t_done >= x.t_start && x.t_start >= x.t_arrive);
  }
  CHECK(maxb == 4);  // max_batch caps a batch
  for (auto& r : ex.runs) {
    std::set<int> cells;
    for (auto& j : r.jobs) cells.insert(j.cell);
    CHECK(cells.size() == 1);  // a batch never mixes cells
  }
  CHECK(ex.max_concurrent.load() <= 2);
  core.stop();
  CHECK(core.arena_free() == (1u << 20));
}

void test_oldest_first_across_cells() {
  std::printf("oldest_first_across_cells\n");
  MockExec ex;
  SrvCore<MockExec> core(ex, 1 << 20, 1, 8);
  const uint64_t t0 = steady_ns() + 3000000;
  // cell 2 arrives first, then cell 1, then cell 0: one slot serves them in that order
  for (int c = 2; c >= 0; --c)
    for (int i = 0; i < 3; ++i) {
      MockJob j;
      j.cell = c;
      core.submit(j, t0 + (uint64_t)(2 - c) * 1000000 + i);
    }
  core.start();
  core.drain();
  CHECK(ex.runs.size() >= 3);
  std::vector<int> order;
  for (auto& r : ex.runs)
    if (order.empty() || order.back() != r.jobs[0].cell) order.push_back(r.jobs[0].cell);
  CHECK((order == std::vector<int>{2, 1, 0}));
  core.stop();
}

void test_future_arrivals_wait() {
  std::printf("future_arrivals_wait\n");
  MockExec ex;
  SrvCore<MockExec> core(ex, 1 << 20, 2, 8);
  core.start();
  const uint64_t t0 = steady_ns() + 20000000;  // 20 ms ahead
  MockJob j;
  core.submit(j, t0);
  core.drain();
  auto d = all_done(core, 1);
  CHECK(d.size() == 1 && d[0].t_start >= t0 && d[0].t_arrive == t0);
  core.stop();
}

void test_budget_zero_and_oversized_rejected() {
  std::printf("budget_zero_and_oversized_rejected\n");
  MockExec ex;
  SrvCore<MockExec> core(ex, 0, 2, 4);
  core.start();
  for (int i = 0; i < 5; ++i) core.submit(MockJob{}, 0);
  core.drain();
  auto d = all_done(core, 5);
  CHECK(d.size() == 5);
  for (auto& x : d) CHECK(x.status == -4);
  CHECK(ex.runs.empty() && ex.discarded.load() == 5);
  core.stop();
  // a budget that holds one request of the small cell but no request of the big one
  MockExec ex2;
  SrvCore<MockExec> c2(ex2, 4096, 2, 4);
  c2.start();
  MockJob small, big;
  small.unit = 1000;
  big.unit = 5000;
  big.cell = 1;
  c2.submit(small, 0);
  c2.submit(big, 0);
  c2.submit(small, 0);
  c2.drain();
  auto d2 = all_done(c2, 3);
  CHECK(d2.size() == 3);
  for (auto& x : d2) CHECK(x.status == (x.ticket == 2 ? -4 : 0));
  c2.stop();
}

void test_batch_cut_to_budget_and_waits_for_memory() {
  std::printf("batch_cut_to_budget_and_waits_for_memory\n");
  MockExec ex;
  // room for 2 requests of 1000 bytes (rounded to 1024) at a time, 4 slots
  SrvCore<MockExec> core(ex, 2048, 4, 8);
  const uint64_t t0 = steady_ns() + 2000000;
  for (int i = 0; i < 9; ++i) {
    MockJob j;
    j.delay_ns = 500000;
    core.submit(j, t0);
  }
  core.start();
  core.drain();
  auto d = all_done(core, 9);
  CHECK(d.size() == 9);
  for (auto& x : d) CHECK(x.status == 0 && x.batch <= 2);
  CHECK(ex.max_arena_end <= 2048);
  // never more scratch in flight than the budget: at most one 2-request batch at a time
  CHECK(ex.max_concurrent.load() == 1);
  core.stop();
  CHECK(core.arena_free() == 2048);
}

void test_injected_errors() {
  std::printf("injected_errors\n");
  MockExec ex;
  SrvCore<MockExec> core(ex, 1 << 20, 2, 1);
  core.start();
  MockJob ok, bad_launch, bad_device;
  bad_launch.launch_status = -5;
  bad_device.done_status = -5;
  core.submit(ok, 0);
  core.submit(bad_launch, 0);
  core.submit(bad_device, 0);
  core.submit(ok, 0);
  core.drain();
  auto d = all_done(core, 4);
  CHECK(d.size() == 4);
  std::map<uint64_t, int> st;
  for (auto& x : d) st[x.ticket] = x.status;
  CHECK(st[1] == 0 && st[2] == -5 && st[3] == -5 && st[4] == 0);
  core.stop();
  CHECK(core.arena_free() == (1u << 20));
}

void test_cancel() {
  std::printf("cancel\n");
  MockExec ex;
  SrvCore<MockExec> core(ex, 1 << 20, 1, 1);
  core.start();
  MockJob slow;
  slow.delay_ns = 20000000;
  core.submit(slow, 0);                              // launches at once
  const uint64_t later = steady_ns() + 1000000000;   // 1 s ahead: still scheduled
  for (int i = 0; i < 3; ++i) core.submit(MockJob{}, 0);
  core.submit(MockJob{}, later);
  std::this_thread::sleep_for(std::chrono::milliseconds(2));
  core.cancel();
  core.drain();
  auto d = all_done(core, 5);
  CHECK(d.size() == 5);
  int ok = 0, cancelled = 0;
  for (auto& x : d) {
    if (x.status == 0) ++ok;
    if (x.status == -6) ++cancelled;
  }
  CHECK(ok == 1 && cancelled == 4 && ex.discarded.load() == 4);
  core.stop();
}

void test_concurrent_submitters() {
  std::printf("concurrent_submitters\n");
  MockExec ex;
  SrvCore<MockExec> core(ex, 64 * 1024, 4, 16);
  core.start();
  std::vector<std::thread> th;
  std::atomic<int> polled{0};
  for (int w = 0; w < 4; ++w)
    th.emplace_back([&, w] {
      for (int i = 0; i < 200; ++i) {
        MockJob j;
        j.cell = (w + i) % 5;
        j.unit = 1000 + 100 * j.cell;
        j.delay_ns = 20000 + 1000 * (i % 7);
        core.submit(j, i % 3 ? 0 : steady_ns() + 100000);
      }
    });
  std::thread poller([&] {
    std::vector<SrvDone> buf(64);
    while (polled.load() < 800) {
      const int n = core.poll(buf.data(), 64);
      for (int i = 0; i < n; ++i) CHECK(buf[i].status == 0);
      polled += n;
      if (!n) std::this_thread::sleep_for(std::chrono::microseconds(200));
    }
  });
  for (auto& t : th) t.join();
  core.drain();
  poller.join();
  CHECK(polled.load() == 800);
  CHECK(ex.max_arena_end <= 64 * 1024);
  core.stop();
  CHECK(core.arena_free() == 64 * 1024);
}

void test_arena() {
  std::printf("arena\n");
  SrvArena a(4096);
  size_t o1, o2, o3, o4;
  CHECK(a.alloc(1000, &o1) && o1 == 0);
  CHECK(a.alloc(1000, &o2) && o2 == 1024);
  CHECK(a.alloc(2048, &o3) && o3 == 2048);
  CHECK(!a.alloc(1, &o4));
  a.release(o2, 1000);
  CHECK(!a.alloc(2048, &o4));       // 1024 free in the middle only
  a.release(o1, 1000);              // merges with the middle range
  CHECK(a.alloc(2048, &o4) && o4 == 0);
  a.release(o4, 2048);
  a.release(o3, 2048);
  CHECK(a.free_bytes() == 4096);
  CHECK(a.alloc(4096, &o4) && o4 == 0);
}

}  // namespace

int main() {
  test_arena();
  test_burst_batches_by_cell();
  test_oldest_first_across_cells();
  test_future_arrivals_wait();
  test_budget_zero_and_oversized_rejected();
  test_batch_cut_to_budget_and_waits_for_memory();
  test_injected_errors();
  test_cancel();
  test_concurrent_submitters();
  std::printf(g_failures ? "FAILED %d\n" : "ALL PASSED\n", g_failures);
  return g_failures ? 1 : 0;
}
