// CPU test of the stage-batched launch layout (queue_layout.h): random cell mixes of
// several branches and kernel variants, checked for the invariants the device lookup
// relies on, and every workgroup of every launch looked up back to its cell.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>
#include <tuple>
#include <vector>

#include "queue_layout.h"

using namespace fhe;

static int failures = 0;
#define CHECK(c)                                                  \
  do {                                                            \
    if (!(c)) {                                                   \
      std::printf("FAIL %s:%d: %s\n", __FILE__, __LINE__, #c);    \
      ++failures;                                                 \
    }                                                             \
  } while (0)

static const int kVariants[4] = {0, 0, 0, 0};  // distinct addresses stand for variants

static void check_layout(const std::vector<std::vector<QRec>>& recs, const std::vector<QLaunch>& lay) {
  const size_t nc = recs.size(), ns = nc ? recs[0].size() : 0;
  // every (cell, step) in exactly one launch of its step, branch and variant
  std::vector<std::vector<int>> seen(nc, std::vector<int>(ns, 0));
  int prev_step = 0;
  for (const QLaunch& L : lay) {
    CHECK(L.step >= prev_step);  // steps in order
    prev_step = L.step;
    CHECK(!L.segs.empty());
    uint32_t end = 0;
    for (size_t i = 0; i < L.segs.size(); ++i) {
      const QSeg& g = L.segs[i];
      const QRec& r = recs[g.cell][L.step];
      CHECK(g.off % 8 == 0);
      CHECK(g.off == end);  // segments end to end
      CHECK(g.gx == r.gx && g.gy == r.gy);
      CHECK(r.branch == L.branch && r.variant == L.variant);
      end = g.off + ((g.gx * g.gy + 7) & ~7u);
      seen[g.cell][L.step]++;
    }
    CHECK(L.blocks == end);
    // cells in order on even steps, reverse on odd ones
    for (size_t i = 1; i < L.segs.size(); ++i)
      CHECK((L.step & 1) ? L.segs[i].cell < L.segs[i - 1].cell : L.segs[i].cell > L.segs[i - 1].cell);
    // every workgroup finds its segment; the rounding workgroups find none
    for (uint32_t w = 0; w < L.blocks; ++w) {
      uint32_t x = 0, y = 0;
      const int k = queue_cell_of(L.segs, w, &x, &y);
      int want = -1;
      for (size_t i = 0; i < L.segs.size(); ++i)
        if (w >= L.segs[i].off && w < L.segs[i].off + L.segs[i].gx * L.segs[i].gy) want = (int)i;
      CHECK(k == want);
      if (k >= 0) {
        const QSeg& g = L.segs[k];
        CHECK(x < g.gx && y < g.gy && g.off + y * g.gx + x == w);
        CHECK((w & 7) == ((y * g.gx + x) & 7));  // the XCD of its own launch
      }
    }
  }
  for (size_t c = 0; c < nc; ++c)
    for (size_t s = 0; s < ns; ++s) CHECK(seen[c][s] == 1);
}

int main() {
  std::mt19937 rng(7);
  // random mixes: 1..20 cells, 11 steps, up to 4 branches and 3 variants per step
  for (int trial = 0; trial < 200; ++trial) {
    const int nc = 1 + (int)(rng() % 20), ns = 11;
    const int nbr = 1 + (int)(rng() % 4);
    std::vector<std::vector<QRec>> recs(nc, std::vector<QRec>(ns));
    for (int c = 0; c < nc; ++c) {
      const int br = (int)(rng() % nbr);
      for (int s = 0; s < ns; ++s) {
        QRec& r = recs[c][s];
        const int v = (int)(rng() % 3);
        r.variant = &kVariants[v];
        r.bx = v == 2 ? 256 : 128;
        r.by = 1;
        r.bz = 1;
        r.gx = 1 + (uint32_t)(rng() % 300);
        r.gy = 1 + (uint32_t)(rng() % 3);
        r.gz = 1;
        r.arg_bytes = 64 * (1 + v);
        r.branch = br;
      }
    }
    std::vector<QLaunch> lay;
    CHECK(queue_layout(recs, &lay) == QL_OK);
    check_layout(recs, lay);
    // one launch per (step, branch, variant) in use
    std::set<std::tuple<int, int, const void*>> keys;
    for (int c = 0; c < nc; ++c)
      for (int s = 0; s < ns; ++s) keys.insert(std::make_tuple(s, recs[c][s].branch, recs[c][s].variant));
    CHECK(lay.size() == keys.size());
  }
  // a pipeline with a different number of steps, and a variant whose argument size
  // differs between cells, are refused
  {
    std::vector<std::vector<QRec>> recs(2, std::vector<QRec>(3));
    for (auto& cell : recs)
      for (auto& r : cell) {
        r.variant = &kVariants[0];
        r.gx = r.gy = r.gz = 1;
        r.arg_bytes = 8;
      }
    std::vector<QLaunch> lay;
    CHECK(queue_layout(recs, &lay) == QL_OK);
    recs[1][2].arg_bytes = 16;
    CHECK(queue_layout(recs, &lay) == QL_MISMATCH);
    recs[1][2].arg_bytes = 8;
    recs[1][1].gz = 2;
    CHECK(queue_layout(recs, &lay) == QL_MISMATCH);
    recs[1][1].gz = 1;
    recs[1].pop_back();
    CHECK(queue_layout(recs, &lay) == QL_MISMATCH);
  }
  // a launch past 2^31 workgroups is refused
  {
    std::vector<std::vector<QRec>> recs(3, std::vector<QRec>(1));
    for (auto& cell : recs) {
      cell[0].variant = &kVariants[0];
      cell[0].gx = 1u << 30;
      cell[0].gy = 1;
      cell[0].gz = 1;
    }
    std::vector<QLaunch> lay;
    CHECK(queue_layout(recs, &lay) == QL_TOO_BIG);
  }
  // no cells: no launches
  {
    std::vector<std::vector<QRec>> recs;
    std::vector<QLaunch> lay(1);
    CHECK(queue_layout(recs, &lay) == QL_OK && lay.empty());
  }
  if (failures) {
    std::printf("%d FAILURES\n", failures);
    return 1;
  }
  std::printf("ALL PASSED\n");
  return 0;
}
