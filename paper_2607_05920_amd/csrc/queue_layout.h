// Layout of stage-batched launches (host only, no HIP types).
//
// A stage-batched batch plan records every cell's pipeline (one launch per step, the
// same steps for every cell) and runs step s of all cells together: one launch per
// (graph branch, kernel variant) over the cells of that branch using that variant.
// This header decides which cells go into which launch and where each cell's
// workgroups sit in it; the device side finds a workgroup's cell by a binary search
// over the segment offsets (cell_of in the kernels).
#pragma once

#include <cstdint>
#include <vector>

namespace fhe {

// One recorded launch: its kernel variant (entry point and workgroup shape), grid, and
// the graph branch of its cell.
struct QRec {
  const void* variant = nullptr;
  uint32_t bx = 0, by = 0, bz = 0;  // workgroup shape
  uint32_t gx = 0, gy = 0, gz = 0;  // grid of the cell's own launch
  uint32_t arg_bytes = 0;           // size of its argument struct
  int branch = 0;
};

// A cell's segment: first workgroup (a multiple of 8) and the grid of its own launch.
struct QSeg {
  uint32_t off = 0, gx = 0, gy = 0;
  int cell = 0;
};

struct QLaunch {
  int step = 0, branch = 0;
  const void* variant = nullptr;
  uint32_t blocks = 0;  // the segments end to end, each rounded up to 8 workgroups
  std::vector<QSeg> segs;
};

enum { QL_OK = 0, QL_MISMATCH = 1, QL_TOO_BIG = 2 };

// recs[c][s]: cell c's launch at step s.  Launches come out step by step; within a
// step, cells are visited in order for even steps and in reverse for odd ones (a step
// then starts on the cells whose data the step before wrote last), and each launch
// takes, from its first cell on in that order, every cell of the same branch and
// variant.  Rounding each segment to 8 workgroups keeps a workgroup on the XCD
// (blockIdx mod 8) its own launch would give it.
inline int queue_layout(const std::vector<std::vector<QRec>>& recs, std::vector<QLaunch>* out) {
  out->clear();
  const size_t nc = recs.size();
  if (nc == 0) return QL_OK;
  const size_t nsteps = recs[0].size();
  for (size_t c = 1; c < nc; ++c)
    if (recs[c].size() != nsteps) return QL_MISMATCH;
  for (size_t s = 0; s < nsteps; ++s) {
    std::vector<size_t> ord(nc);
    for (size_t i = 0; i < nc; ++i) ord[i] = (s & 1) ? nc - 1 - i : i;
    std::vector<char> done(nc, 0);
    for (size_t i0 = 0; i0 < nc; ++i0) {
      const size_t c0 = ord[i0];
      if (done[c0]) continue;
      const QRec& r0 = recs[c0][s];
      QLaunch L;
      L.step = (int)s;
      L.branch = r0.branch;
      L.variant = r0.variant;
      unsigned long long off = 0;
      for (size_t i = i0; i < nc; ++i) {
        const size_t ci = ord[i];
        const QRec& r = recs[ci][s];
        if (done[ci] || r.branch != r0.branch || r.variant != r0.variant || r.bx != r0.bx || r.by != r0.by ||
            r.bz != r0.bz)
          continue;
        if (r.arg_bytes != r0.arg_bytes || r.gz != 1) return QL_MISMATCH;
        done[ci] = 1;
        QSeg sg;
        sg.off = (uint32_t)off;
        sg.gx = r.gx;
        sg.gy = r.gy;
        sg.cell = (int)ci;
        off += ((unsigned long long)r.gx * r.gy + 7) & ~7ull;
        if (off > 0x7FFFFFFFull) return QL_TOO_BIG;
        L.segs.push_back(sg);
      }
      L.blocks = (uint32_t)off;
      out->push_back(std::move(L));
    }
  }
  return QL_OK;
}

// The host form of the device lookup: the segment holding workgroup w (the last with
// off <= w), or -1 for a workgroup in a segment's rounding.
inline int queue_cell_of(const std::vector<QSeg>& segs, uint32_t w, uint32_t* x, uint32_t* y) {
  int lo = 0, hi = (int)segs.size();
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (segs[mid].off <= w) lo = mid;
    else hi = mid;
  }
  const QSeg& sg = segs[lo];
  const uint32_t l = w - sg.off;
  if (l >= sg.gx * sg.gy) return -1;
  *x = l % sg.gx;
  *y = l / sg.gx;
  return lo;
}

}  // namespace fhe
