// Orderings of the locations (plan time, host). The paper orders components
// before taking nearest preceding neighbours and notes the cost is small
// (Section 3.2); it names no rule. Implemented here:
//   COORD  - lexicographic by (x, y, index).
//   MAXMIN - first the point nearest the bounding-box centre, then repeatedly
//            the unselected point whose squared distance to the selected set is
//            largest; ties go to the lowest index. Distances are compared as
//            d^2 = dx*dx + dy*dy without fused multiply-add, so the result is
//            the exact O(D^2) definition. It is computed in about O(D log D):
//            after a point with distance l is selected, only points within l
//            of it can get closer (every other point is already within l of
//            the set), so only the grid cells meeting that disc are visited;
//            an indexed max-heap keyed by (d^2 desc, index asc) gives the next
//            point. Points are kept in grid-cell order so a visit streams
//            contiguous memory.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <limits>
#include <numeric>
#include <vector>

#include "host_order.h"

#pragma STDC FP_CONTRACT OFF

namespace vecchia {
namespace {

inline double sqd(double ax, double ay, double bx, double by) {
  const double dx = ax - bx;
  const double dy = ay - by;
  const double xx = dx * dx;
  const double yy = dy * dy;
  return xx + yy;
}

// Indexed binary max-heap over slots whose keys only decrease; ties rank the
// lower original index first.
struct MaxHeap {
  std::vector<int32_t> heap;   // heap position -> slot
  std::vector<int32_t> pos;    // slot -> heap position
  const double* key = nullptr;
  const int32_t* id = nullptr; // slot -> original index (tie-break)

  bool before(int32_t a, int32_t b) const {   // a ranks above b
    const double ka = key[a], kb = key[b];
    return ka > kb || (ka == kb && id[a] < id[b]);
  }
  void sift_down(int32_t i) {
    const int32_t n = (int32_t)heap.size();
    const int32_t v = heap[i];
    for (;;) {
      const int32_t l = 2 * i + 1;
      if (l >= n) break;
      int32_t b = l;
      if (l + 1 < n && before(heap[l + 1], heap[l])) b = l + 1;
      if (!before(heap[b], v)) break;
      heap[i] = heap[b];
      pos[heap[i]] = i;
      i = b;
    }
    heap[i] = v;
    pos[v] = i;
  }
  // every slot except the one holding original index `skip`
  void build(int32_t n, int64_t skip) {
    heap.clear();
    heap.reserve(n);
    pos.assign(n, -1);
    for (int32_t q = 0; q < n; ++q)
      if (id[q] != skip) heap.push_back(q);
    for (int32_t i = 0; i < (int32_t)heap.size(); ++i) pos[heap[i]] = i;
    for (int32_t i = (int32_t)heap.size() / 2 - 1; i >= 0; --i) sift_down(i);
  }
  int32_t pop() {
    const int32_t top = heap[0];
    heap[0] = heap.back();
    pos[heap[0]] = 0;
    heap.pop_back();
    if (!heap.empty()) sift_down(0);
    return top;
  }
};

}  // namespace

void order_coord(const double* locs, int64_t D, int64_t* perm) {
  std::vector<int64_t> idx(D);
  std::iota(idx.begin(), idx.end(), 0);
  std::sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) {
    if (locs[2 * a] != locs[2 * b]) return locs[2 * a] < locs[2 * b];
    if (locs[2 * a + 1] != locs[2 * b + 1]) return locs[2 * a + 1] < locs[2 * b + 1];
    return a < b;
  });
  std::copy(idx.begin(), idx.end(), perm);
}

void order_maxmin(const double* locs, int64_t D, int64_t* perm) {
  if (D <= 0) return;
  double x0 = locs[0], x1 = locs[0], y0 = locs[1], y1 = locs[1];
  for (int64_t j = 1; j < D; ++j) {
    x0 = std::min(x0, locs[2 * j]);
    x1 = std::max(x1, locs[2 * j]);
    y0 = std::min(y0, locs[2 * j + 1]);
    y1 = std::max(y1, locs[2 * j + 1]);
  }
  const double cx = (x0 + x1) / 2.0, cy = (y0 + y1) / 2.0;
  int64_t first = 0;
  double best = sqd(locs[0], locs[1], cx, cy);
  for (int64_t j = 1; j < D; ++j) {
    const double d = sqd(locs[2 * j], locs[2 * j + 1], cx, cy);
    if (d < best) {
      best = d;
      first = j;
    }
  }
  perm[0] = first;
  if (D == 1) return;

  // Uniform grid of about 2 points per cell over the bounding box; the points
  // are copied into cell order ("slots") so that a cell's points are contiguous.
  const int64_t G = std::max<int64_t>(1, (int64_t)std::sqrt((double)D / 2.0));
  const double wx = (x1 - x0) > 0 ? (x1 - x0) / (double)G : 1.0;
  const double wy = (y1 - y0) > 0 ? (y1 - y0) / (double)G : 1.0;
  auto cell_x = [&](double v) { return std::min<int64_t>(std::max<int64_t>((int64_t)std::floor((v - x0) / wx), 0), G - 1); };
  auto cell_y = [&](double v) { return std::min<int64_t>(std::max<int64_t>((int64_t)std::floor((v - y0) / wy), 0), G - 1); };
  std::vector<int32_t> start(G * G + 1, 0);
  std::vector<int32_t> cell(D);
  for (int64_t j = 0; j < D; ++j) {
    cell[j] = (int32_t)(cell_x(locs[2 * j]) * G + cell_y(locs[2 * j + 1]));
    ++start[cell[j] + 1];
  }
  for (int64_t c = 0; c < G * G; ++c) start[c + 1] += start[c];
  std::vector<double> px(D), py(D), mind2(D);
  std::vector<int32_t> id(D);
  {
    std::vector<int32_t> fill(start.begin(), start.end() - 1);
    for (int64_t j = 0; j < D; ++j) {
      const int32_t q = fill[cell[j]]++;
      px[q] = locs[2 * j];
      py[q] = locs[2 * j + 1];
      id[q] = (int32_t)j;
    }
  }
  // a selected slot's key is -inf: no distance is below it, and it is never
  // compared again
  const double fx = locs[2 * first], fy = locs[2 * first + 1];
  for (int64_t q = 0; q < D; ++q) mind2[q] = id[q] == first ? -INFINITY : sqd(px[q], py[q], fx, fy);
  MaxHeap h;
  h.key = mind2.data();
  h.id = id.data();
  h.build((int32_t)D, first);
  // a point can only move closer to the set through the newly selected point s
  // if its distance to s is below l = sqrt(mind2[s]) (every other point is
  // already within l of the set); the cells meeting the disc of radius l' > l
  // are visited, l' enlarged by a relative and an absolute margin against the
  // rounding of the cell bounds
  const double span = std::max(std::max(std::fabs(x0), std::fabs(x1)), std::max(std::fabs(y0), std::fabs(y1)));
  const double abs_margin = 8.0 * span * std::numeric_limits<double>::epsilon();
  for (int64_t t = 1; t < D; ++t) {
    const int32_t s = h.pop();
    perm[t] = id[s];
    const double l2 = mind2[s];
    mind2[s] = -INFINITY;
    if (!(l2 > 0.0)) continue;   // duplicates of selected points: nothing can improve
    const double sx = px[s], sy = py[s];
    const double l = std::sqrt(l2) * (1.0 + 1e-9) + abs_margin;
    const int64_t ax = cell_x(sx - l), bx = cell_x(sx + l);
    const int64_t ay = cell_y(sy - l), by = cell_y(sy + l);
    for (int64_t gx = ax; gx <= bx; ++gx) {
      const int32_t q0 = start[gx * G + ay], q1 = start[gx * G + by + 1];   // cells (gx, ay..by) are contiguous
      for (int32_t q = q0; q < q1; ++q) {
        const double d = sqd(px[q], py[q], sx, sy);
        if (d < mind2[q]) {
          mind2[q] = d;
          h.sift_down(h.pos[q]);
        }
      }
    }
  }
}

}  // namespace vecchia
