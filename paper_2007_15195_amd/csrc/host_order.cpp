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
//            point.
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

// Indexed binary max-heap over point ids with keys that only decrease.
struct MaxHeap {
  std::vector<int64_t> heap;   // heap position -> point
  std::vector<int64_t> pos;    // point -> heap position, -1 when removed
  const std::vector<double>* key;

  bool before(int64_t a, int64_t b) const {   // a ranks above b
    const double ka = (*key)[a], kb = (*key)[b];
    return ka > kb || (ka == kb && a < b);
  }
  void swap_at(int64_t i, int64_t j) {
    std::swap(heap[i], heap[j]);
    pos[heap[i]] = i;
    pos[heap[j]] = j;
  }
  void sift_down(int64_t i) {
    const int64_t n = (int64_t)heap.size();
    for (;;) {
      int64_t b = i;
      const int64_t l = 2 * i + 1, r = 2 * i + 2;
      if (l < n && before(heap[l], heap[b])) b = l;
      if (r < n && before(heap[r], heap[b])) b = r;
      if (b == i) return;
      swap_at(i, b);
      i = b;
    }
  }
  void build(const std::vector<int64_t>& items) {
    heap = items;
    for (int64_t i = 0; i < (int64_t)heap.size(); ++i) pos[heap[i]] = i;
    for (int64_t i = (int64_t)heap.size() / 2 - 1; i >= 0; --i) sift_down(i);
  }
  int64_t pop() {
    const int64_t top = heap[0];
    swap_at(0, (int64_t)heap.size() - 1);
    heap.pop_back();
    pos[top] = -1;
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

  // uniform grid of about 2 points per cell over the bounding box
  const int64_t G = std::max<int64_t>(1, (int64_t)std::sqrt((double)D / 2.0));
  const double wx = (x1 - x0) > 0 ? (x1 - x0) / (double)G : 1.0;
  const double wy = (y1 - y0) > 0 ? (y1 - y0) / (double)G : 1.0;
  auto cell_of = [&](double v, double lo, double w) {
    int64_t c = (int64_t)std::floor((v - lo) / w);
    return std::min<int64_t>(std::max<int64_t>(c, 0), G - 1);
  };
  std::vector<int64_t> start(G * G + 1, 0), items(D);
  std::vector<int64_t> cx_of(D), cy_of(D);
  for (int64_t j = 0; j < D; ++j) {
    cx_of[j] = cell_of(locs[2 * j], x0, wx);
    cy_of[j] = cell_of(locs[2 * j + 1], y0, wy);
    ++start[cx_of[j] * G + cy_of[j] + 1];
  }
  for (int64_t c = 0; c < G * G; ++c) start[c + 1] += start[c];
  {
    std::vector<int64_t> fillp(start.begin(), start.end() - 1);
    for (int64_t j = 0; j < D; ++j) items[fillp[cx_of[j] * G + cy_of[j]]++] = j;
  }

  std::vector<double> mind2(D);
  std::vector<char> taken(D, 0);
  const double fx = locs[2 * first], fy = locs[2 * first + 1];
  for (int64_t j = 0; j < D; ++j) mind2[j] = sqd(locs[2 * j], locs[2 * j + 1], fx, fy);
  taken[first] = 1;
  MaxHeap h;
  h.key = &mind2;
  h.pos.assign(D, -1);
  {
    std::vector<int64_t> rest;
    rest.reserve(D - 1);
    for (int64_t j = 0; j < D; ++j)
      if (j != first) rest.push_back(j);
    h.build(rest);
  }
  for (int64_t t = 1; t < D; ++t) {
    const int64_t s = h.pop();
    perm[t] = s;
    taken[s] = 1;
    const double sx = locs[2 * s], sy = locs[2 * s + 1];
    // Points with d(j, s) >= l cannot improve (mind2[j] <= l^2). Visit the cells
    // meeting the disc of radius l (plus one cell of margin against rounding).
    const double l = std::sqrt(mind2[s]) * (1.0 + 1e-12);
    const int64_t ax = std::max<int64_t>(0, (int64_t)std::floor((sx - l - x0) / wx) - 1);
    const int64_t bx = std::min<int64_t>(G - 1, (int64_t)std::floor((sx + l - x0) / wx) + 1);
    const int64_t ay = std::max<int64_t>(0, (int64_t)std::floor((sy - l - y0) / wy) - 1);
    const int64_t by = std::min<int64_t>(G - 1, (int64_t)std::floor((sy + l - y0) / wy) + 1);
    for (int64_t gx = ax; gx <= bx; ++gx) {
      for (int64_t gy = ay; gy <= by; ++gy) {
        const int64_t c = gx * G + gy;
        for (int64_t q = start[c]; q < start[c + 1]; ++q) {
          const int64_t j = items[q];
          if (taken[j]) continue;
          const double d = sqd(locs[2 * j], locs[2 * j + 1], sx, sy);
          if (d < mind2[j]) {
            mind2[j] = d;
            h.sift_down(h.pos[j]);
          }
        }
      }
    }
  }
}

}  // namespace vecchia
