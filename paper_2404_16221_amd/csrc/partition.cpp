// Spatial partitioning (Sec. 4.4, App. A.3): recursive splits of a point set
// at the plane where the per-axis CDF reaches one half, keeping at each node
// the axis whose two children are closest to cubic.  A one-off preprocess
// over a point cloud (structure-from-motion points, or samples of random
// training rays), run on the host: O(n) selections per level.
//
// Tree layout (shared with the pack kernels): heap order, node i has children
// 2i+1 (coordinate below the plane) and 2i+2 (at or above it); box b is leaf
// node b + 2^levels - 1.  The outermost boxes are unbounded.
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"

namespace {

struct Builder {
  const float* pts;
  int levels;
  int32_t* axis;
  float* plane;
  std::vector<float> coord;  // selection buffer

  // longest over shortest extent; a flat box is infinitely elongated, a point
  // box counts as cubic
  static double ratio(const double e[3]) {
    const double mx = std::max(e[0], std::max(e[1], e[2]));
    const double mn = std::min(e[0], std::min(e[1], e[2]));
    if (mn == 0.0) return mx == 0.0 ? 1.0 : INFINITY;
    return mx / mn;
  }

  void split(int64_t node, int64_t* idx, int64_t m, const double lo[3], const double hi[3],
             int depth) {
    if (depth == levels) return;
    double best_score = 0.0;
    int best_axis = -1;
    float best_cut = 0.f;
    for (int a = 0; a < 3; ++a) {
      float cut;
      if (m > 0) {
        coord.resize(static_cast<size_t>(m));
        for (int64_t i = 0; i < m; ++i) coord[i] = pts[3 * idx[i] + a];
        std::nth_element(coord.begin(), coord.begin() + m / 2, coord.end());
        cut = coord[m / 2];  // order statistic of rank floor(m/2): the CDF-1/2 plane
      } else {
        cut = static_cast<float>((lo[a] + hi[a]) / 2.0);
      }
      double el[3], eh[3];
      for (int c = 0; c < 3; ++c) el[c] = eh[c] = hi[c] - lo[c];
      el[a] = static_cast<double>(cut) - lo[a];
      eh[a] = hi[a] - static_cast<double>(cut);
      const double score = std::max(ratio(el), ratio(eh));
      if (best_axis < 0 || score < best_score) {
        best_score = score;
        best_axis = a;
        best_cut = cut;
      }
    }
    axis[node] = best_axis;
    plane[node] = best_cut;
    const int a = best_axis;
    int64_t* mid = std::partition(idx, idx + m, [&](int64_t i) { return pts[3 * i + a] < best_cut; });
    const int64_t m_low = mid - idx;
    double hi_low[3] = {hi[0], hi[1], hi[2]}, lo_high[3] = {lo[0], lo[1], lo[2]};
    hi_low[a] = lo_high[a] = static_cast<double>(best_cut);
    split(2 * node + 1, idx, m_low, lo, hi_low, depth + 1);
    split(2 * node + 2, mid, m - m_low, lo_high, hi, depth + 1);
  }
};

}  // namespace

namespace xl {

int partition_build(const float* points, int64_t n, int levels, int32_t* axis, float* plane) {
  double lo[3] = {0.0, 0.0, 0.0}, hi[3] = {0.0, 0.0, 0.0};
  for (int64_t i = 0; i < n; ++i)
    for (int c = 0; c < 3; ++c) {
      const float v = points[3 * i + c];
      if (!std::isfinite(v)) return XL_EINVAL;
      if (i == 0 || v < lo[c]) lo[c] = v;
      if (i == 0 || v > hi[c]) hi[c] = v;
    }
  std::vector<int64_t> idx(static_cast<size_t>(n));
  for (int64_t i = 0; i < n; ++i) idx[i] = i;
  Builder b{points, levels, axis, plane, {}};
  b.split(0, idx.data(), n, lo, hi, 0);
  return XL_OK;
}

}  // namespace xl
