// Cluster tree, block cluster tree and translation classes.
//
// Sec. 3.2 / Alg. ConstructClusterTree (arxiv 2511.03109): the box of a node is
// halved along every axis; a point with x_k <= midpoint goes to the lower half.
// Children are created in little-endian child-id order (axis 1 least
// significant), only when they hold a point, and every node below l_max is
// split, so all leaves sit at l_max.  Built breadth first, so node ids come out
// ordered by (level, parent id, child id) and the leaves of the last level are in
// depth-first order, which is the tree order of the points.
//
// Sec. 3.3 / Alg. ConstructBlockClusterTree with the admissibility condition
// max(diam) <= eta dist.  Pairs are always at equal level with equal box sides h,
// so diam^2 = d h^2 and dist^2 = h^2 sum_k g_k^2 with g_k = max(0, |k_s - k_t| - 1)
// box widths of empty space along axis k; the test is done exactly in integers:
// d * eta2_den <= eta2_num * sum_k g_k^2 (equality admissible).
//
// Sec. 5.2: far blocks with the same (level, offset k_t - k_s) share the far
// tensor of a stationary kernel (translation classes).
#include <algorithm>
#include <cmath>
#include <map>

#include "ph_host.hpp"

namespace ph {

std::shared_ptr<TreeData> build_tree(const double* pts, int64_t n, const ph_tree_opts& o) {
  if (!pts) fail(PH_EINVAL, "ph_build_tree: pts is NULL");
  if (n < 1) fail(PH_EINVAL, "ph_build_tree: n must be >= 1");
  if (o.d < 1 || o.d > 3) fail(PH_EINVAL, "ph_build_tree: d must be 1, 2 or 3");
  if (!(o.lo < o.hi)) fail(PH_EINVAL, "ph_build_tree: need lo < hi");
  if (o.eta2_num <= 0 || o.eta2_den <= 0) fail(PH_EINVAL, "ph_build_tree: eta^2 must be positive");
  const int d = o.d;
  for (int64_t i = 0; i < n * d; ++i) {
    double v = pts[i];
    if (std::isnan(v)) fail(PH_EINVAL, "ph_build_tree: NaN coordinate");
    if (v < o.lo || v > o.hi) fail(PH_EINVAL, "ph_build_tree: point outside [lo, hi]^d");
  }
  int l_max = o.l_max;
  if (l_max < 0) {
    if (o.leaf_size < 1) fail(PH_EINVAL, "ph_build_tree: leaf_size must be >= 1 when l_max < 0");
    l_max = 0;
    while ((double)n > (double)o.leaf_size * std::ldexp(1.0, d * l_max)) ++l_max;
  }
  if (l_max > 20) fail(PH_EINVAL, "ph_build_tree: l_max > 20");

  auto t = std::make_shared<TreeData>();
  t->n = n; t->d = d; t->l_max = l_max; t->lo = o.lo; t->hi = o.hi;
  t->eta2_num = o.eta2_num; t->eta2_den = o.eta2_den;

  // node point lists, breadth first
  std::vector<std::vector<int64_t>> idx;
  idx.emplace_back(n);
  for (int64_t i = 0; i < n; ++i) idx[0][i] = i;
  t->level.push_back(0);
  t->parent.push_back(-1);
  t->cid.push_back(0);
  for (int k = 0; k < d; ++k) {
    t->coords.push_back(0);
    t->box_lo.push_back(o.lo);
    t->box_hi.push_back(o.hi);
  }
  t->level_start.push_back(0);
  int32_t lev_begin = 0, lev_end = 1;
  for (int lev = 0; lev < l_max; ++lev) {
    t->level_start.push_back(lev_end);
    for (int32_t s = lev_begin; s < lev_end; ++s) {
      double mid[3];
      for (int k = 0; k < d; ++k) mid[k] = (t->box_lo[s * d + k] + t->box_hi[s * d + k]) / 2.0;
      const int nc = 1 << d;
      std::vector<std::vector<int64_t>> ch(nc);
      for (int64_t i : idx[s]) {
        int c = 0;
        for (int k = 0; k < d; ++k)
          if (pts[i * d + k] > mid[k]) c |= 1 << k;
        ch[c].push_back(i);  // stable: keeps the parent's order
      }
      t->first_child.resize(s + 1, -1);
      t->nchild.resize(s + 1, 0);
      t->first_child[s] = (int32_t)t->level.size();
      for (int c = 0; c < nc; ++c) {
        if (ch[c].empty()) continue;
        const int32_t id = (int32_t)t->level.size();
        t->level.push_back(lev + 1);
        t->parent.push_back(s);
        t->cid.push_back(c);
        for (int k = 0; k < d; ++k) {
          const bool up = (c >> k) & 1;
          t->coords.push_back(2 * t->coords[s * d + k] + (up ? 1 : 0));
          t->box_lo.push_back(up ? mid[k] : t->box_lo[s * d + k]);
          t->box_hi.push_back(up ? t->box_hi[s * d + k] : mid[k]);
        }
        idx.push_back(std::move(ch[c]));
        t->nchild[s]++;
        (void)id;
      }
    }
    lev_begin = lev_end;
    lev_end = (int32_t)t->level.size();
  }
  t->level_start.push_back(lev_end);
  const int64_t nn = (int64_t)t->level.size();
  t->first_child.resize(nn, -1);
  t->nchild.resize(nn, 0);

  // leaves (all at l_max) in id order = tree order
  t->begin.assign(nn, 0);
  t->end.assign(nn, 0);
  t->perm.resize(n);
  t->pts_t.resize(n * d);
  int64_t pos = 0;
  for (int32_t s = lev_begin; s < lev_end; ++s) {
    t->leaves.push_back(s);
    t->begin[s] = pos;
    for (int64_t i : idx[s]) {
      t->perm[pos] = i;
      for (int k = 0; k < d; ++k) t->pts_t[pos * d + k] = pts[i * d + k];
      ++pos;
    }
    t->end[s] = pos;
  }
  for (int64_t s = lev_begin - 1; s >= 0; --s) {
    int32_t f = t->first_child[s];
    t->begin[s] = t->begin[f];
    t->end[s] = t->end[f + t->nchild[s] - 1];
  }

  // block cluster tree
  auto admissible = [&](int32_t s, int32_t u) {
    int64_t g2 = 0;
    for (int k = 0; k < d; ++k) {
      int64_t diff = std::llabs((int64_t)t->coords[s * d + k] - (int64_t)t->coords[u * d + k]);
      int64_t g = diff > 0 ? diff - 1 : 0;
      g2 += g * g;
    }
    return (int64_t)d * t->eta2_den <= (int64_t)t->eta2_num * g2;
  };
  std::vector<std::pair<int32_t, int32_t>> stack{{0, 0}}, near, far;
  while (!stack.empty()) {
    auto [s, u] = stack.back();
    stack.pop_back();
    bool a = admissible(s, u);
    if (!a && t->nchild[s] > 0 && t->nchild[u] > 0) {
      for (int32_t cs = 0; cs < t->nchild[s]; ++cs)
        for (int32_t cu = 0; cu < t->nchild[u]; ++cu)
          stack.push_back({t->first_child[s] + cs, t->first_child[u] + cu});
    } else if (a) {
      far.push_back({s, u});
    } else {
      near.push_back({s, u});
    }
  }
  auto key = [&](const std::pair<int32_t, int32_t>& b) {
    return std::make_tuple(t->level[b.first], b.first, b.second);
  };
  auto cmp = [&](const auto& a, const auto& b) { return key(a) < key(b); };
  std::sort(near.begin(), near.end(), cmp);
  std::sort(far.begin(), far.end(), cmp);
  for (auto& b : near) {
    t->near.push_back(b.first);
    t->near.push_back(b.second);
    t->near_entries += t->size(b.first) * t->size(b.second);
  }
  std::map<std::vector<int32_t>, int32_t> cls;
  std::vector<std::vector<int32_t>> fkeys;
  for (auto& b : far) {
    t->far.push_back(b.first);
    t->far.push_back(b.second);
    std::vector<int32_t> kk{t->level[b.first]};
    for (int k = 0; k < d; ++k) kk.push_back(t->coords[b.second * d + k] - t->coords[b.first * d + k]);
    fkeys.push_back(kk);
    cls.emplace(kk, 0);
  }
  int32_t ci = 0;
  for (auto& kv : cls) {
    kv.second = ci++;
    t->class_level.push_back(kv.first[0]);
    for (int k = 0; k < d; ++k) t->class_off.push_back(kv.first[1 + k]);
  }
  t->class_first_block.assign(ci, -1);
  for (size_t b = 0; b < fkeys.size(); ++b) {
    int32_t c = cls[fkeys[b]];
    t->far_class.push_back(c);
    if (t->class_first_block[c] < 0) t->class_first_block[c] = (int32_t)b;
  }
  t->min_far_level = far.empty() ? -1 : t->level[far.front().first];
  return t;
}

}  // namespace ph
