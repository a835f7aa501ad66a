// Linearised factor trees over arbitrary factor sets (Sec. 4): host parse.
//
// The factors / children / coefficients arrays are read in depth-first order
// with an explicit stack of vertices whose children are still to be read.
// That checks that they form exactly one tree and yields each vertex's
// children and depth; vertices are then grouped by depth (narrow ones first)
// for the level-by-level evaluation of factor_tree.hip.
#include <algorithm>
#include <stdexcept>
#include <utility>

#include "factor_tree.hpp"

namespace mbc {

void build_tree_host(const int32_t* factors, const int32_t* children, int64_t n_vertices, const double* coef,
                     int64_t n_leaves, int32_t n_values, TreeHost* out) {
  if (n_vertices < 1 || n_vertices > (int64_t(1) << 30)) throw std::invalid_argument("n_vertices out of range");
  if (n_values < 0 || n_leaves < 0) throw std::invalid_argument("n_values and n_leaves must be >= 0");
  TreeHost& t = *out;
  t = TreeHost();
  t.n_vertices = n_vertices;
  t.n_values = n_values;
  t.factor.assign(factors, factors + n_vertices);
  if (t.factor[0] != -1) throw std::invalid_argument("the root (vertex 0) must have factor -1");
  for (int64_t v = 1; v < n_vertices; ++v)
    if (t.factor[v] < 0 || t.factor[v] >= n_values) throw std::invalid_argument("factor index out of range");
  for (int64_t v = 0; v < n_vertices; ++v)
    if (children[v] < 0) throw std::invalid_argument("negative child count");
  // depth-first parse
  std::vector<int32_t> depth(n_vertices, 0);
  std::vector<std::vector<int32_t>> kids(n_vertices);
  std::vector<std::pair<int32_t, int32_t>> stack;  // (vertex, children still to read)
  stack.push_back({0, children[0]});
  int64_t pos = 1;
  while (!stack.empty()) {
    auto& top = stack.back();
    if (top.second == 0) {
      stack.pop_back();
      continue;
    }
    --top.second;
    if (pos >= n_vertices) throw std::invalid_argument("children counts need more vertices than given");
    const int32_t c = int32_t(pos++);
    kids[top.first].push_back(c);
    depth[c] = depth[top.first] + 1;
    stack.push_back({c, children[c]});
  }
  if (pos != n_vertices) throw std::invalid_argument("vertices left over after the root's subtree");
  t.leaf.assign(n_vertices, -1);
  int64_t l = 0;
  for (int64_t v = 1; v < n_vertices; ++v)
    if (children[v] == 0) t.leaf[v] = int32_t(l++);
  if (l != n_leaves) throw std::invalid_argument("number of leaves differs from the number of coefficients");
  t.coef.assign(coef, coef + 2 * n_leaves);
  t.child_begin.assign(1, 0);
  for (int64_t v = 0; v < n_vertices; ++v) {
    t.child_list.insert(t.child_list.end(), kids[v].begin(), kids[v].end());
    t.child_begin.push_back(int32_t(t.child_list.size()));
  }
  for (int64_t v = 0; v < n_vertices; ++v) t.depth = std::max(t.depth, depth[v]);
  t.level_begin.assign(t.depth + 2, 0);
  for (int64_t v = 0; v < n_vertices; ++v) ++t.level_begin[depth[v] + 1];
  for (int d = 0; d <= t.depth; ++d) t.level_begin[d + 1] += t.level_begin[d];
  // per level: narrow vertices, then wide ones, each in depth-first order
  t.level_vertices.assign(n_vertices, 0);
  t.level_wide.assign(t.depth + 1, 0);
  std::vector<int32_t> fill(t.level_begin.begin(), t.level_begin.end() - 1);
  for (int64_t v = 0; v < n_vertices; ++v)
    if (children[v] <= kTreeNarrow) t.level_vertices[fill[depth[v]]++] = int32_t(v);
  for (int d = 0; d <= t.depth; ++d) t.level_wide[d] = fill[d];
  for (int64_t v = 0; v < n_vertices; ++v)
    if (children[v] > kTreeNarrow) t.level_vertices[fill[depth[v]]++] = int32_t(v);
  t.flops = 8.0 * double(n_vertices - 1);
}

}  // namespace mbc
