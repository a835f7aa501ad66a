// Linearised factor trees over arbitrary factor sets (Sec. 4): host form and
// device evaluation (factor_tree.hip).
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>
#include <vector>

namespace mbc {

// The validated tree: children of every vertex as a list (depth-first
// order), the vertices of every depth, and each leaf's coefficient index.
// Within a level, vertices with at most kTreeNarrow children come first
// (level_begin[d] .. level_wide[d]), then the wide ones (.. level_begin[d+1]).
constexpr int kTreeNarrow = 16;
struct TreeHost {
  int64_t n_vertices = 0;
  int32_t n_values = 0, depth = 0;
  std::vector<int32_t> factor, child_begin, child_list, leaf, level_begin, level_wide, level_vertices;
  std::vector<double> coef;  // [n_leaves][2]
  double flops = 0;
};

// Throws std::invalid_argument unless the arrays describe one tree in
// depth-first order with valid factor indices and n_leaves leaves.
void build_tree_host(const int32_t* factors, const int32_t* children, int64_t n_vertices, const double* coef,
                     int64_t n_leaves, int32_t n_values, TreeHost* out);

struct TreeDev {
  int32_t* factor = nullptr;
  int32_t* child_begin = nullptr;
  int32_t* child_list = nullptr;
  int32_t* leaf = nullptr;
  int32_t* level_vertices = nullptr;
  double* coef = nullptr;
};

hipError_t launch_tree_eval(const TreeHost& h, const TreeDev& d, const double* values, int64_t batch, double* out,
                            void* workspace, hipStream_t st);

}  // namespace mbc
