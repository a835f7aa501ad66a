// Linearised factor trees over arbitrary factor sets (Sec. 4): device
// evaluation of a tree parsed by factor_tree.cpp.  The tree is evaluated
// bottom up, deepest level first: a vertex's value is its factor's
// value (1 for the root) times its leaf coefficient or the sum of its
// children's values: one thread per (table, vertex) for vertices with few
// children, a wavefront per (table, vertex) for the others (its lanes
// stride over the children and combine in a fixed butterfly).  The root's
// value is the tree's.
#include <hip/hip_runtime.h>

#include "factor_tree.hpp"

namespace mbc {

namespace {

constexpr int kTT = 256;

struct TreeArgs {
  const int32_t* factor;
  const int32_t* child_begin;
  const int32_t* child_list;
  const int32_t* leaf;
  const double2* coef;
  const double2* values;
  double2* vals;  // workspace [batch][n_vertices]
  double2* out;
  int64_t n_vertices, batch;
  int32_t n_values;
};

// G lanes per (table, vertex): lane l sums children l, l + G, ..; the G
// partial sums are combined by a fixed butterfly within the wavefront
template <int G>
__global__ __launch_bounds__(kTT) void tree_level_kernel(TreeArgs a, const int32_t* verts, int n, int root) {
  const int64_t idx = (int64_t(blockIdx.x) * kTT + threadIdx.x) / G;
  const int lane = int(threadIdx.x) % G;
  const bool live = idx < int64_t(n) * a.batch;
  int64_t b = 0;
  int32_t v = 0;
  double2 s = make_double2(0, 0);
  if (live) {
    b = idx / n;
    v = verts[idx - b * n];
    if (a.leaf[v] >= 0) {
      if (lane == 0) s = a.coef[a.leaf[v]];
    } else {
      const double2* row = a.vals + b * a.n_vertices;
      for (int32_t c = a.child_begin[v] + lane; c < a.child_begin[v + 1]; c += G) {
        const double2 x = row[a.child_list[c]];
        s.x += x.x;
        s.y += x.y;
      }
    }
  }
  if constexpr (G > 1) {
    for (int w = G / 2; w > 0; w >>= 1) {
      s.x += __shfl_xor(s.x, w, G);
      s.y += __shfl_xor(s.y, w, G);
    }
  }
  if (!live || lane != 0) return;
  double2 r = s;
  if (a.factor[v] >= 0) {
    const double2 f = a.values[b * a.n_values + a.factor[v]];
    r = make_double2(f.x * s.x - f.y * s.y, f.x * s.y + f.y * s.x);
  }
  if (root)
    a.out[b] = r;
  else
    a.vals[b * a.n_vertices + v] = r;
}

}  // namespace

hipError_t launch_tree_eval(const TreeHost& h, const TreeDev& d, const double* values, int64_t batch, double* out,
                            void* workspace, hipStream_t st) {
  TreeArgs a{};
  a.factor = d.factor;
  a.child_begin = d.child_begin;
  a.child_list = d.child_list;
  a.leaf = d.leaf;
  a.coef = reinterpret_cast<const double2*>(d.coef);
  a.values = reinterpret_cast<const double2*>(values);
  a.vals = reinterpret_cast<double2*>(workspace);
  a.out = reinterpret_cast<double2*>(out);
  a.n_vertices = h.n_vertices;
  a.batch = batch;
  a.n_values = h.n_values;
  for (int dd = h.depth; dd >= 0; --dd) {
    const int n_narrow = h.level_wide[dd] - h.level_begin[dd];
    const int n_wide = h.level_begin[dd + 1] - h.level_wide[dd];
    if (n_narrow > 0) {
      const unsigned nb = unsigned((int64_t(n_narrow) * batch + kTT - 1) / kTT);
      hipLaunchKernelGGL((tree_level_kernel<1>), dim3(nb), dim3(kTT), 0, st, a, d.level_vertices + h.level_begin[dd],
                         n_narrow, dd == 0 ? 1 : 0);
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    if (n_wide > 0) {
      const unsigned nb = unsigned((int64_t(n_wide) * batch * 64 + kTT - 1) / kTT);
      hipLaunchKernelGGL((tree_level_kernel<64>), dim3(nb), dim3(kTT), 0, st, a, d.level_vertices + h.level_wide[dd],
                         n_wide, dd == 0 ? 1 : 0);
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

}  // namespace mbc
