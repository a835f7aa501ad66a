// Tensor e-graphs (Sec. 5): host data structures shared by the planner, the
// block-correlator expression builder, the C ABI and the device executor.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/mbc_egraph.h"

namespace mbc {

// One element of a tensor's symmetry group: T[x_p0, x_p1, ..] = s T[x].
struct SymElem {
  uint8_t p[MBC_EGRAPH_MAX_RANK];
  int8_t s;
};

struct TensorInfo {
  int rank = 0;
  int ext[MBC_EGRAPH_MAX_RANK] = {};
  std::vector<SymElem> group;  // closure of the generators, identity first
};

struct Fac {
  int t = 0;
  uint8_t lab[MBC_EGRAPH_MAX_RANK] = {};
};
using Expr = std::vector<Fac>;

// A sum of tensor expressions as handed to the planner.
struct TensorProblem {
  std::vector<mbc_tensor_decl> decls;
  std::vector<std::vector<double>> constant;  // per tensor: library values (complex128), or empty
  std::vector<mbc_tensor_factor> factors;
  std::vector<int32_t> term_begin;            // [n_terms + 1]
  std::vector<double> coef;                   // [n_terms][2]
};

// E = sign x child1[o1] child2[o2]: child k's open slot j is E's label ok[j].
struct ENode {
  int c1 = -1, c2 = -1, sign = 1;
  std::vector<uint8_t> o1, o2;
};

struct EClass {
  std::vector<int16_t> code;  // canonical code
  Expr factors;               // canonical expression (labels = codes)
  int n_open = 0;
  std::vector<int> open_ext;  // extent of open slot k (label 2k + 1)
  int label_ext[MBC_EGRAPH_MAX_LABEL] = {};
  uint64_t labels = 0;        // bit mask of the labels used
  std::vector<ENode> nodes;
};

struct TermRoot {
  int cls = -1;
  double re = 0, im = 0;       // coefficient x canonical sign
  std::vector<uint8_t> opens;  // caller label of the class's open slot k
};

struct Step {
  int cls = -1, node = -1;
  int64_t ws_off = 0, elems = 0;  // output in the workspace, per batch entry
};

struct EGraphHost {
  std::vector<TensorInfo> tensors;
  std::vector<EClass> cls;                  // M
  std::vector<int> parent;                  // U
  std::unordered_map<std::string, int> H;   // hash-cons: canonical codes and e-nodes -> class
  std::vector<int> work;
  size_t work_head = 0;
  int64_t n_nodes = 0;
  bool saturated = true;
  std::vector<TermRoot> terms;              // one per input term (vanishing terms dropped)
  int n_input_terms = 0;
  std::vector<TermRoot> roots;              // terms merged by (class, open map)
  std::vector<Step> steps;
  std::vector<int> step_of;                 // class -> step index (-1: leaf / not extracted)
  std::vector<uint8_t> out_labels;          // result's open labels, increasing
  std::vector<int> out_ext;
  int64_t out_elems = 1, ws_elems = 0;
  double flops_direct = 0, flops_plan = 0;
  std::vector<std::vector<double>> constant;

  int find(int a);  // with path compression
  int rep(int a) const {
    while (parent[a] != a) a = parent[a];
    return a;
  }
};

// Builds the e-graph of a problem and extracts its plan (throws
// std::invalid_argument for bad input, std::domain_error when unsupported).
void egraph_build(const TensorProblem& prob, int64_t node_limit, int objective, EGraphHost* g);

// Device evaluation of an extracted plan (egraph_exec.hip).  The steps are
// grouped by dependency level (a step's level is one more than its
// children's); each level is one launch over a device table of its steps, and
// the sum over the terms one more.  The tables depend on the batch size and
// are rebuilt when it changes.
constexpr int kEgraphMaxInputs = 64;
struct EGraphExec {
  int64_t batch = -1;
  void* steps = nullptr;               // step records, sorted by level
  void* roots = nullptr;               // root records
  void* blk_step = nullptr;            // per level: the step of each workgroup
  std::vector<int> level_begin;        // first step of each level, then the step count
  std::vector<unsigned> level_blocks;  // workgroups of each level
  int root_g = 1;
  unsigned root_blocks = 0;
};
hipError_t egraph_launch(const EGraphHost& g, EGraphExec* x, const double* const* inputs,
                         const int64_t* batch_stride, int64_t batch, double* out, void* workspace, hipStream_t st);
void egraph_exec_free(EGraphExec* x);

}  // namespace mbc
