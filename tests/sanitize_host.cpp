// Host planner under AddressSanitizer and UndefinedBehaviorSanitizer (built
// with g++, host code only, by tests/test_sanitizers.py): index sets and plan
// tables of every operator family, block sets with their factor trees, block
// plans and multiplicity counts, the tensor e-graphs of block-level
// correlators (including displaced sources and a node limit that stops
// saturation), and the parse of linearised factor trees.  Any sanitizer report aborts with a non-zero status.
#include <cstdio>
#include <vector>

#include <stdexcept>

#include "../paper_2201_04269_amd/csrc/egraph.hpp"
#include "../paper_2201_04269_amd/csrc/factor_tree.hpp"
#include "../paper_2201_04269_amd/csrc/mbc_internal.hpp"

namespace {

mbc_block_corr_desc corr(int op, int snk, int src, int mode, std::vector<std::vector<int>> moms, std::vector<int> pts) {
  mbc_block_corr_desc d{};
  d.op = op;
  d.snk_spin = snk;
  d.src_spin = src;
  d.sign_mode = mode;
  for (size_t i = 0; i < moms.size(); ++i)
    for (int k = 0; k < 3; ++k) d.mom[i][k] = moms[i][k];
  for (size_t i = 0; i < pts.size(); ++i) d.src_pt[i] = pts[i];
  return d;
}

}  // namespace

int main() {
  using namespace mbc;
  long checks = 0;
  const int ops[][4] = {{MBC_OP_PROTON, 1, 2, MBC_SIGNS_EXACT}, {MBC_OP_NEUTRON, 3, 0, MBC_SIGNS_EXACT},
                        {MBC_OP_DI, 0, 0, MBC_SIGNS_EXACT},     {MBC_OP_DII, 0, 0, MBC_SIGNS_EXACT},
                        {MBC_OP_DII, 0, 0, MBC_SIGNS_R2},       {MBC_OP_HE3_I, 1, 1, MBC_SIGNS_EXACT}};
  for (const auto& o : ops) {
    mbc_op_desc d{o[0], o[1], o[2], o[3], 1};
    IndexSet s;
    build_index_set(&d, 1, &s);
    for (int prec : {MBC_F64, MBC_F32C}) {
      PlanHost h;
      compile_plan(s, prec, &h);
      checks += h.n_tiles;
    }
  }
  std::vector<mbc_block_corr_desc> cs = {
      corr(MBC_OP_DI, 0, 0, MBC_SIGNS_EXACT, {{1, 0, 0}, {-1, 0, 0}}, {}),
      corr(MBC_OP_DII, 0, 0, MBC_SIGNS_EXACT, {{1, 0, 0}, {-1, 0, 0}}, {0, 1}),
      corr(MBC_OP_DII, 0, 0, MBC_SIGNS_R2, {{0, 0, 0}, {0, 1, 0}}, {}),
      corr(MBC_OP_HE3_I, 1, 3, MBC_SIGNS_EXACT, {{1, 0, 0}, {0, 0, 0}, {-1, 0, 0}}, {}),
      corr(MBC_OP_PROTON, 2, 1, MBC_SIGNS_EXACT, {{1, 0, 0}}, {1})};
  for (const mbc_block_corr_desc& c : cs) {
    BlockSet bs;
    build_block_set(&c, 1, &bs);
    BlockPlanHost bp;
    compile_block_plan(bs, &bp);
    int64_t n = 0, nd = 0;
    std::vector<int64_t> hist;
    block_multiplicities(c, 5000000, &n, &nd, &hist);
    checks += bp.n_terms + nd;
    for (int obj : {MBC_EXTRACT_REUSE, MBC_EXTRACT_FLOPS})
      for (int64_t limit : {int64_t(0), int64_t(300)}) {
        TensorProblem prob;
        block_expressions(bs, 0, &prob);
        EGraphHost g;
        egraph_build(prob, limit, obj, &g);
        checks += int64_t(g.steps.size());
      }
  }
  // linearised factor trees: Fig. 4's arrays, a wide root, and rejected inputs
  {
    const int32_t f4[] = {-1, 0, 2, 1, 2, 3};
    const int32_t c4[] = {2, 1, 0, 2, 0, 0};
    const double w4[] = {5, 0, 1, 0, -1, 0};
    TreeHost t;
    build_tree_host(f4, c4, 6, w4, 3, 4, &t);
    checks += t.depth;
    std::vector<int32_t> fw(101), cw(101, 0);
    std::vector<double> ww(200, 1.0);
    fw[0] = -1;
    cw[0] = 100;
    for (int v = 1; v <= 100; ++v) fw[v] = v % 7;
    build_tree_host(fw.data(), cw.data(), 101, ww.data(), 100, 7, &t);
    checks += t.level_wide[0];
    const int32_t bad_c[] = {3, 0, 0};
    const int32_t bad_f[] = {-1, 0, 1};
    const double bw[] = {1, 0, 1, 0};
    int rejected = 0;
    try {
      build_tree_host(bad_f, bad_c, 3, bw, 2, 2, &t);
    } catch (const std::invalid_argument&) {
      ++rejected;
    }
    const int32_t neg_c[] = {1, -1};
    try {
      build_tree_host(bad_f, neg_c, 2, bw, 1, 2, &t);
    } catch (const std::invalid_argument&) {
      ++rejected;
    }
    if (rejected != 2) return 1;
  }
  std::printf("sanitized host run ok (%ld)\n", checks);
  return 0;
}
