// Internal structures shared by the host-side builder/planner and the HIP
// kernels.  Nothing here is part of the public ABI (include/mbc.h).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/mbc.h"
#include "../../include/mbc_blocks.h"

namespace mbc {

constexpr int kMaxQuarks = 6;  // per flavour

// A sorted (canonical) or written-order (raw) tuple of quark indices.
struct Key {
  uint8_t n = 0;
  uint8_t v[kMaxQuarks] = {0, 0, 0, 0, 0, 0};
};
bool operator<(const Key& a, const Key& b);
bool operator==(const Key& a, const Key& b);

struct Entry {
  Key ru, cu, rd, cd;  // sink u, source u, sink d, source d
  int64_t w_re = 0, w_im = 0;
  int32_t corr = 0;
};

struct IndexSet {
  int n_u = 0, n_d = 0, n_corr = 0;
  bool canonical = true;
  std::vector<Entry> entries;         // grouped by correlator
  std::vector<int64_t> corr_begin;    // [n_corr + 1]
  std::vector<int64_t> w_den;         // [n_corr]
};

void build_index_set(const mbc_op_desc* ops, int n_corr, IndexSet* out);

// ---------------------------------------------------------------------------
// Operator algebra used by the block-level expansion (index_set.cpp).
struct Gauss {  // Gaussian integer
  int64_t re = 0, im = 0;
};
enum : uint8_t { kFlavU = 0, kFlavD = 1 };
// One baryon of a written product: family (MBC_FAMILY_P: q1 = u, q2 = d;
// MBC_FAMILY_N: q1 = d, q2 = u), projector (0, +1, -1) of its Gamma, open spin.
struct BaryonSlot {
  int family = 0, proj = 0, spin = 0;
};
// The sink operator as sum coef * prod_i B_i: coef is the written relative
// sign (+1 under MBC_SIGNS_R2) times (C gamma5)_{alpha beta} of the first two
// baryons; the third baryon (3He) carries the open index j.
struct SinkProduct {
  Gauss coef;
  int nb = 0;
  BaryonSlot b[3];
};
std::vector<SinkProduct> sink_products(int op, int spin, int sign_mode, int* den);
// The written products of eq. "ops" before the spin sums: relative sign (+1
// under MBC_SIGNS_R2) and baryons (family, projector) in written order; the
// spins are left open (X^T (C gamma5) Y [Z^j]).  A single baryon is one
// product of one baryon.  *den: the s^2 denominator.
struct WrittenProduct {
  int sign = 1, nb = 0;
  BaryonSlot b[3];
};
std::vector<WrittenProduct> written_baryon_products(int op, int sign_mode, int* den);
// A source operator term: coefficient (not conjugated) and n antiquark
// fields (flavour, index, source point).  Baryon slot i of the written
// source sits at source point pts[i] (pts == nullptr: all at point 0).
// canonical: the sorted keys u..u d..d, each flavour ordered by (point,
// index), flavour-separation and sorting signs in the coefficient;
// otherwise the written terms in written field order.
struct FieldTerm {
  Gauss coef;
  int n = 0;
  uint8_t flav[12];
  uint8_t idx[12];
  uint8_t pt[12];
};
std::vector<FieldTerm> source_terms(int op, int spin, int sign_mode, bool canonical, const int32_t* pts);
// Entries (re, im) of C gamma5 (proj 0) or C gamma5 P+- (proj +-1), row-major 4x4.
void gamma_cg5(int proj, int64_t re[16], int64_t im[16]);

// ---------------------------------------------------------------------------
// Block-level correlators (block_set.cpp): types and merged product terms.
// A block type: family, projector, sink momentum and the source points of
// its antiquarks (A, Y, C) in block order.
struct BlockType {
  int family = 0, proj = 0;
  int mom[3] = {0, 0, 0};
  int src[3] = {0, 0, 0};
};
struct BlockSet {
  int n_corr = 0, n_slots = 0, n_points = 1;
  std::vector<BlockType> types;
  std::vector<int32_t> factor;         // [n_terms][n_slots], -1 in unused slots
  std::vector<int32_t> corr;           // [n_terms]
  std::vector<int64_t> num_re, num_im; // [n_terms]
  std::vector<int64_t> den;            // [n_corr]
  std::vector<int64_t> corr_begin;     // [n_corr + 1]
  // Linearised factor tree of each correlator (Sec. 4), vertices in
  // depth-first order: the block factor of each vertex (-1 for the root) and
  // its number of children; the leaves are the correlator's terms, in order.
  std::vector<int32_t> tree_factor, tree_children;
  std::vector<int64_t> tree_vertex;    // [n_corr + 1] first vertex of each tree
  std::vector<mbc_block_corr_desc> descs;  // the correlators the set was built from
};
void build_block_set(const mbc_block_corr_desc* corrs, int n_corr, BlockSet* out);
// The block-level correlator `corr` of a set as tensor expressions over its
// block types and the constants eps, C gamma5 (P+-) and e_j (egraph.hpp).
struct TensorProblem;
void block_expressions(const BlockSet& s, int corr, TensorProblem* out);
// Sec. 3 multiplicity count of one correlator (see mbc_block_multiplicities);
// hist[m] for every multiplicity m up to the largest.  Returns false, with
// only *n_terms set, when the expansion has more than max_terms terms.
bool block_multiplicities(const mbc_block_corr_desc& c, int64_t max_terms, int64_t* n_terms,
                          int64_t* n_distinct, std::vector<int64_t>* hist);

// ---------------------------------------------------------------------------
// Plan layout (all int32 unless noted), mirrored to the device.
//
// Correlator record (kCorrInts ints):
//   [0] n_src        source keys (c_u, c_d) of the correlator
//   [1] src_off      offset into src_cu / src_cd
//   [2] n_snk        sink keys
//   [3] tile_begin   first tile of the correlator; [4] tile_end
//   [5] entry_begin  first index-set entry of the correlator
//   [6] btile_begin [7] btile_end   tiles of the backward tiling
//   [8 + 2*(6*f + k-1)]     ncol[f][k]   columns (k-subsets) at level k, flavour f
//   [8 + 2*(6*f + k-1) + 1] tab_off[f][k] offset of the level's column table
//   [40 + 6*f + k-1]  offset in btab of the level-k "j-lists": 13 relative
//                     pointers then entries C | sub << 12 | pos << 24, the
//                     columns C of level k that contain column j at position
//                     pos, with sub = index of C \ {j} (level k-1; for k = 2
//                     the remaining column number); for k = 1: C | col << 12
//   [52 + 6*f + k-1]  offset in btab of the level-k "superset lists" (parents
//                     of level k+1): ncol[f][k] + 1 relative pointers, then
//                     entries C | j << 12 | pos << 16 for every column C of
//                     level k+1 that is C' + {j}, j at position pos of C
//   [64] csr_u_off [65] csr_d_off  offsets in btab of: ncol_top + 1 relative
//                     pointers, then the source keys s with that top column
//   [66] w_base       plan-ordered W offset of the correlator's first entry
//   [67 + 6*f + k-1]  offset in btab of the "up" table of level k (k < n_f):
//                     per column C', 12 uint16 (packed two per int32): the
//                     index of C' + {j} in level k+1 | (position of j) << 12,
//                     0xffff if C' + {j} is not a needed column
//                     (12 uint16 per column C'), followed by the ncol[f][k]
//                     column numbers ordered by their count of such
//                     supersets, most first
//   [80 + f]          longest source-key list of a top column of flavour f
//   [82 + 6*f + k-1]  longest j-list of level k
//   [32] snk_vec_off  offset of the correlator's sink keys (plan order) in
//                     the sink factor wu; the source factor wv is indexed by
//                     src_off + s like src_cu / src_cd
//   [33] ftile_begin [34] ftile_end   tiles of the factored dS tiling
// Column table of level k >= 2: ncol*k uint16 entries (sub << 4) | col, the k
//   terms of the expansion along the first row; col = C_j, sub = index of
//   C \ C_j in level k-1 (for k = 2: the remaining column number itself).
//   Level 1: ncol entries, the column numbers.
// Tile record (kTileInts ints):
//   [0] corr [1] B (sink keys) [2] w_off (complex units into the plan-ordered W)
//   [3] op_begin [4] n_ops [5] meta_off [6] row_lds (complex units of row slots)
//   [7] n_phases [8 .. 8+kMaxPhases] phase boundaries (op indices, relative)
//   [16] snk_begin (index of the tile's first sink key in plan order)
//   [17] virt_begin [18] n_virt  (backward tiles) level-1 parent records
//   [19] extra_off   (backward tiles) offset in b_extra of: n_runs, n_dgroups,
//        rsum_off, then runs (u_slot, b_begin, b_end), d-groups (d_slot, b
//        mask), the children lists of the ops (each child row as its slot << 4
//        | its first row r0), and at rsum_off the S-bar row
//        lists: 25 relative pointers over the 24 (flavour, S row) pairs, then
//        the records (rows and level-1 parents) whose adjoint lands in that row
//   [15] extra_len   (backward tiles) ints of that extra block
//   [14] n_virt_u    (backward tiles) level-1 records of flavour u (listed first)
//   [20 + 2*(7f + k)], [21 + 2*(7f + k)]: first op (relative) and number of
//   ops of flavour f at level k; ops are ordered by (level, flavour).
// Row op (kOpInts ints): flav, level, r0, in, out, tab_off, ncol, item_begin
//   in: the S row r1 for level 2, the parent row's slot for level >= 3.
//   out: slot (complex offset inside the row area).
// Backward row op: flav, level, r0, in, out, child_begin, n_children, virtual
//   (virtual = a level-1 parent standing for S row r0: out = 12 * its index
//   in the tile's level-1 adjoint rows).
// Meta per sink key of a tile (kMetaInts ints): u_slot, d_slot, run_end, snk
//   (factored dS tiling: run_end | 2 if no earlier key of the tile has the
//   key's d-tuple)
// Four tilings of the sink keys per plan: the forward's (tiles/ops/meta),
// the dS kernel's (b_*: backward records, every row slot followed by one
// zero element that padded table entries point at), the dW kernel's
// (w_*: forward-style records, at most dw_keys_per_tile keys per tile), and,
// when every correlator's exact weights are a product W[b, s] = wu[b] wv[s]
// (a sink vector times a source vector, as a single operator's
// sigma s^2 w_r conj(w_c) is), the factored dS tiling (f_*: backward
// records whose tiles stage the n_src + B factors instead of the B x n_src
// weights, so that more sink keys share a tile's rows).
// ---------------------------------------------------------------------------
constexpr int kCorrInts = 96;
constexpr int kTileInts = 48;
constexpr int kOpInts = 8;
constexpr int kMetaInts = 4;
constexpr int kMaxPhases = 7;

// Threads per workgroup of the kernels of an operator family: the (5,4)
// family's columns (up to 489 per level) and source keys (up to 1308) fit
// one slot per thread at 512, halving the per-thread register tables.
constexpr int family_threads(int n_u, int n_d) { return n_u + n_d >= 8 ? 512 : 256; }
// The dS kernel of the (5,4) family in FP64 keeps 256 (at 512 its registers
// spill to scratch memory).
constexpr int ds_threads(int n_u, int n_d, int precision) {
  return (n_u + n_d >= 8 && precision == MBC_F64) ? 256 : family_threads(n_u, n_d);
}

// Whether the dS kernel of a family and precision takes the factored
// schedule for the exact weights (when they factor): measured faster for the
// 3He batch (FP32-comp 4.92 -> 4.24 s per 32^3 timeslice) and the FP64
// dinucleon (594 -> 524 ms on 16^3 x 32), slower for the FP32-comp dinucleon
// (312 -> 331 ms), whose factored leaf sums read the factors once per key
// and source slot instead of one weight.
constexpr bool ds_factored(int n_u, int n_d, int precision) {
  return !(n_u + n_d == 6 && precision == MBC_F32C);
}

// Sink keys per tile of the dW schedule, and source keys per thread the dW
// kernel is built for, per operator family (n_u, n_d) and precision (the
// kernel keeps keys x source slots compensated accumulators in registers;
// on the D_I bench workload 2 keys (FP32) and 1 (FP64) measured fastest; on
// the 3He batch 4 keys in FP32 (1.20 s per 32^3 timeslice, against 1.75 s
// with 2 and 1.47 s with 8), 2 in FP64, where 4 spills registers).
constexpr int dw_keys_per_tile(int n_u, int n_d, int precision) {
  return n_u + n_d >= 8 ? (precision == MBC_F64 ? 2 : 4) : (n_u + n_d >= 6 ? (precision == MBC_F64 ? 1 : 2) : 4);
}
constexpr int dw_src_per_thread(int n_u, int n_d) { return n_u + n_d >= 8 ? 3 : (n_u + n_d >= 6 ? 3 : 1); }

// Longest source-key list of a top column (source keys sharing their u or d
// tuple) the factored forward and the dS kernels are built for, per family.
constexpr int top_list_max(int n_u, int n_d) { return n_u + n_d >= 8 ? 10 : (n_u + n_d >= 6 ? 6 : 2); }

struct PlanHost {
  int n_u = 0, n_d = 0, n_corr = 0, precision = MBC_F64;
  int64_t nnz = 0;
  int threads = 256;
  int max_src = 0;       // max source keys of a correlator
  int max_ncol = 0;      // max columns of a level (the kernels' per-thread slots follow)
  int max_b = 0;         // max sink keys per tile
  int max_ops = 0;       // max row ops per tile
  int64_t lds_bytes = 0; // dynamic LDS of the forward kernel
  int n_tiles = 0;
  std::vector<int32_t> corr, tiles, ops, meta, src_cu, src_cd;
  // backward tiling (smaller tiles: adjoint rows need their own slots)
  int b_n_tiles = 0, b_max_ops = 0, b_max_b = 0;
  int64_t b_lds_ds = 0, b_lds_dw = 0;  // dS kernel, dW kernel
  std::vector<int32_t> b_tiles, b_ops, b_meta, b_extra, btab;
  // dW tiling (at most dw_keys_per_tile sink keys: the kernel keeps every
  // (key, source key) accumulator of a tile in registers)
  int w_n_tiles = 0, w_max_ops = 0, w_max_b = 0;
  std::vector<int32_t> w_tiles, w_ops, w_meta;
  int max_csr = 0;       // longest source-key list of a top column
  int max_bin[7] = {0, 0, 0, 0, 0, 0, 0};  // longest j-list per level
  // factored tiling (the exact weights when rank1): dS of the families
  // ds_factored admits, and the factored forward (fwd_fact)
  bool rank1 = false;
  int f_n_tiles = 0, f_max_ops = 0, f_max_b = 0;
  int64_t f_lds_ds = 0;
  bool fwd_fact = false;     // the forward of the exact weights runs factored on the f_* tiles
  int64_t f_lds_fwd = 0;     // its dynamic LDS
  double fact_alg_flops_per_site = 0, fact_ds_alg_flops_per_site = 0;
  std::vector<int32_t> f_tiles, f_ops, f_meta, f_extra;
  std::vector<double> wu, wv;     // (re, im): sink factor [sum n_snk], source factor [sum n_src]
  std::vector<uint16_t> tabs;
  std::vector<int64_t> perm;      // plan-ordered W slot -> index-set entry
  std::vector<double> w_exact;    // plan-ordered exact W (re, im)
  double alg_flops_per_site = 0, exec_flops_per_site = 0;
  double ds_alg_flops_per_site = 0, dw_alg_flops_per_site = 0;
};

// Compiles a plan; throws std::invalid_argument / std::runtime_error.
void compile_plan(const IndexSet& s, int precision, PlanHost* out);

struct PlanDevice {
  int32_t* corr = nullptr;
  int32_t* tiles = nullptr;
  int32_t* ops = nullptr;
  int32_t* meta = nullptr;
  int32_t* src_cu = nullptr;
  int32_t* src_cd = nullptr;
  uint16_t* tabs = nullptr;
  int64_t* perm = nullptr;
  void* w_exact = nullptr;  // plan precision complex
  int32_t* b_tiles = nullptr;
  int32_t* b_ops = nullptr;
  int32_t* b_meta = nullptr;
  int32_t* b_extra = nullptr;
  int32_t* btab = nullptr;
  int32_t* w_tiles = nullptr;
  int32_t* w_ops = nullptr;
  int32_t* w_meta = nullptr;
  int32_t* f_tiles = nullptr;
  int32_t* f_ops = nullptr;
  int32_t* f_meta = nullptr;
  int32_t* f_extra = nullptr;
  void* wu = nullptr;  // plan precision complex
  void* wv = nullptr;
};

// Block plan: per block type the non-zero entries of its Gamma and its
// momentum (read by every workgroup of the block kernel), the terms as
// factor indices and FP64 weights, and term chunks of one correlator each.
// One G matrix of the block kernel (a "G type"): family, Gamma, momentum and
// the source points of its three propagator factors: pt[0] for the S1 rows,
// pt[1] and pt[2] for the S1 and S2 of B.  C gamma5 and C gamma5 P+- have at
// most one non-zero entry per row, a real +-1 in the Dirac basis: row beta
// is (gcol[beta], gsign[beta]), gcol = -1 for a zero row.
struct BlockTypeDev {
  int32_t family = 0, n_gamma = 0;
  int32_t mom[3] = {0, 0, 0};
  int32_t pt[3] = {0, 0, 0};
  int32_t gcol[4] = {-1, -1, -1, -1};
  double gsign[4] = {0, 0, 0, 0};
};
constexpr int kBlockTermChunk = 4096;  // terms per workgroup of the contraction
constexpr int kTreeLeafRun = 16;       // leaves per thread of the factor-tree contraction
constexpr int kTreeMaxDepth = 3;       // levels below a correlator's root the GPU evaluates
constexpr int kTreeItemInts = 6;
constexpr int kTreeMaxItemsPerThread = 8;
constexpr int kBlockMaxChunk = 1024;   // sites per workgroup of the block kernel (LDS phase table)
struct BlockPlanHost {
  int n_types = 0, n_slots = 0, n_corr = 0, n_points = 1;
  int64_t n_terms = 0;
  // G types, and for each block type the two G types whose difference it is:
  // f(A, Y, C) = G_g1[(alpha, A)][(C, Y)] - G_g2[(alpha, C)][(A, Y)]
  std::vector<BlockTypeDev> types;  // the first n_single use one source point
  int n_single = 0;
  std::vector<int32_t> block_g;  // [n_types][2]
  std::vector<int32_t> factor;   // [n_terms][n_slots]
  std::vector<double> coef;      // [n_terms][2]
  std::vector<int32_t> chunks;   // [n_chunks][3]: correlator, first term, end term
  std::vector<int32_t> corr_chunk;  // [n_corr + 1]: first chunk of each correlator
  // factor-tree contraction: the trees' vertex factors, leaf weights in term order, and work
  // items [n_items][kTreeItemInts] = (grandparent vertex or -1, parent vertex
  // or -1, first leaf vertex, leaf count, first leaf weight, 0): a run of at
  // most kTreeLeafRun sibling leaves and the vertices above them; each
  // correlator's items padded to whole workgroups of tree_ipt x 256 items
  // (corr_wg: first workgroup of each correlator)
  std::vector<int32_t> tree_factor, items, corr_wg;
  int64_t tree_vertices = 0;
  int tree_ipt = 1;  // items per thread: enough workgroups for small sets, fewer reductions for large
  double block_flops_per_site = 0, contract_flops_per_t = 0, tree_flops_per_t = 0;
};
void compile_block_plan(const BlockSet& s, BlockPlanHost* out);

void set_error(const std::string& msg);

}  // namespace mbc

struct mbc_index_set {
  mbc::IndexSet s;
};

struct mbc_plan {
  mbc::PlanHost h;
  mbc::PlanDevice d;
  int device = 0;
};

struct mbc_block_set {
  mbc::BlockSet s;
};

struct mbc_block_plan {
  mbc::BlockPlanHost h;
  mbc::BlockTypeDev* types = nullptr;
  int32_t* factor = nullptr;
  double* coef = nullptr;
  int32_t* chunks = nullptr;
  int32_t* corr_chunk = nullptr;
  int32_t* block_g = nullptr;
  int32_t* tree_factor = nullptr;
  int32_t* items = nullptr;
  int32_t* corr_wg = nullptr;
  int device = 0;
};
