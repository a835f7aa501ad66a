// Block-level correlators (host, exact integer arithmetic).
//
// Expands a multi-baryon correlator whose baryons sit at separate,
// separately momentum-projected sink points into products of baryon blocks
// (Sec. 2 blocks, Sec. 3 expanded form).  Wick's theorem splits every
// contraction < h_1 .. h_A qbar_1 .. qbar_n > by the set partition of the
// source antiquarks among the baryons:
//
//   sum_P sign(P) (-1)^{A(A-1)/2} prod_i < h_i Qbar_i >,
//
// Qbar_i the three antiquarks of baryon i in block order (q1, q2, q1),
// sign(P) the parity of bringing the source's antiquarks to Qbar_1 .. Qbar_A,
// and (-1)^{A(A-1)/2} the sign of moving each three-field group next to its
// baryon.  The source runs over the canonical keys of eq. 1's index set
// (antiquarks u..u d..d, each flavour sorted), so the two like antiquarks of
// a block always arrive in increasing order and no block factor has a
// repeated like index.  The factors of a product are sorted and equal
// products merged exactly (the canonical ordering with multiplicities of
// Sec. 3).
#include <algorithm>
#include <climits>
#include <functional>
#include <array>
#include <stdexcept>
#include <unordered_map>

#include "egraph.hpp"
#include "mbc_internal.hpp"

namespace mbc {

namespace {

inline Gauss gmul(Gauss a, Gauss b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
inline Gauss gconj(Gauss a) { return {a.re, -a.im}; }

int parity(const int* v, int n) {
  int inv = 0;
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) inv += v[i] > v[j];
  return (inv & 1) ? -1 : 1;
}

// One set partition of the source antiquarks: grp[i] = positions (first q1,
// q2, second q1) of baryon i's antiquarks; sign includes (-1)^{A(A-1)/2}.
struct Partition {
  int grp[3][3];
  int sign;
};

void enumerate(const int* family, int A, const uint8_t* flav, int n, int i, bool* used, int (*grp)[3],
               std::vector<Partition>* out) {
  if (i == A) {
    int seq[9];
    for (int k = 0; k < A; ++k)
      for (int m = 0; m < 3; ++m) seq[3 * k + m] = grp[k][m];
    Partition p;
    for (int k = 0; k < 3; ++k)
      for (int m = 0; m < 3; ++m) p.grp[k][m] = k < A ? grp[k][m] : -1;
    p.sign = parity(seq, 3 * A) * (((A * (A - 1) / 2) & 1) ? -1 : 1);
    out->push_back(p);
    return;
  }
  const uint8_t q1 = family[i] == MBC_FAMILY_P ? kFlavU : kFlavD;
  const uint8_t q2 = family[i] == MBC_FAMILY_P ? kFlavD : kFlavU;
  for (int a = 0; a < n; ++a) {
    if (used[a] || flav[a] != q1) continue;
    for (int c = a + 1; c < n; ++c) {
      if (used[c] || flav[c] != q1) continue;
      for (int y = 0; y < n; ++y) {
        if (used[y] || flav[y] != q2) continue;
        used[a] = used[c] = used[y] = true;
        grp[i][0] = a;
        grp[i][1] = y;
        grp[i][2] = c;
        enumerate(family, A, flav, n, i + 1, used, grp, out);
        used[a] = used[c] = used[y] = false;
      }
    }
  }
}

std::vector<Partition> partitions(const int* family, int A, const uint8_t* flav, int n) {
  std::vector<Partition> out;
  if (3 * A != n) return out;
  bool used[12] = {};
  int grp[3][3];
  enumerate(family, A, flav, n, 0, used, grp, &out);
  return out;
}

int baryons_of(int op) { return op <= MBC_OP_NEUTRON ? 1 : (op <= MBC_OP_DII ? 2 : 3); }

void check_desc(const mbc_block_corr_desc& d) {
  if (d.op < MBC_OP_PROTON || d.op > MBC_OP_HE3_II) throw std::invalid_argument("unknown operator");
  if (d.sign_mode != MBC_SIGNS_EXACT && d.sign_mode != MBC_SIGNS_R2) throw std::invalid_argument("sign_mode");
  if (d.snk_spin < 0 || d.snk_spin > 3 || d.src_spin < 0 || d.src_spin > 3)
    throw std::invalid_argument("spin index out of range");
  for (int i = 0; i < baryons_of(d.op); ++i)
    if (d.src_pt[i] < 0 || d.src_pt[i] > 2) throw std::invalid_argument("source point out of range (0..2)");
}

int type_index(std::vector<BlockType>* types, int family, int proj, const int32_t* mom, const int* src) {
  for (size_t k = 0; k < types->size(); ++k) {
    const BlockType& t = (*types)[k];
    if (t.family == family && t.proj == proj && t.mom[0] == mom[0] && t.mom[1] == mom[1] && t.mom[2] == mom[2] &&
        t.src[0] == src[0] && t.src[1] == src[1] && t.src[2] == src[2])
      return int(k);
  }
  BlockType t;
  t.family = family;
  t.proj = proj;
  for (int d = 0; d < 3; ++d) {
    t.mom[d] = mom[d];
    t.src[d] = src[d];
  }
  types->push_back(t);
  return int(types->size()) - 1;
}

using Factors = std::array<int32_t, 3>;

struct Pending {
  Factors f;
  Gauss w;
};

}  // namespace

void build_block_set(const mbc_block_corr_desc* corrs, int n_corr, BlockSet* out) {
  *out = BlockSet();
  out->n_corr = n_corr;
  out->descs.assign(corrs, corrs + n_corr);
  out->den.assign(n_corr, 1);
  out->corr_begin.assign(n_corr + 1, 0);
  std::vector<std::vector<Pending>> per_corr(n_corr);
  for (int c = 0; c < n_corr; ++c) {
    const mbc_block_corr_desc& d = corrs[c];
    check_desc(d);
    int den = 1;
    const std::vector<SinkProduct> prods = sink_products(d.op, d.snk_spin, d.sign_mode, &den);
    const std::vector<FieldTerm> src = source_terms(d.op, d.src_spin, d.sign_mode, true, d.src_pt);
    out->den[c] = den;
    for (int i = 0; i < baryons_of(d.op); ++i) out->n_points = std::max(out->n_points, d.src_pt[i] + 1);
    const int A = prods.empty() ? 0 : prods[0].nb;
    out->n_slots = std::max(out->n_slots, A);
    std::vector<Pending> terms;
    for (const SinkProduct& sp : prods) {
      int family[3];
      for (int i = 0; i < sp.nb; ++i) family[i] = sp.b[i].family;
      if (src.empty()) continue;
      // every canonical key has the same flavour sequence u..u d..d
      const std::vector<Partition> parts = partitions(family, sp.nb, src[0].flav, src[0].n);
      for (const Partition& P : parts) {
        for (const FieldTerm& key : src) {
          Pending t;
          t.w = gmul(sp.coef, gconj(key.coef));
          if (P.sign < 0) t.w = {-t.w.re, -t.w.im};
          t.f = {-1, -1, -1};
          for (int i = 0; i < sp.nb; ++i) {
            const int ga = P.grp[i][0], gy = P.grp[i][1], gc = P.grp[i][2];
            const int a = key.idx[ga], y = key.idx[gy], cc = key.idx[gc];
            if (12 * key.pt[ga] + a >= 12 * key.pt[gc] + cc)
              throw std::logic_error("like antiquarks of a canonical key out of order");
            const int srcs[3] = {key.pt[ga], key.pt[gy], key.pt[gc]};
            const int type = type_index(&out->types, sp.b[i].family, sp.b[i].proj, d.mom[i], srcs);
            t.f[i] = ((type * 4 + sp.b[i].spin) * 12 + a) * 144 + y * 12 + cc;
          }
          std::sort(t.f.begin(), t.f.begin() + sp.nb);
          terms.push_back(t);
        }
      }
    }
    std::sort(terms.begin(), terms.end(), [](const Pending& x, const Pending& y) { return x.f < y.f; });
    std::vector<Pending> merged;
    for (size_t k = 0; k < terms.size();) {
      Pending m = terms[k];
      size_t e = k + 1;
      for (; e < terms.size() && terms[e].f == m.f; ++e) {
        m.w.re += terms[e].w.re;
        m.w.im += terms[e].w.im;
      }
      if (m.w.re != 0 || m.w.im != 0) merged.push_back(m);
      k = e;
    }
    per_corr[c].swap(merged);
  }
  for (int c = 0; c < n_corr; ++c) {
    for (const Pending& t : per_corr[c]) {
      for (int i = 0; i < out->n_slots; ++i) out->factor.push_back(t.f[i]);
      out->corr.push_back(c);
      out->num_re.push_back(t.w.re);
      out->num_im.push_back(t.w.im);
    }
    out->corr_begin[c + 1] = int64_t(out->corr.size());
  }
  // Factor trees: the prefix tree of each correlator's sorted factor strings.
  // A term shares its first p factors with the previous term and opens new
  // vertices for the rest, so creation order is depth-first order and the
  // leaves come in term order.
  for (int c = 0; c < n_corr; ++c) {
    out->tree_vertex.push_back(int64_t(out->tree_factor.size()));
    const int32_t root = int32_t(out->tree_factor.size());
    out->tree_factor.push_back(-1);
    out->tree_children.push_back(0);
    int32_t path[3] = {-1, -1, -1};
    for (int64_t k = out->corr_begin[c]; k < out->corr_begin[c + 1]; ++k) {
      const int32_t* f = &out->factor[size_t(k) * out->n_slots];
      int A = 0;
      while (A < out->n_slots && f[A] >= 0) ++A;
      int p = 0;
      if (k > out->corr_begin[c]) {
        const int32_t* g = &out->factor[size_t(k - 1) * out->n_slots];
        while (p < A && f[p] == g[p]) ++p;
        if (p == A) throw std::logic_error("repeated factor string after merging");
      }
      for (int l = p; l < A; ++l) {
        ++out->tree_children[l == 0 ? root : path[l - 1]];
        path[l] = int32_t(out->tree_factor.size());
        out->tree_factor.push_back(f[l]);
        out->tree_children.push_back(0);
      }
    }
  }
  out->tree_vertex.push_back(int64_t(out->tree_factor.size()));
}

void compile_block_plan(const BlockSet& s, BlockPlanHost* out) {
  *out = BlockPlanHost();
  out->n_types = int(s.types.size());
  out->n_slots = s.n_slots;
  out->n_corr = s.n_corr;
  out->n_points = s.n_points;
  out->n_terms = int64_t(s.corr.size());
  // G types: a block type with source points (zA, zY, zC) is
  // G(zA; zC, zY)[(alpha, A)][(C, Y)] - G(zC; zA, zY)[(alpha, C)][(A, Y)]
  // (rows from S1 at the first point, B from S1 and S2 at the other two);
  // one G when zA == zC
  std::vector<BlockType> gt;  // src = (row point, B's S1 point, B's S2 point)
  for (const BlockType& t : s.types) {
    for (int w = 0; w < 2; ++w) {
      BlockType g = t;
      g.src[0] = w == 0 ? t.src[0] : t.src[2];
      g.src[1] = w == 0 ? t.src[2] : t.src[0];
      g.src[2] = t.src[1];
      out->block_g.push_back(type_index(&gt, g.family, g.proj, g.mom, g.src));
    }
  }
  // G types whose two S1 factors share a source point first (the kernel's
  // common case), then the mixed ones
  std::vector<int32_t> order, where(gt.size());
  for (int mixed = 0; mixed < 2; ++mixed)
    for (size_t k = 0; k < gt.size(); ++k)
      if ((gt[k].src[0] != gt[k].src[1]) == bool(mixed)) {
        where[k] = int32_t(order.size());
        order.push_back(int32_t(k));
      }
  out->n_single = 0;
  for (const BlockType& g : gt) out->n_single += g.src[0] == g.src[1];
  for (int32_t& g : out->block_g) g = where[g];
  std::vector<BlockType> sorted;
  for (int32_t k : order) sorted.push_back(gt[k]);
  gt.swap(sorted);
  for (const BlockType& t : gt) {
    BlockTypeDev d;
    d.family = t.family;
    for (int k = 0; k < 3; ++k) {
      d.mom[k] = t.mom[k];
      d.pt[k] = t.src[k];
    }
    int64_t re[16], im[16];
    gamma_cg5(t.proj, re, im);
    for (int be = 0; be < 4; ++be)
      for (int ga = 0; ga < 4; ++ga) {
        const int e = 4 * be + ga;
        if (re[e] == 0 && im[e] == 0) continue;
        if (im[e] != 0 || (re[e] != 1 && re[e] != -1) || d.gcol[be] >= 0)
          throw std::logic_error("Gamma row with more than one entry or an entry other than +-1");
        d.gcol[be] = ga;
        d.gsign[be] = double(re[e]);
        ++d.n_gamma;
      }
    out->types.push_back(d);
    // B: 432 entries x (2 colour pairs x n_gamma products + one phase
    // multiply); G: 48 x 144 entries x 3 colours, 8 flops per multiply-add
    out->block_flops_per_site += 432.0 * (2.0 * d.n_gamma * 8.0 + 6.0) + 6912.0 * 3.0 * 8.0;
  }
  out->factor = s.factor;
  out->coef.resize(size_t(out->n_terms) * 2);
  for (int64_t k = 0; k < out->n_terms; ++k) {
    const double den = double(s.den[s.corr[k]]);
    out->coef[2 * k] = double(s.num_re[k]) / den;
    out->coef[2 * k + 1] = double(s.num_im[k]) / den;
    int used = 0;
    for (int i = 0; i < s.n_slots; ++i) used += s.factor[k * s.n_slots + i] >= 0;
    out->contract_flops_per_t += 6.0 * used + 2.0;
  }
  out->tree_flops_per_t = 8.0 * double(int64_t(s.tree_factor.size()) - s.n_corr);
  if (out->n_terms > INT32_MAX - kBlockTermChunk) throw std::domain_error("more than 2^31 block terms");
  for (int c = 0; c < s.n_corr; ++c) {
    out->corr_chunk.push_back(int32_t(out->chunks.size() / 3));
    for (int64_t b = s.corr_begin[c]; b < s.corr_begin[c + 1]; b += kBlockTermChunk) {
      out->chunks.push_back(c);
      out->chunks.push_back(int32_t(b));
      out->chunks.push_back(int32_t(std::min<int64_t>(b + kBlockTermChunk, s.corr_begin[c + 1])));
    }
  }
  out->corr_chunk.push_back(int32_t(out->chunks.size() / 3));

  // Factor-tree work items: the tree cut above its leaves.  Every vertex whose
  // children are leaves (a leaf parent) gives runs of at most kTreeLeafRun of
  // its leaves; an item also names the parent and grandparent (the factors
  // its run shares).  Trees are at most kTreeMaxDepth levels deep, so these
  // are all the factors of a path.
  if (int64_t(s.tree_factor.size()) > INT32_MAX) throw std::domain_error("factor tree too large");
  out->tree_factor = s.tree_factor;
  out->tree_vertices = int64_t(s.tree_factor.size());
  const std::vector<int32_t>& nch = s.tree_children;
  std::vector<size_t> corr_items(s.n_corr + 1, 0);
  for (int c = 0; c < s.n_corr; ++c) {
    corr_items[c] = out->items.size() / kTreeItemInts;
    const size_t first_item = corr_items[c];
    const int64_t root = s.tree_vertex[c], vend = s.tree_vertex[c + 1];
    int64_t leaf = s.corr_begin[c];
    // depth-first walk with the path of ancestors: path[l] = vertex at level l
    int64_t path[kTreeMaxDepth + 1] = {-1, -1, -1, -1};
    std::function<void(int64_t, int)> walk = [&](int64_t v, int level) -> void {
      if (level > kTreeMaxDepth - 1) throw std::domain_error("factor tree deeper than the GPU evaluator");
      path[level] = v;
      const int n = nch[size_t(v)];
      int64_t w = v + 1;
      if (n > 0 && nch[size_t(w)] == 0) {
        for (int k = 1; k < n; ++k)
          if (nch[size_t(w + k)] != 0) throw std::domain_error("factor tree with leaves at several depths");
        for (int k0 = 0; k0 < n; k0 += kTreeLeafRun) {
          const int cnt = std::min(kTreeLeafRun, n - k0);
          const int32_t parent = level >= 1 ? int32_t(v) : -1;
          const int32_t grand = level >= 2 ? int32_t(path[level - 1]) : -1;
          out->items.insert(out->items.end(), {grand, parent, int32_t(w + k0), cnt, int32_t(leaf), 0});
          leaf += cnt;
        }
        return;
      }
      for (int k = 0; k < n; ++k) {
        const int64_t child = w;
        walk(child, level + 1);
        // skip the child's subtree: the next sibling follows it
        int64_t open = 1;
        while (open > 0) {
          open += nch[size_t(w)] - 1;
          ++w;
        }
      }
    };
    if (nch[size_t(root)] > 0) walk(root, 0);
    // the items must hold every leaf of the tree once, in term order
    if (leaf != s.corr_begin[c + 1]) throw std::logic_error("factor-tree items miss leaves");
    int64_t expect = s.corr_begin[c];
    for (size_t it = first_item; it < out->items.size() / kTreeItemInts; ++it) {
      const int32_t* r = &out->items[kTreeItemInts * it];
      if (r[4] != expect || r[2] <= root || r[2] + r[3] > vend) throw std::logic_error("factor-tree item out of range");
      for (int k = 0; k < r[3]; ++k)
        if (nch[size_t(r[2] + k)] != 0 || out->tree_factor[size_t(r[2] + k)] < 0)
          throw std::logic_error("factor-tree item holds a non-leaf");
      for (int k = 0; k < 2; ++k)
        if (r[k] >= 0 && (r[k] <= root || r[k] >= vend)) throw std::logic_error("factor-tree item ancestor out of range");
      expect += r[3];
    }
  }
  corr_items[s.n_corr] = out->items.size() / kTreeItemInts;
  // items per thread: 1 up to 256 x 1024 items, doubling to at most
  // kTreeMaxItemsPerThread, then each correlator padded to whole workgroups
  const size_t total = corr_items[s.n_corr];
  out->tree_ipt = 1;
  while (out->tree_ipt < kTreeMaxItemsPerThread && total > size_t(256) * 1024 * size_t(out->tree_ipt))
    out->tree_ipt *= 2;
  const size_t per_wg = size_t(256) * out->tree_ipt;
  std::vector<int32_t> padded_items;
  int wg = 0;
  for (int c = 0; c < s.n_corr; ++c) {
    out->corr_wg.push_back(wg);
    const size_t n_items = corr_items[c + 1] - corr_items[c];
    padded_items.insert(padded_items.end(), out->items.begin() + corr_items[c] * kTreeItemInts,
                        out->items.begin() + corr_items[c + 1] * kTreeItemInts);
    const size_t padded = (n_items + per_wg - 1) / per_wg * per_wg;
    for (size_t k = n_items; k < padded; ++k) padded_items.insert(padded_items.end(), {-1, -1, 0, 0, 0, 0});
    wg += int(padded / per_wg);
  }
  out->items.swap(padded_items);
  out->corr_wg.push_back(wg);
}

bool block_multiplicities(const mbc_block_corr_desc& d, int64_t max_terms, int64_t* n_terms, int64_t* n_distinct,
                          std::vector<int64_t>* hist) {
  check_desc(d);
  int den = 1;
  const std::vector<SinkProduct> prods = sink_products(d.op, d.snk_spin, d.sign_mode, &den);
  const std::vector<FieldTerm> src = source_terms(d.op, d.src_spin, d.sign_mode, false, d.src_pt);
  // partitions depend on the slots' families and the source term's flavour
  // sequence only: count the expansion before forming any string
  std::unordered_map<uint64_t, std::vector<Partition>> cache;
  int64_t total = 0;
  for (size_t p = 0; p < prods.size(); ++p) {
    int family[3];
    uint64_t fkey = 0;
    for (int i = 0; i < prods[p].nb; ++i) {
      family[i] = prods[p].b[i].family;
      fkey = fkey * 2 + uint64_t(family[i]);
    }
    for (size_t s = 0; s < src.size(); ++s) {
      uint64_t key = fkey;
      for (int i = 0; i < src[s].n; ++i) key = key * 2 + src[s].flav[i];
      key = key * 16 + uint64_t(prods[p].nb);
      auto it = cache.find(key);
      if (it == cache.end()) it = cache.emplace(key, partitions(family, prods[p].nb, src[s].flav, src[s].n)).first;
      total += int64_t(it->second.size());
    }
  }
  *n_terms = total;
  if (total > max_terms) return false;
  // hadron (family, projector) and momentum of a slot -> small id
  std::vector<BlockType> ids;
  std::vector<Factors> strings;
  strings.reserve(size_t(total));
  for (const SinkProduct& sp : prods) {
    int family[3];
    uint64_t fkey = 0;
    for (int i = 0; i < sp.nb; ++i) {
      family[i] = sp.b[i].family;
      fkey = fkey * 2 + uint64_t(family[i]);
    }
    for (const FieldTerm& t : src) {
      uint64_t key = fkey;
      for (int i = 0; i < t.n; ++i) key = key * 2 + t.flav[i];
      key = key * 16 + uint64_t(sp.nb);
      for (const Partition& P : cache.at(key)) {
        Factors f = {-1, -1, -1};
        for (int i = 0; i < sp.nb; ++i) {
          const int ga = P.grp[i][0], gy = P.grp[i][1], gc = P.grp[i][2];
          const int a = t.idx[ga], y = t.idx[gy], cc = t.idx[gc];
          const int srcs[3] = {t.pt[ga], t.pt[gy], t.pt[gc]};
          const int id = type_index(&ids, sp.b[i].family, sp.b[i].proj, d.mom[i], srcs);
          f[i] = (((id * 12 + a) * 12 + y) * 12 + cc) * 4 + sp.b[i].spin;
        }
        std::sort(f.begin(), f.begin() + sp.nb);
        strings.push_back(f);
      }
    }
  }
  std::sort(strings.begin(), strings.end());
  hist->assign(1, 0);
  int64_t distinct = 0;
  for (size_t k = 0; k < strings.size();) {
    size_t e = k + 1;
    while (e < strings.size() && strings[e] == strings[k]) ++e;
    const size_t m = e - k;
    if (hist->size() <= m) hist->resize(m + 1, 0);
    ++(*hist)[m];
    ++distinct;
    k = e;
  }
  *n_distinct = distinct;
  return true;
}

}  // namespace mbc

namespace mbc {

// The block-level correlator `corr` as a sum of tensor expressions (Sec. 5
// applied to the partition sum of Sec. 3).  Tensors: the set's block types
// [sigma][c_A][s_A][c_Y][s_Y][c_C][s_C] (the A <-> C antisymmetry when the two
// like antiquarks share a source point), then eps, C gamma5, C gamma5 P+,
// C gamma5 P- and the unit vectors e_0..e_3.  Labels: sink spin of baryon i
// is i; source antiquark k (written order) has colour A + 2k, spin A + 2k + 1.
void block_expressions(const BlockSet& s, int corr, TensorProblem* out) {
  if (corr < 0 || corr >= s.n_corr) throw std::invalid_argument("correlator index out of range");
  const mbc_block_corr_desc& d = s.descs[corr];
  *out = TensorProblem();
  const int nty = int(s.types.size());
  for (const BlockType& t : s.types) {
    mbc_tensor_decl dc{};
    dc.rank = 7;
    const int ext[7] = {4, 3, 4, 3, 4, 3, 4};
    for (int k = 0; k < 7; ++k) dc.ext[k] = ext[k];
    if (t.src[0] == t.src[2]) {
      const int sw[7] = {0, 5, 6, 3, 4, 1, 2};
      dc.n_sym = 1;
      for (int k = 0; k < 7; ++k) dc.perm[0][k] = sw[k];
      dc.sign[0] = -1;
    }
    out->decls.push_back(dc);
    out->constant.emplace_back();
  }
  const int t_eps = nty, t_gam = nty + 1, t_unit = nty + 4;
  {
    mbc_tensor_decl dc{};
    dc.rank = 3;
    dc.ext[0] = dc.ext[1] = dc.ext[2] = 3;
    dc.n_sym = 2;
    const int p0[3] = {1, 0, 2}, p1[3] = {1, 2, 0};
    for (int k = 0; k < 3; ++k) {
      dc.perm[0][k] = p0[k];
      dc.perm[1][k] = p1[k];
    }
    dc.sign[0] = -1;
    dc.sign[1] = 1;
    out->decls.push_back(dc);
    std::vector<double> v(2 * 27, 0.0);
    const int e3[6][3] = {{0, 1, 2}, {1, 2, 0}, {2, 0, 1}, {1, 0, 2}, {0, 2, 1}, {2, 1, 0}};
    for (int q = 0; q < 6; ++q) v[2 * ((e3[q][0] * 3 + e3[q][1]) * 3 + e3[q][2])] = q < 3 ? 1.0 : -1.0;
    out->constant.push_back(v);
  }
  for (int proj : {0, 1, -1}) {
    int64_t re[16], im[16];
    gamma_cg5(proj, re, im);
    bool anti = true;
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) anti = anti && re[4 * i + j] == -re[4 * j + i] && im[4 * i + j] == -im[4 * j + i];
    mbc_tensor_decl dc{};
    dc.rank = 2;
    dc.ext[0] = dc.ext[1] = 4;
    if (anti) {
      dc.n_sym = 1;
      dc.perm[0][0] = 1;
      dc.perm[0][1] = 0;
      dc.sign[0] = -1;
    }
    out->decls.push_back(dc);
    std::vector<double> v(32);
    for (int k = 0; k < 16; ++k) {
      v[2 * k] = double(re[k]);
      v[2 * k + 1] = double(im[k]);
    }
    out->constant.push_back(v);
  }
  for (int j = 0; j < 4; ++j) {
    mbc_tensor_decl dc{};
    dc.rank = 1;
    dc.ext[0] = 4;
    out->decls.push_back(dc);
    std::vector<double> v(8, 0.0);
    v[2 * j] = 1.0;
    out->constant.push_back(v);
  }
  auto gam = [&](int proj) { return t_gam + (proj == 0 ? 0 : (proj > 0 ? 1 : 2)); };

  int den = 1;
  const std::vector<WrittenProduct> prods = written_baryon_products(d.op, d.sign_mode, &den);
  const int A = prods.empty() ? 0 : prods[0].nb;
  auto col = [&](int k) { return A + 2 * k; };
  auto spn = [&](int k) { return A + 2 * k + 1; };
  out->term_begin.push_back(0);
  auto push = [&](int t, std::initializer_list<int> lab) {
    mbc_tensor_factor f{};
    f.tensor = t;
    int k = 0;
    for (int x : lab) f.label[k++] = x;
    out->factors.push_back(f);
  };
  for (const WrittenProduct& snk : prods)
    for (const WrittenProduct& src : prods) {
      int family[3];
      for (int i = 0; i < A; ++i) family[i] = snk.b[i].family;
      uint8_t flav[9];
      for (int b = 0; b < A; ++b) {
        const bool p = src.b[b].family == MBC_FAMILY_P;
        flav[3 * b] = flav[3 * b + 2] = p ? kFlavU : kFlavD;
        flav[3 * b + 1] = p ? kFlavD : kFlavU;
      }
      for (const Partition& P : partitions(family, A, flav, 3 * A)) {
        double coef = double(snk.sign * src.sign * P.sign) / double(den);
        if (A == 1) {
          push(t_unit + d.snk_spin, {0});
        } else {
          push(t_gam, {0, 1});
          if (A == 3) push(t_unit + d.snk_spin, {2});
        }
        for (int i = 0; i < A; ++i) {
          int a = P.grp[i][0], y = P.grp[i][1], c = P.grp[i][2];
          int z[3] = {d.src_pt[a / 3], d.src_pt[y / 3], d.src_pt[c / 3]};
          int ty = -1;
          for (int k = 0; k < nty && ty < 0; ++k) {
            const BlockType& t = s.types[k];
            if (t.family == snk.b[i].family && t.proj == snk.b[i].proj && t.mom[0] == d.mom[i][0] &&
                t.mom[1] == d.mom[i][1] && t.mom[2] == d.mom[i][2] && t.src[0] == z[0] && t.src[1] == z[1] &&
                t.src[2] == z[2])
              ty = k;
          }
          if (ty < 0) {
            // the type with the like antiquarks' points exchanged: f(A,Y,C) = -f'(C,Y,A)
            std::swap(a, c);
            std::swap(z[0], z[2]);
            coef = -coef;
            for (int k = 0; k < nty && ty < 0; ++k) {
              const BlockType& t = s.types[k];
              if (t.family == snk.b[i].family && t.proj == snk.b[i].proj && t.mom[0] == d.mom[i][0] &&
                  t.mom[1] == d.mom[i][1] && t.mom[2] == d.mom[i][2] && t.src[0] == z[0] && t.src[1] == z[1] &&
                  t.src[2] == z[2])
                ty = k;
            }
          }
          if (ty < 0)
            throw std::invalid_argument(
                "a block type of this correlator is not in the block set (a correlator whose canonical "
                "expansion is empty adds no types: build the set together with one that uses them)");
          push(ty, {i, col(a), spn(a), col(y), spn(y), col(c), spn(c)});
        }
        for (int b = 0; b < A; ++b) {
          push(t_eps, {col(3 * b), col(3 * b + 1), col(3 * b + 2)});
          push(gam(src.b[b].proj), {spn(3 * b), spn(3 * b + 1)});
        }
        if (A == 1) {
          push(t_unit + d.src_spin, {spn(2)});
        } else {
          push(t_gam, {spn(2), spn(5)});
          if (A == 3) push(t_unit + d.src_spin, {spn(8)});
        }
        out->term_begin.push_back(int32_t(out->factors.size()));
        out->coef.push_back(coef);
        out->coef.push_back(0.0);
      }
    }
}

}  // namespace mbc
