// Tensor e-graphs (Sec. 5): canonical forms, e-graph construction and plan
// extraction on the host.
//
// Canonical form.  The factors of a product are listed by increasing tensor
// id and each may be rewritten by any element of its tensor's symmetry group;
// labels are renamed by first appearance (summed label k -> 2k, open label
// k -> 2k + 1).  The canonical code is the lexicographically smallest
// (tensor id, slot codes) sequence.  Every factor contributes a block of
// fixed length, so the smallest sequence is found position by position: all
// partial arrangements whose blocks so far are minimal are kept (two with the
// same used factors and the same renaming have the same future and are
// merged, their signs collected).  Among the complete arrangements the one
// with the smallest tuple of open labels gives the open-slot map and the
// sign; reaching it with both signs means the product vanishes identically.
//
// E-graph.  Classes are created on first sight of a canonical code (the
// hash-cons H maps codes and e-nodes to class ids) and expanded first in,
// first out: every split E = E1 E2 of the class's canonical factors (E1
// holds factor 0; splits by increasing subset mask) that passes the paper's
// two conditions (each part holds a label summed in E; one part holds a
// factor with no open label of E) becomes an e-node sign x [E1] [E2] whose children are the
// classes of the canonicalised parts.  An e-node already owned by another
// class unites the two classes (union-find U).  Expansion stops adding
// e-nodes at the node limit; a class left without an e-node is split at the
// root of a greedy pairwise contraction order of its factors.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cstring>
#include <functional>
#include <map>
#include <stdexcept>

#include "egraph.hpp"

namespace mbc {

namespace {

using i128 = __int128;
constexpr size_t kMaxStates = size_t(1) << 20;

void closure(const mbc_tensor_decl& d, TensorInfo* t) {
  t->rank = d.rank;
  for (int k = 0; k < d.rank; ++k) t->ext[k] = d.ext[k];
  SymElem id{};
  for (int k = 0; k < d.rank; ++k) id.p[k] = uint8_t(k);
  id.s = 1;
  t->group.assign(1, id);
  std::map<std::vector<uint8_t>, int> seen;
  seen[std::vector<uint8_t>(id.p, id.p + d.rank)] = 1;
  for (size_t i = 0; i < t->group.size(); ++i) {
    const SymElem p = t->group[i];
    for (int g = 0; g < d.n_sym; ++g) {
      SymElem r{};
      for (int k = 0; k < d.rank; ++k) r.p[k] = p.p[d.perm[g][k]];
      r.s = int8_t(p.s * d.sign[g]);
      const std::vector<uint8_t> key(r.p, r.p + d.rank);
      auto it = seen.find(key);
      if (it != seen.end()) {
        if (it->second != r.s) throw std::domain_error("a symmetry group contains -identity: the tensor vanishes");
        continue;
      }
      if (t->group.size() >= 40320) throw std::domain_error("symmetry group too large");
      seen[key] = r.s;
      t->group.push_back(r);
    }
  }
}

struct Canon {
  std::vector<int16_t> code;
  int sign = 0;  // 0: vanishes identically
  std::vector<uint8_t> opens;
};

void count_labels(const Expr& e, const std::vector<TensorInfo>& T, int* cnt) {
  std::memset(cnt, 0, sizeof(int) * MBC_EGRAPH_MAX_LABEL);
  for (const Fac& f : e)
    for (int k = 0; k < T[f.t].rank; ++k) ++cnt[f.lab[k]];
}

Canon canonical(const Expr& e, const std::vector<TensorInfo>& T) {
  int cnt[MBC_EGRAPH_MAX_LABEL];
  count_labels(e, T, cnt);
  const int n = int(e.size());
  std::vector<int> tids(n);
  for (int i = 0; i < n; ++i) tids[i] = e[i].t;
  std::sort(tids.begin(), tids.end());
  struct St {
    uint32_t used = 0;
    int8_t name[MBC_EGRAPH_MAX_LABEL];
    uint8_t nd = 0, no = 0, signs = 1;  // signs: bit 0 reached with +, bit 1 with -
  };
  St init;
  std::memset(init.name, -1, sizeof(init.name));
  std::vector<St> cur(1, init);
  Canon out;
  std::vector<int16_t> best, blk;
  for (int pos = 0; pos < n; ++pos) {
    const int tid = tids[pos];
    const TensorInfo& ti = T[tid];
    std::vector<St> next;
    std::unordered_map<std::string, size_t> seen;
    best.clear();
    for (const St& st : cur) {
      for (int i = 0; i < n; ++i) {
        if ((st.used >> i & 1u) || e[i].t != tid) continue;
        for (const SymElem& g : ti.group) {
          St ns = st;
          blk.clear();
          for (int k = 0; k < ti.rank; ++k) {
            const int x = e[i].lab[g.p[k]];
            if (ns.name[x] < 0) ns.name[x] = int8_t(cnt[x] == 2 ? 2 * ns.nd++ : 2 * ns.no++ + 1);
            blk.push_back(ns.name[x]);
          }
          if (!best.empty()) {
            if (blk > best) continue;
            if (blk < best) {
              next.clear();
              seen.clear();
            }
          }
          best = blk;
          ns.used |= 1u << i;
          if (g.s < 0) ns.signs = uint8_t(((ns.signs & 1u) << 1) | ((ns.signs >> 1) & 1u));
          std::string key(reinterpret_cast<const char*>(&ns.used), 4);
          key.append(reinterpret_cast<const char*>(ns.name), MBC_EGRAPH_MAX_LABEL);
          auto it = seen.find(key);
          if (it != seen.end()) {
            next[it->second].signs |= ns.signs;
          } else {
            seen.emplace(std::move(key), next.size());
            next.push_back(ns);
            if (next.size() > kMaxStates) throw std::domain_error("canonical form: too many partial arrangements");
          }
        }
      }
    }
    out.code.push_back(int16_t(tid));
    out.code.insert(out.code.end(), best.begin(), best.end());
    cur.swap(next);
  }
  // the smallest tuple of open labels among the complete arrangements
  bool have = false;
  uint8_t signs = 0;
  std::vector<uint8_t> bo, op;
  for (const St& st : cur) {
    op.assign(st.no, 0);
    for (int x = 0; x < MBC_EGRAPH_MAX_LABEL; ++x)
      if (st.name[x] >= 0 && (st.name[x] & 1)) op[st.name[x] >> 1] = uint8_t(x);
    if (!have || op < bo) {
      bo = op;
      signs = st.signs;
      have = true;
    } else if (op == bo) {
      signs |= st.signs;
    }
  }
  out.opens = bo;
  out.sign = signs == 3 ? 0 : (signs == 1 ? 1 : -1);
  return out;
}

std::string code_key(const std::vector<int16_t>& code) {
  std::string k("E");
  k.append(reinterpret_cast<const char*>(code.data()), code.size() * sizeof(int16_t));
  return k;
}

// The canonical expression: the code split into factors.
Expr relabel(const std::vector<int16_t>& code, const std::vector<TensorInfo>& T) {
  Expr e;
  for (size_t p = 0; p < code.size();) {
    Fac f;
    f.t = code[p];
    for (int k = 0; k < T[f.t].rank; ++k) f.lab[k] = uint8_t(code[p + 1 + k]);
    p += 1 + T[f.t].rank;
    e.push_back(f);
  }
  return e;
}

i128 prod_ext(const EClass& c, uint64_t mask) {
  i128 p = 1;
  for (int x = 0; x < MBC_EGRAPH_MAX_LABEL; ++x)
    if (mask >> x & 1u) p *= c.label_ext[x];
  return p;
}

// Root split (subset mask holding factor 0) of a greedy pairwise contraction
// order: repeatedly join the two operands whose join removes the most
// intermediate elements (size of the join - sizes of the two), then the one
// whose two operands carry the fewest label combinations, then the first pair.
uint32_t greedy_split(const Expr& cf, const std::vector<TensorInfo>& T) {
  const int n = int(cf.size());
  int ext[MBC_EGRAPH_MAX_LABEL] = {};
  for (const Fac& f : cf)
    for (int k = 0; k < T[f.t].rank; ++k) ext[f.lab[k]] = T[f.t].ext[k];
  auto opens = [&](uint32_t mask) {
    int c[MBC_EGRAPH_MAX_LABEL] = {};
    for (int i = 0; i < n; ++i)
      if (mask >> i & 1u)
        for (int k = 0; k < T[cf[i].t].rank; ++k) ++c[cf[i].lab[k]];
    uint64_t m = 0;
    for (int x = 0; x < MBC_EGRAPH_MAX_LABEL; ++x)
      if (c[x] == 1) m |= uint64_t(1) << x;
    return m;
  };
  auto size = [&](uint64_t m) {
    i128 p = 1;
    for (int x = 0; x < MBC_EGRAPH_MAX_LABEL; ++x)
      if (m >> x & 1u) p *= ext[x];
    return p;
  };
  std::vector<uint32_t> ops;
  for (int i = 0; i < n; ++i) ops.push_back(1u << i);
  while (ops.size() > 2) {
    int bi = -1, bj = -1;
    i128 b0 = 0, b1 = 0;
    for (int i = 0; i < int(ops.size()); ++i)
      for (int j = i + 1; j < int(ops.size()); ++j) {
        const uint64_t oi = opens(ops[i]), oj = opens(ops[j]);
        const i128 k0 = size(opens(ops[i] | ops[j])) - size(oi) - size(oj), k1 = size(oi | oj);
        if (bi < 0 || k0 < b0 || (k0 == b0 && k1 < b1)) {
          bi = i;
          bj = j;
          b0 = k0;
          b1 = k1;
        }
      }
    ops[bi] |= ops[bj];
    ops.erase(ops.begin() + bj);
  }
  return (ops[0] & 1u) ? ops[0] : ops[1];
}

struct Builder {
  EGraphHost& g;

  // (class, sign, open labels), or class -1 if the product vanishes
  int add_expr(const Expr& e, int* sign, std::vector<uint8_t>* opens) {
    Canon c = canonical(e, g.tensors);
    *sign = c.sign;
    *opens = c.opens;
    if (c.sign == 0) return -1;
    const std::string key = code_key(c.code);
    auto it = g.H.find(key);
    if (it == g.H.end()) {
      EClass k;
      k.code = c.code;
      k.factors = relabel(c.code, g.tensors);
      k.n_open = int(c.opens.size());
      for (const Fac& f : k.factors)
        for (int s = 0; s < g.tensors[f.t].rank; ++s) {
          k.label_ext[f.lab[s]] = g.tensors[f.t].ext[s];
          k.labels |= uint64_t(1) << f.lab[s];
        }
      for (int o = 0; o < k.n_open; ++o) k.open_ext.push_back(k.label_ext[2 * o + 1]);
      const int id = int(g.cls.size());
      g.cls.push_back(std::move(k));
      g.parent.push_back(id);
      g.H.emplace(key, id);
      g.work.push_back(id);
      return id;
    }
    return g.find(it->second);
  }

  void unite(int a, int b) {
    a = g.find(a);
    b = g.find(b);
    if (a == b) return;
    const int lo = std::min(a, b), hi = std::max(a, b);
    g.parent[hi] = lo;
    g.cls[lo].nodes.insert(g.cls[lo].nodes.end(), g.cls[hi].nodes.begin(), g.cls[hi].nodes.end());
  }

  void add_node(int cid, const Expr& e1, const Expr& e2) {
    int s1, s2;
    std::vector<uint8_t> o1, o2;
    const int c1 = add_expr(e1, &s1, &o1);
    const int c2 = add_expr(e2, &s2, &o2);
    if (c1 < 0 || c2 < 0) return;
    ENode nd;
    nd.c1 = c1;
    nd.c2 = c2;
    nd.sign = s1 * s2;
    nd.o1 = o1;
    nd.o2 = o2;
    std::string key("N");
    const int32_t hdr[4] = {c1, c2, nd.sign, int32_t(o1.size())};
    key.append(reinterpret_cast<const char*>(hdr), sizeof(hdr));
    key.append(reinterpret_cast<const char*>(o1.data()), o1.size());
    key.append(reinterpret_cast<const char*>(o2.data()), o2.size());
    auto it = g.H.find(key);
    if (it != g.H.end()) {
      if (g.find(it->second) != g.find(cid)) unite(it->second, cid);
      return;
    }
    g.H.emplace(std::move(key), cid);
    g.cls[cid].nodes.push_back(std::move(nd));
    ++g.n_nodes;
  }

  // the admitted splits of class cid, in increasing subset mask
  void expand(int cid, int64_t node_limit) {
    const Expr cf = g.cls[cid].factors;
    const int n = int(cf.size());
    int cnt[MBC_EGRAPH_MAX_LABEL];
    count_labels(cf, g.tensors, cnt);
    bool full = false;  // a factor with no open label of E
    for (const Fac& f : cf) {
      bool all = true;
      for (int k = 0; k < g.tensors[f.t].rank; ++k) all = all && cnt[f.lab[k]] == 2;
      full = full || all;
    }
    if (!full) return;
    const uint32_t all_mask = (1u << n) - 1;
    for (uint32_t m = 1; m < all_mask; m += 2) {
      Expr p[2];
      for (int i = 0; i < n; ++i) p[(m >> i & 1u) ? 0 : 1].push_back(cf[i]);
      // (1) each part holds a label summed in E (condition (2) holds for
      // every split once E has a factor with no open label)
      bool summed = true;
      for (int k = 0; k < 2 && summed; ++k) {
        bool any = false;
        for (const Fac& f : p[k])
          for (int q = 0; q < g.tensors[f.t].rank; ++q) any = any || cnt[f.lab[q]] == 2;
        summed = any;
      }
      if (!summed) continue;
      if (g.n_nodes >= node_limit) {
        g.saturated = false;
        return;
      }
      add_node(cid, p[0], p[1]);
    }
  }
};

}  // namespace

int EGraphHost::find(int a) {
  while (parent[a] != a) {
    parent[a] = parent[parent[a]];
    a = parent[a];
  }
  return a;
}

void egraph_build(const TensorProblem& prob, int64_t node_limit, int objective, EGraphHost* gp) {
  EGraphHost& g = *gp;
  g = EGraphHost();
  if (node_limit < 0) throw std::invalid_argument("node_limit must be >= 0");
  if (objective != MBC_EXTRACT_REUSE && objective != MBC_EXTRACT_FLOPS && objective != MBC_EXTRACT_SHARED)
    throw std::invalid_argument("objective");
  const int nt = int(prob.decls.size());
  if (nt < 1) throw std::invalid_argument("no tensors declared");
  for (const mbc_tensor_decl& d : prob.decls) {
    if (d.rank < 1 || d.rank > MBC_EGRAPH_MAX_RANK) throw std::invalid_argument("tensor rank out of range");
    for (int k = 0; k < d.rank; ++k)
      if (d.ext[k] < 1 || d.ext[k] > 4096) throw std::invalid_argument("tensor extent out of range");
    if (d.n_sym < 0 || d.n_sym > MBC_EGRAPH_MAX_SYM) throw std::invalid_argument("too many symmetry generators");
    for (int s = 0; s < d.n_sym; ++s) {
      if (d.sign[s] != 1 && d.sign[s] != -1) throw std::invalid_argument("symmetry sign must be +1 or -1");
      uint32_t seen = 0;
      for (int k = 0; k < d.rank; ++k) {
        const int p = d.perm[s][k];
        if (p < 0 || p >= d.rank || (seen >> p & 1u)) throw std::invalid_argument("symmetry is not a permutation");
        if (d.ext[p] != d.ext[k]) throw std::invalid_argument("symmetry exchanges slots of different extents");
        seen |= 1u << p;
      }
    }
    TensorInfo t;
    closure(d, &t);
    g.tensors.push_back(std::move(t));
  }
  g.constant = prob.constant;
  g.constant.resize(nt);
  const int n_terms = int(prob.term_begin.size()) - 1;
  if (n_terms < 1) throw std::invalid_argument("n_terms must be >= 1");
  g.n_input_terms = n_terms;
  Builder b{g};
  bool first = true;
  uint64_t open_mask = 0;
  int ext_of[MBC_EGRAPH_MAX_LABEL] = {};
  for (int k = 0; k < n_terms; ++k) {
    const int f0 = prob.term_begin[k], f1 = prob.term_begin[k + 1];
    if (f1 - f0 < 1 || f1 - f0 > MBC_EGRAPH_MAX_FACTORS) throw std::invalid_argument("a term needs 1..16 factors");
    Expr e;
    int cnt[MBC_EGRAPH_MAX_LABEL] = {};
    int ext[MBC_EGRAPH_MAX_LABEL] = {};
    i128 direct = 1;
    for (int i = f0; i < f1; ++i) {
      const mbc_tensor_factor& f = prob.factors[i];
      if (f.tensor < 0 || f.tensor >= nt) throw std::invalid_argument("factor names an undeclared tensor");
      Fac x;
      x.t = f.tensor;
      for (int s = 0; s < prob.decls[f.tensor].rank; ++s) {
        const int l = f.label[s];
        if (l < 0 || l >= MBC_EGRAPH_MAX_LABEL) throw std::invalid_argument("label out of range");
        if (++cnt[l] > 2) throw std::invalid_argument("a label occurs more than twice in a term");
        const int xe = prob.decls[f.tensor].ext[s];
        if (ext[l] && ext[l] != xe) throw std::invalid_argument("a label has two extents");
        ext[l] = xe;
        x.lab[s] = uint8_t(l);
      }
      e.push_back(x);
    }
    uint64_t om = 0;
    for (int l = 0; l < MBC_EGRAPH_MAX_LABEL; ++l) {
      if (cnt[l] == 1) om |= uint64_t(1) << l;
      if (cnt[l]) direct *= ext[l];
    }
    if (first) {
      open_mask = om;
      std::memcpy(ext_of, ext, sizeof(ext));
      first = false;
    } else if (om != open_mask) {
      throw std::invalid_argument("terms have different open labels");
    }
    g.flops_direct += double(8 * (i128(e.size()) - 1) * direct);
    int sign;
    std::vector<uint8_t> opens;
    const int c = b.add_expr(e, &sign, &opens);
    if (c < 0) continue;
    TermRoot r;
    r.cls = c;
    r.re = prob.coef[2 * k] * sign;
    r.im = prob.coef[2 * k + 1] * sign;
    r.opens = opens;
    g.terms.push_back(std::move(r));
  }
  for (int l = 0; l < MBC_EGRAPH_MAX_LABEL; ++l)
    if (open_mask >> l & 1u) {
      g.out_labels.push_back(uint8_t(l));
      g.out_ext.push_back(ext_of[l]);
      g.out_elems *= ext_of[l];
    }

  // saturation (first in, first out), then the fallback split
  for (;;) {
    while (g.work_head < g.work.size()) {
      const int cid = g.work[g.work_head++];
      if (g.cls[cid].factors.size() < 2) continue;
      b.expand(cid, node_limit);
    }
    std::vector<int> missing;
    for (int c = 0; c < int(g.cls.size()); ++c)
      if (g.find(c) == c && g.cls[c].factors.size() >= 2 && g.cls[c].nodes.empty()) missing.push_back(c);
    if (missing.empty()) break;
    for (int c : missing) {
      const Expr cf = g.cls[c].factors;
      const uint32_t m = greedy_split(cf, g.tensors);
      Expr p[2];
      for (int i = 0; i < int(cf.size()); ++i) p[(m >> i & 1u) ? 0 : 1].push_back(cf[i]);
      b.add_node(c, p[0], p[1]);
      if (g.cls[c].nodes.empty()) throw std::domain_error("a sub-expression vanishes identically");
    }
  }

  // extraction
  const int nc = int(g.cls.size());
  std::vector<int> npar(nc, 0);
  {
    std::vector<std::vector<int>> par(nc);
    for (int c = 0; c < nc; ++c) {
      if (g.find(c) != c) continue;
      for (const ENode& nd : g.cls[c].nodes)
        for (int k : {nd.c1, nd.c2}) {
          auto& v = par[g.find(k)];  // distinct parent classes
          if (std::find(v.begin(), v.end(), c) == v.end()) v.push_back(c);
        }
    }
    for (int c = 0; c < nc; ++c) npar[c] = int(par[c].size());
  }
  auto is_leaf = [&](int c) { return g.cls[g.find(c)].factors.size() < 2; };
  auto naive = [&](int c) -> i128 {
    const EClass& k = g.cls[c];
    if (k.factors.size() < 2) return 0;
    return 8 * i128(k.factors.size() - 1) * prod_ext(k, k.labels);
  };
  auto node_flops = [&](int c, const ENode& nd) -> i128 {
    uint64_t m = 0;
    for (uint8_t x : nd.o1) m |= uint64_t(1) << x;
    for (uint8_t x : nd.o2) m |= uint64_t(1) << x;
    return 8 * prod_ext(g.cls[c], m);
  };
  std::vector<i128> memo(nc, -1);
  std::function<i128(int)> tree_cost = [&](int c) -> i128 {
    c = g.find(c);
    if (is_leaf(c)) return 0;
    if (memo[c] < 0) {
      i128 best = -1;
      for (const ENode& nd : g.cls[c].nodes) {
        const i128 v = node_flops(c, nd) + tree_cost(nd.c1) + tree_cost(nd.c2);
        if (best < 0 || v < best) best = v;
      }
      memo[c] = best;
    }
    return memo[c];
  };
  std::vector<int> choice(nc, -1);
  std::function<void(int)> pick = [&](int c) {
    c = g.find(c);
    if (choice[c] >= 0 || is_leaf(c)) return;
    const std::vector<ENode>& nodes = g.cls[c].nodes;
    int best = 0;
    i128 bk0 = 0, bk1 = 0;
    for (int i = 0; i < int(nodes.size()); ++i) {
      const ENode& nd = nodes[i];
      i128 k0, k1 = 0;
      if (objective == MBC_EXTRACT_REUSE) {
        i128 score = 0;
        const int kids[2] = {nd.c1, nd.c2};
        for (int j = 0; j < 2; ++j) {
          if (j == 1 && kids[1] == kids[0]) break;
          const int kc = g.find(kids[j]);
          if (is_leaf(kc)) continue;
          const int np = npar[kc] > 0 ? npar[kc] : 1;
          score += i128(np - 1) * naive(kc);
        }
        k0 = -score;
        k1 = node_flops(c, nd);
      } else {
        k0 = node_flops(c, nd) + tree_cost(nd.c1) + tree_cost(nd.c2);
      }
      if (i == 0 || k0 < bk0 || (k0 == bk0 && k1 < bk1)) {
        best = i;
        bk0 = k0;
        bk1 = k1;
      }
    }
    choice[c] = best;
    pick(nodes[best].c1);
    pick(nodes[best].c2);
  };
  // roots: terms merged by (class, open map), in order of first appearance;
  // exact zeros dropped (those terms cancel)
  for (const TermRoot& r : g.terms) {
    const int c = g.find(r.cls);
    bool merged = false;
    for (TermRoot& q : g.roots)
      if (q.cls == c && q.opens == r.opens) {
        q.re += r.re;
        q.im += r.im;
        merged = true;
        break;
      }
    if (!merged) {
      TermRoot q = r;
      q.cls = c;
      g.roots.push_back(q);
    }
  }
  g.roots.erase(std::remove_if(g.roots.begin(), g.roots.end(),
                               [](const TermRoot& q) { return q.re == 0.0 && q.im == 0.0; }),
                g.roots.end());
  for (const TermRoot& r : g.roots) pick(r.cls);
  if (objective == MBC_EXTRACT_SHARED) {
    // Sharing-aware refinement of the tree-cost choice: in rounds (at most
    // 10), with P the classes of the current plan, every class of P (by id)
    // takes the e-node minimising its own flops plus the tree cost of each
    // distinct child with two or more factors that is not in P; a change is
    // kept only if strictly cheaper, and new children get their tree-cost
    // choice.
    std::function<void(int)> tree_pick = [&](int c) {
      c = g.find(c);
      if (choice[c] >= 0 || is_leaf(c)) return;
      const std::vector<ENode>& nodes = g.cls[c].nodes;
      int best = 0;
      i128 bv = -1;
      for (int i = 0; i < int(nodes.size()); ++i) {
        const i128 v = node_flops(c, nodes[i]) + tree_cost(nodes[i].c1) + tree_cost(nodes[i].c2);
        if (bv < 0 || v < bv) {
          best = i;
          bv = v;
        }
      }
      choice[c] = best;
      tree_pick(nodes[best].c1);
      tree_pick(nodes[best].c2);
    };
    for (int round = 0; round < 10; ++round) {
      std::vector<char> in_plan(nc, 0);
      std::vector<int> P, stack;
      for (const TermRoot& r : g.roots) stack.push_back(r.cls);
      while (!stack.empty()) {
        const int c = g.find(stack.back());
        stack.pop_back();
        if (in_plan[c] || is_leaf(c)) continue;
        in_plan[c] = 1;
        P.push_back(c);
        const ENode& nd = g.cls[c].nodes[choice[c]];
        stack.push_back(nd.c1);
        stack.push_back(nd.c2);
      }
      std::sort(P.begin(), P.end());
      bool changed = false;
      for (int c : P) {
        const std::vector<ENode>& nodes = g.cls[c].nodes;
        auto cost = [&](const ENode& nd) {
          i128 v = node_flops(c, nd);
          const int k1 = g.find(nd.c1), k2 = g.find(nd.c2);
          if (!in_plan[k1] && !is_leaf(k1)) v += tree_cost(k1);
          if (k2 != k1 && !in_plan[k2] && !is_leaf(k2)) v += tree_cost(k2);
          return v;
        };
        int best = 0;
        i128 bv = cost(nodes[0]);
        for (int i = 1; i < int(nodes.size()); ++i) {
          const i128 v = cost(nodes[i]);
          if (v < bv) {
            best = i;
            bv = v;
          }
        }
        if (bv < cost(nodes[choice[c]])) {
          choice[c] = best;
          changed = true;
          tree_pick(nodes[best].c1);
          tree_pick(nodes[best].c2);
        }
      }
      if (!changed) break;
    }
  }

  // steps: post-order from the terms, each class once
  g.step_of.assign(nc, -1);
  std::function<void(int)> visit = [&](int c) {
    c = g.find(c);
    if (g.step_of[c] >= 0 || is_leaf(c)) return;
    const ENode& nd = g.cls[c].nodes[choice[c]];
    visit(nd.c1);
    visit(nd.c2);
    // the executor addresses at most 16 open and 16 summed labels per step
    int shared = 0, traces = 0;
    for (uint8_t x : nd.o1) shared += std::count(nd.o2.begin(), nd.o2.end(), x) > 0;
    for (int k : {nd.c1, nd.c2}) {
      const EClass& ch = g.cls[g.find(k)];
      if (ch.factors.size() == 1)
        for (int x = 0; x < MBC_EGRAPH_MAX_LABEL; x += 2) traces += (ch.labels >> x & 1u) ? 1 : 0;
    }
    if (g.cls[c].n_open > 16 || shared + traces > 16)
      throw std::domain_error("a plan step has more than 16 open or summed labels");
    Step s;
    s.cls = c;
    s.node = choice[c];
    s.elems = 1;
    for (int e : g.cls[c].open_ext) s.elems *= e;
    s.ws_off = g.ws_elems;
    g.ws_elems += s.elems;
    g.step_of[c] = int(g.steps.size());
    g.steps.push_back(s);
    g.flops_plan += double(node_flops(c, nd));
  };
  for (const TermRoot& r : g.roots) visit(r.cls);
  g.flops_plan += 8.0 * double(g.out_elems) * double(g.roots.size());
}

}  // namespace mbc
