// Plan compiler: turns a canonical index set into the evaluation schedule the
// kernels interpret.
//
// Evaluation order (factor tree of Sec. 4 over the determinant form of eq. 1):
//   C_c(x) = sum_{runs rho} sum_{s} Du[r_u(rho), c_u(s)] * L_{rho,s},
//   L_{rho,s} = sum_{b in rho} W[b, s] * Dd[r_d(b), c_d(s)],
// where a run is a maximal set of sink keys sharing their u-tuple (the first
// factor of the tree) and s runs over the correlator's source keys.
//
// Determinants are rows of compound matrices built by the Laplace expansion
// along the first row,
//   M_k(r, C) = sum_j (-1)^j S[r_0, C_j] M_{k-1}(r[1:], C \ C_j),
// so a level-k row (fixed row tuple, all needed column k-subsets) is made
// from the level-(k-1) row of its suffix r[1:]; every minor of the tile's
// rows is computed once per tile and shared by all determinants that need it.
//
// Sink keys are sorted by their reversed u-tuple so that equal u-tuples (runs)
// and equal u-suffixes are adjacent; tiles are groups of whole runs sized to a
// local-memory budget.
#include <algorithm>
#include <map>
#include <set>
#include <stdexcept>

#include "mbc_internal.hpp"

namespace mbc {

namespace {

Key drop(const Key& c, int j) {
  Key r;
  r.n = uint8_t(c.n - 1);
  int w = 0;
  for (int i = 0; i < c.n; ++i)
    if (i != j) r.v[w++] = c.v[i];
  return r;
}

Key tail(const Key& c, int k) {  // last k elements
  Key r;
  r.n = uint8_t(k);
  for (int i = 0; i < k; ++i) r.v[i] = c.v[c.n - k + i];
  return r;
}

void k_subsets(const Key& c, int k, std::set<Key>* out) {
  // all k-element subsequences of a sorted tuple (bitmask enumeration)
  const int n = c.n;
  for (int mask = 0; mask < (1 << n); ++mask) {
    if (__builtin_popcount(mask) != k) continue;
    Key s;
    s.n = uint8_t(k);
    int w = 0;
    for (int i = 0; i < n; ++i)
      if (mask & (1 << i)) s.v[w++] = c.v[i];
    out->insert(s);
  }
}

struct Levels {
  int n = 0;
  std::vector<std::vector<Key>> cols;     // cols[k], k = 1..n
  std::vector<std::map<Key, int>> index;  // index[k]
};

// Needed columns of every level.  `top` lists the source tuples with their
// multiplicity; the top level is ordered by decreasing multiplicity (the
// length of a column's source-key list), so that the threads of a wavefront,
// which own consecutive top columns, walk lists of similar length.
Levels column_levels(const std::vector<Key>& top, int n) {
  Levels L;
  L.n = n;
  L.cols.resize(n + 1);
  L.index.resize(n + 1);
  for (int k = 1; k <= n; ++k) {
    std::set<Key> s;
    for (const Key& c : top) k_subsets(c, k, &s);
    L.cols[k].assign(s.begin(), s.end());
    if (k == n) {
      std::map<Key, int> mult;
      for (const Key& c : top) ++mult[c];
      std::stable_sort(L.cols[k].begin(), L.cols[k].end(),
                       [&](const Key& a, const Key& b) { return mult[a] > mult[b]; });
    }
    for (size_t i = 0; i < L.cols[k].size(); ++i) L.index[k][L.cols[k][i]] = int(i);
  }
  return L;
}

struct RowId {
  int f, k;
  Key t;
  bool operator<(const RowId& o) const {
    if (k != o.k) return k < o.k;
    if (f != o.f) return f < o.f;
    return t < o.t;
  }
};

bool rev_less(const Key& a, const Key& b) {
  for (int i = a.n - 1; i >= 0; --i)
    if (a.v[i] != b.v[i]) return a.v[i] < b.v[i];
  return false;
}

// rows (with their suffix chains) needed by a set of top rows
void add_chain(int f, const Key& top, std::set<RowId>* rows) {
  const int n = top.n;
  if (n == 1) {
    rows->insert({f, 1, top});
    return;
  }
  for (int k = n; k >= 2; --k) rows->insert({f, k, tail(top, k)});
}

}  // namespace

namespace {

// Everything about one correlator the tilings need.
struct CorrCtx {
  int c = 0, n_src = 0, n_snk = 0;
  int nf[2] = {0, 0};
  std::vector<std::pair<Key, Key>> snk, src;  // sink keys in plan order; source keys
  Levels lev[2];
  int tab_off[2][kMaxQuarks + 1] = {};
  int64_t w_base = 0;
  int ncol(int f, int k) const { return int(lev[f].cols[k].size()); }
};

struct TileSetOut {
  std::vector<int32_t>* tiles;
  std::vector<int32_t>* ops;
  std::vector<int32_t>* meta;
  std::vector<int32_t>* extra;  // backward only
  int* n_tiles;
  int* max_ops;
  int* max_b;
  double* exec;                 // forward flop count (forward tiling only)
};

// LDS model of a tile: complex units of (S, W, rows) plus bytes of staged records.
struct LdsModel {
  bool backward;  // dS kernel (rows carry a zero element, adjoint rows)
  int csz;
  bool with_w = true;     // forward: the tile's weights are staged (not for dW)
  bool factored = false;  // the n_src + B weight factors instead of B x n_src weights
  int64_t weights(int B, int n_src) const { return factored ? int64_t(n_src) + B : int64_t(B) * n_src; }
  int64_t operator()(int B, int n_src, int64_t row_units, int n_ops, int n_virt, int64_t n_child) const {
    if (!backward) {
      int64_t bytes = (576 + (with_w ? int64_t(B) * n_src : 0) + row_units) * csz;
      return ((bytes + 15) & ~int64_t(15)) + int64_t(n_ops) * 16 + int64_t(B) * 16;
    }
    // dS kernel: S, W (or its factors), rows, adjoint rows, level-1 adjoints,
    // per-op j-partials, S-bar accumulators (16 B each), staged op records
    // and child lists
    const int64_t ds = (288 + weights(B, n_src) + 2 * row_units + 12 * int64_t(n_virt) + 12 * int64_t(n_ops)) * csz +
                       288 * 16 + int64_t(n_ops + n_virt) * 32 + n_child * 4 + 64 * 4;
    return ds;
  }
};

void rows_of(const CorrCtx& X, const std::vector<int>& sk, std::set<RowId>* rows) {
  for (int i : sk) {
    add_chain(0, X.snk[i].first, rows);
    add_chain(1, X.snk[i].second, rows);
  }
}

int64_t tile_lds(const CorrCtx& X, const std::vector<int>& sk, const LdsModel& m) {
  std::set<RowId> rows;
  rows_of(X, sk, &rows);
  int64_t units = 0;
  int n_virt = 0;
  std::set<std::pair<int, int>> v1;
  for (auto& r : rows) {
    units += X.ncol(r.f, r.k) + (m.backward ? 1 : 0);
    if (r.k == 2) v1.insert({r.f, r.t.v[1]});
  }
  n_virt = int(v1.size());
  return m(int(sk.size()), X.n_src, units, int(rows.size()), n_virt, int64_t(rows.size()));
}

// Greedy tiling of the sink keys (plan order) into groups of whole runs of
// equal u-tuples under an LDS budget; a run longer than a tile is split.
std::vector<std::vector<int>> make_tiles(const CorrCtx& X, int64_t budget, int max_b, const LdsModel& m) {
  std::vector<std::vector<int>> tiles;
  std::vector<int> cur;
  for (int i = 0; i < X.n_snk;) {
    int j = i + 1;
    while (j < X.n_snk && X.snk[j].first == X.snk[i].first) ++j;
    std::vector<int> trial = cur;
    for (int q = i; q < j; ++q) trial.push_back(q);
    if (!cur.empty() && (int(trial.size()) > max_b || tile_lds(X, trial, m) > budget)) {
      tiles.push_back(cur);
      cur.clear();
    }
    for (int q = i; q < j; ++q) {
      std::vector<int> t2 = cur;
      t2.push_back(q);
      if (!cur.empty() && (int(t2.size()) > max_b || tile_lds(X, t2, m) > budget)) {
        tiles.push_back(cur);
        cur.clear();
      }
      cur.push_back(q);
    }
    i = j;
  }
  if (!cur.empty()) tiles.push_back(cur);
  return tiles;
}

// Emits the records of one tiling.  Returns the largest LDS of a tile.
int64_t emit_tiles(const CorrCtx& X, const std::vector<std::vector<int>>& tiles, const LdsModel& m,
                   TileSetOut& o) {
  int64_t max_lds = 0;
  for (auto& sk : tiles) {
    const int B = int(sk.size());
    std::set<RowId> rowset;
    rows_of(X, sk, &rowset);
    std::map<RowId, int> slot;
    // backward rows carry one trailing zero element after their ncol columns:
    // padded table entries of the reverse sweep point there
    const bool pad_rows = o.extra != nullptr;
    int units = 0;
    for (auto& r : rowset) {
      slot[r] = units;
      units += X.ncol(r.f, r.k) + (pad_rows ? 1 : 0);
    }
    std::vector<int32_t> tr(kTileInts, 0);
    tr[0] = X.c;
    tr[1] = B;
    tr[2] = int32_t(X.w_base + int64_t(sk[0]) * X.n_src);
    tr[3] = int32_t(o.ops->size() / kOpInts);
    tr[5] = int32_t(o.meta->size() / kMetaInts);
    tr[6] = units;
    tr[16] = sk[0];
    std::vector<RowId> order(rowset.begin(), rowset.end());
    std::map<RowId, int> op_index;
    int n_ops = 0, phase = -1, cur_level = 0;
    for (auto& r : order) {
      if (r.k != cur_level) {
        ++phase;
        if (phase >= 5) throw std::runtime_error("too many phases (at most five levels of rows per tile)");
        tr[8 + phase] = n_ops;
        cur_level = r.k;
      }
      if (tr[21 + 2 * (7 * r.f + r.k)] == 0) tr[20 + 2 * (7 * r.f + r.k)] = n_ops;
      ++tr[21 + 2 * (7 * r.f + r.k)];
      op_index[r] = n_ops;
      ++n_ops;
      if (r.k >= 2 && o.exec) *o.exec += double(X.ncol(r.f, r.k)) * (8.0 * r.k - 2.0);
    }
    tr[4] = n_ops;
    tr[7] = phase + 1;
    tr[8 + phase + 1] = n_ops;
    // level-1 parents (S rows) of the level-2 rows, and children lists
    std::vector<std::pair<int, int>> virt;  // (f, r1)
    std::map<std::pair<int, int>, int> virt_index;
    for (auto& r : order)
      if (r.k == 2 && !virt_index.count({r.f, r.t.v[1]})) {
        virt_index[{r.f, r.t.v[1]}] = int(virt.size());
        virt.push_back({r.f, r.t.v[1]});
      }
    std::vector<std::vector<int>> children(size_t(n_ops) + virt.size());
    for (auto& r : order) {
      if (r.k == 2) children[n_ops + virt_index.at({r.f, r.t.v[1]})].push_back(op_index.at(r));
      if (r.k >= 3) children[op_index.at({r.f, r.k - 1, tail(r.t, r.k - 1)})].push_back(op_index.at(r));
    }
    const bool bwd = o.extra != nullptr;
    int64_t child_total = 0;
    int item_begin = 0;
    cur_level = 0;
    for (auto& r : order) {
      if (r.k != cur_level) {
        cur_level = r.k;
        item_begin = 0;
      }
      int in = 0;
      if (r.k == 2) in = r.t.v[1];
      if (r.k >= 3) in = slot.at({r.f, r.k - 1, tail(r.t, r.k - 1)});
      const int nc = X.ncol(r.f, r.k);
      const int oi = op_index.at(r);
      int32_t op[kOpInts] = {r.f, r.k, r.t.v[0], in, slot.at(r), X.tab_off[r.f][r.k], nc, item_begin};
      if (bwd) {
        op[5] = int32_t(child_total);
        op[6] = int32_t(children[oi].size());
        op[7] = 0;
        child_total += int64_t(children[oi].size());
      }
      o.ops->insert(o.ops->end(), op, op + kOpInts);
      item_begin += nc;
    }
    if (bwd) {
      tr[17] = n_ops;
      tr[18] = int32_t(virt.size());
      for (auto& v : virt) tr[14] += (v.first == 0);  // level-1 records of the u flavour come first
      for (size_t v = 0; v < virt.size(); ++v) {
        const auto& ch = children[n_ops + v];
        const int32_t op[kOpInts] = {virt[v].first, 1, virt[v].second, 0, int32_t(12 * v),
                                     int32_t(child_total), int32_t(ch.size()), 1};
        child_total += int64_t(ch.size());
        o.ops->insert(o.ops->end(), op, op + kOpInts);
      }
      tr[4] = n_ops + int32_t(virt.size());
    }
    // per sink key metadata
    for (int b = 0; b < B; ++b) {
      const int i = sk[b];
      const bool run_end = (b + 1 == B) || !(X.snk[sk[b + 1]].first == X.snk[i].first);
      const int u_slot = slot.at({0, X.nf[0], X.snk[i].first});
      const int d_slot = slot.at({1, X.nf[1], X.snk[i].second});
      bool first_d = true;  // no earlier key of the tile shares the d-tuple
      for (int q = 0; q < b && first_d; ++q) first_d = !(X.snk[sk[q]].second == X.snk[i].second);
      const int32_t flags = (run_end ? 1 : 0) | ((m.factored && first_d) ? 2 : 0);
      const int32_t mm[kMetaInts] = {u_slot, d_slot, flags, i};
      o.meta->insert(o.meta->end(), mm, mm + kMetaInts);
      if (o.exec) *o.exec += 8.0 * X.n_src + (run_end ? 8.0 * X.n_src : 0.0);
    }
    if (bwd) {
      tr[19] = int32_t(o.extra->size());
      std::vector<int32_t> runs, dgs;
      std::map<int, int> dmask;
      for (int b = 0; b < B;) {
        int e = b + 1;
        while (e < B && X.snk[sk[e]].first == X.snk[sk[b]].first) ++e;
        runs.insert(runs.end(), {slot.at({0, X.nf[0], X.snk[sk[b]].first}), b, e});
        b = e;
      }
      for (int b = 0; b < B; ++b) dmask[slot.at({1, X.nf[1], X.snk[sk[b]].second})] |= (1 << b);
      for (auto& kv : dmask) dgs.insert(dgs.end(), {kv.first, kv.second});
      // rows of S-bar touched by the tile: for each (flavour, S row r0), the
      // records (real rows with that first row, level-1 parents of that row)
      std::vector<std::vector<int32_t>> rsum(24);
      for (auto& r : order) rsum[12 * r.f + r.t.v[0]].push_back(op_index.at(r));
      for (size_t v = 0; v < virt.size(); ++v) rsum[12 * virt[v].first + virt[v].second].push_back(n_ops + int(v));
      int64_t nchild = 0;
      for (auto& ch : children) nchild += int64_t(ch.size());
      o.extra->push_back(int32_t(runs.size() / 3));
      o.extra->push_back(int32_t(dgs.size() / 2));
      o.extra->push_back(int32_t(3 + runs.size() + dgs.size() + nchild));  // offset of the S-bar row lists
      o.extra->insert(o.extra->end(), runs.begin(), runs.end());
      o.extra->insert(o.extra->end(), dgs.begin(), dgs.end());
      // children as (row slot << 4 | first row r0), what the parent sums read
      for (auto& ch : children)
        for (int ci : ch) o.extra->push_back(int32_t(slot.at(order[size_t(ci)]) << 4) | order[size_t(ci)].t.v[0]);
      int32_t acc = 25;
      for (int q = 0; q < 24; ++q) {
        o.extra->push_back(acc);
        acc += int32_t(rsum[q].size());
      }
      o.extra->push_back(acc);
      for (auto& v : rsum) o.extra->insert(o.extra->end(), v.begin(), v.end());
    }
    int64_t lds = m(B, X.n_src, units, n_ops, bwd ? int(virt.size()) : 0, child_total);
    if (bwd) {
      const int nv = int(virt.size());
      const int64_t ex_len = int64_t(o.extra->size()) - tr[19];
      tr[15] = int32_t(ex_len);
      // dS kernel layout: S, W, rows, adjoint rows, level-1 adjoints, per-row
      // S-bar partials (complex, rounded up to 16 B), then int4 op records
      // (real ops; all ops twice), the extra ints (rounded up to 8 B) and the
      // (u slot, d slot) pairs of the sink keys
      int64_t cunits = 288 + m.weights(B, X.n_src) + 2 * int64_t(units) + 12 * int64_t(nv) + 12 * int64_t(n_ops);
      int64_t bytes = cunits * m.csz;
      bytes = (bytes + 15) & ~int64_t(15);
      lds = bytes + int64_t(n_ops + 2 * (n_ops + nv)) * 16 + ((ex_len + 1) & ~int64_t(1)) * 4 + int64_t(B) * 8;
    }
    if (lds > 160 * 1024) throw std::runtime_error("a tile exceeds the 160 KiB local memory of a CU");
    max_lds = std::max(max_lds, lds);
    *o.max_ops = std::max(*o.max_ops, int(tr[4]));
    *o.max_b = std::max(*o.max_b, B);
    o.tiles->insert(o.tiles->end(), tr.begin(), tr.end());
    ++*o.n_tiles;
  }
  return max_lds;
}

// Backward tables of one correlator (see the correlator record layout).
void backward_tables(const CorrCtx& X, int32_t* cr, std::vector<int32_t>& btab) {
  for (int f = 0; f < 2; ++f) {
    for (int k = 1; k <= X.nf[f]; ++k) {
      const auto& cols = X.lev[f].cols[k];
      // j-lists of level k
      cr[40 + 6 * f + k - 1] = int32_t(btab.size());
      std::vector<std::vector<int32_t>> jl(12);
      for (size_t i = 0; i < cols.size(); ++i) {
        const Key& C = cols[i];
        for (int pos = 0; pos < k; ++pos) {
          int32_t e;
          if (k == 1) {
            e = int32_t(i) | (int32_t(C.v[0]) << 12);
          } else {
            const Key rest = drop(C, pos);
            const int sub = (k == 2) ? rest.v[0] : X.lev[f].index[k - 1].at(rest);
            e = int32_t(i) | (sub << 12) | (pos << 24);
          }
          jl[C.v[pos]].push_back(e);
        }
      }
      for (int j = 0; j < 12; ++j) cr[82 + 6 * f + k - 1] = std::max<int32_t>(cr[82 + 6 * f + k - 1], int32_t(jl[j].size()));
      const size_t base = btab.size();
      btab.resize(base + 13);
      int32_t acc = 13;
      for (int j = 0; j < 12; ++j) {
        btab[base + j] = acc;
        acc += int32_t(jl[j].size());
      }
      btab[base + 12] = acc;
      for (int j = 0; j < 12; ++j) btab.insert(btab.end(), jl[j].begin(), jl[j].end());
      // superset lists: parents at level k, children at level k + 1
      if (k < X.nf[f]) {
        cr[52 + 6 * f + k - 1] = int32_t(btab.size());
        std::vector<std::vector<int32_t>> sup(cols.size());
        const auto& up = X.lev[f].cols[k + 1];
        for (size_t i = 0; i < up.size(); ++i)
          for (int pos = 0; pos < k + 1; ++pos) {
            const Key rest = drop(up[i], pos);
            const int pi = X.lev[f].index[k].at(rest);
            sup[pi].push_back(int32_t(i) | (int32_t(up[i].v[pos]) << 12) | (pos << 16));
          }
        const size_t b2 = btab.size();
        btab.resize(b2 + cols.size() + 1);
        int32_t a2 = int32_t(cols.size() + 1);
        for (size_t i = 0; i < cols.size(); ++i) {
          btab[b2 + i] = a2;
          a2 += int32_t(sup[i].size());
        }
        btab[b2 + cols.size()] = a2;
        for (auto& v : sup) btab.insert(btab.end(), v.begin(), v.end());
      }
    }
  }
  // "up" tables of the parent levels: for each column C' of level k < n_f and
  // each column number j, the index of C' + {j} in level k + 1 (0xffff if it
  // is not a needed column), packed two per int32
  for (int f = 0; f < 2; ++f)
    for (int k = 1; k < X.nf[f]; ++k) {
      cr[67 + 6 * f + k - 1] = int32_t(btab.size());
      const auto& cols = X.lev[f].cols[k];
      std::vector<int> n_up(cols.size(), 0);
      for (size_t ci = 0; ci < cols.size(); ++ci) {
        const Key& Cp = cols[ci];
        uint32_t pk[6] = {0, 0, 0, 0, 0, 0};
        for (int j = 0; j < 12; ++j) {
          int idx = 0xffff;
          bool in = false;
          for (int q = 0; q < Cp.n; ++q) in |= (Cp.v[q] == j);
          if (!in) {
            Key up;
            up.n = uint8_t(k + 1);
            int w = 0;
            bool put = false;
            for (int q = 0; q < Cp.n; ++q) {
              if (!put && j < Cp.v[q]) { up.v[w++] = uint8_t(j); put = true; }
              up.v[w++] = Cp.v[q];
            }
            if (!put) up.v[w++] = uint8_t(j);
            auto it = X.lev[f].index[k + 1].find(up);
            if (it != X.lev[f].index[k + 1].end()) {
              int pos = 0;
              for (int q = 0; q < Cp.n; ++q) pos += Cp.v[q] < j;
              if (it->second >= 4096) throw std::runtime_error("column list too long");
              idx = it->second | (pos << 12);
              ++n_up[ci];
            }
          }
          pk[j / 2] |= (uint32_t(idx) & 0xffffu) << (16 * (j % 2));
        }
        for (uint32_t w : pk) btab.push_back(int32_t(w));
      }
      // then the columns ordered by their number of supersets (most first),
      // so that the columns a wave takes have similar counts
      std::vector<int32_t> perm(cols.size());
      for (size_t ci = 0; ci < cols.size(); ++ci) perm[ci] = int32_t(ci);
      std::stable_sort(perm.begin(), perm.end(), [&](int32_t x, int32_t y) { return n_up[x] > n_up[y]; });
      btab.insert(btab.end(), perm.begin(), perm.end());
    }
  // source keys grouped by their top u column and by their top d column
  for (int f = 0; f < 2; ++f) {
    const int ntop = X.ncol(f, X.nf[f]);
    std::vector<std::vector<int32_t>> lists(ntop);
    for (int s = 0; s < X.n_src; ++s) {
      const Key& col = f == 0 ? X.src[s].first : X.src[s].second;
      lists[X.lev[f].index[X.nf[f]].at(col)].push_back(s);
    }
    cr[64 + f] = int32_t(btab.size());
    for (auto& v : lists) cr[80 + f] = std::max<int32_t>(cr[80 + f], int32_t(v.size()));
    const size_t b3 = btab.size();
    btab.resize(b3 + ntop + 1);
    int32_t a3 = ntop + 1;
    for (int i = 0; i < ntop; ++i) {
      btab[b3 + i] = a3;
      a3 += int32_t(lists[i].size());
    }
    btab[b3 + ntop] = a3;
    for (auto& v : lists) btab.insert(btab.end(), v.begin(), v.end());
  }
}

}  // namespace

void compile_plan(const IndexSet& s, int precision, PlanHost* out) {
  if (!s.canonical) throw std::invalid_argument("plans need a canonical (symmetrised) index set");
  if (s.n_corr < 1) throw std::invalid_argument("empty batch of correlators");
  if (s.n_u < 1 || s.n_u > kMaxQuarks || s.n_d < 1 || s.n_d > kMaxQuarks)
    throw std::invalid_argument("n_u and n_d must lie in 1..6");
  PlanHost& P = *out;
  P = PlanHost();
  P.n_u = s.n_u;
  P.n_d = s.n_d;
  P.n_corr = s.n_corr;
  P.precision = precision;
  P.nnz = int64_t(s.entries.size());
  P.threads = family_threads(s.n_u, s.n_d);
  const int csz = precision == MBC_F64 ? 16 : 8;
  // local-memory budgets per workgroup (forward; backward dS kernel), sized
  // to the workgroups per CU that the kernels' registers allow (measured
  // best on the D_I bench workload): two share a CU's 160 KiB, four for the
  // FP32 forward of the small families; the (5,4) family's 512-thread
  // workgroups run one per CU, so their tiles may take nearly all of it
  const bool big = s.n_u + s.n_d >= 8;
  const int64_t budget = big ? 150 * 1024 : (precision == MBC_F64 ? 76 : 38) * 1024;
  const int64_t bbudget = big ? 150 * 1024 : (precision == MBC_F64 ? 76 : 78) * 1024;
  const int kMaxB = 16;
  const LdsModel fwd_model{false, csz}, bwd_model{true, csz}, dw_model{false, csz, false};
  const LdsModel bwdf_model{true, csz, true, true};
  P.rank1 = true;
  const int dw_keys = dw_keys_per_tile(s.n_u, s.n_d, precision);
  P.corr.assign(size_t(s.n_corr) * kCorrInts, 0);
  P.w_exact.assign(size_t(2 * P.nnz), 0.0);
  P.perm.assign(size_t(P.nnz), 0);
  int64_t w_pos = 0;
  double alg = 0, exec = 0, ds_alg = 0, dw_alg = 0, fact_alg = 0, fact_ds_alg = 0;
  TileSetOut fo{&P.tiles, &P.ops, &P.meta, nullptr, &P.n_tiles, &P.max_ops, &P.max_b, &exec};
  TileSetOut bo{&P.b_tiles, &P.b_ops, &P.b_meta, &P.b_extra, &P.b_n_tiles, &P.b_max_ops, &P.b_max_b, nullptr};
  TileSetOut wo{&P.w_tiles, &P.w_ops, &P.w_meta, nullptr, &P.w_n_tiles, &P.w_max_ops, &P.w_max_b, nullptr};
  TileSetOut fo2{&P.f_tiles, &P.f_ops, &P.f_meta, &P.f_extra, &P.f_n_tiles, &P.f_max_ops, &P.f_max_b, nullptr};

  for (int c = 0; c < s.n_corr; ++c) {
    int32_t* cr = &P.corr[size_t(c) * kCorrInts];
    const int64_t e0 = s.corr_begin[c], e1 = s.corr_begin[c + 1];
    cr[3] = cr[4] = P.n_tiles;
    cr[6] = cr[7] = P.b_n_tiles;
    cr[5] = int32_t(e0);
    cr[66] = int32_t(w_pos);
    cr[1] = int32_t(P.src_cu.size());
    cr[32] = int32_t(P.wu.size() / 2);
    cr[33] = cr[34] = P.f_n_tiles;
    if (e0 == e1) continue;  // empty correlator: C = 0, no tiles
    CorrCtx X;
    X.c = c;
    X.nf[0] = s.n_u;
    X.nf[1] = s.n_d;
    X.w_base = w_pos;
    std::map<std::pair<Key, Key>, int> snk_id, src_id;
    for (int64_t e = e0; e < e1; ++e) {
      snk_id.emplace(std::make_pair(s.entries[e].ru, s.entries[e].rd), 0);
      src_id.emplace(std::make_pair(s.entries[e].cu, s.entries[e].cd), 0);
    }
    X.n_snk = int(snk_id.size());
    X.n_src = int(src_id.size());
    if (int64_t(X.n_snk) * X.n_src != e1 - e0)
      throw std::domain_error("index set of a correlator is not a Cartesian product of sink and source keys");
    for (auto& kv : snk_id) X.snk.push_back(kv.first);
    for (auto& kv : src_id) X.src.push_back(kv.first);
    // plan order of sink keys: by reversed u-tuple, then d-tuple
    std::sort(X.snk.begin(), X.snk.end(), [](const std::pair<Key, Key>& a, const std::pair<Key, Key>& b) {
      if (!(a.first == b.first)) return rev_less(a.first, b.first);
      return a.second < b.second;
    });
    for (int i = 0; i < X.n_snk; ++i) snk_id[X.snk[i]] = i;
    for (int i = 0; i < X.n_src; ++i) src_id[X.src[i]] = i;
    std::vector<int64_t> ent(size_t(X.n_snk) * X.n_src, -1);
    for (int64_t e = e0; e < e1; ++e) {
      const int i = snk_id[{s.entries[e].ru, s.entries[e].rd}];
      const int j = src_id[{s.entries[e].cu, s.entries[e].cd}];
      int64_t& sl = ent[size_t(i) * X.n_src + j];
      if (sl >= 0) throw std::domain_error("duplicate index-set entry");
      sl = e;
    }
    // plan-ordered weights: [sink key in plan order][source key]
    for (int i = 0; i < X.n_snk; ++i)
      for (int j = 0; j < X.n_src; ++j) {
        const int64_t e = ent[size_t(i) * X.n_src + j];
        P.perm[size_t(w_pos)] = e;
        const double den = double(s.w_den[c]);
        P.w_exact[size_t(2 * w_pos)] = double(s.entries[e].w_re) / den;
        P.w_exact[size_t(2 * w_pos + 1)] = double(s.entries[e].w_im) / den;
        ++w_pos;
      }
    // Exact weights as a product of a sink and a source vector: with the
    // pivot (0, j0) (j0 the largest weight of sink key 0), W is a product iff
    // W[i, j] W[0, j0] = W[i, j0] W[0, j] for every entry (checked in exact
    // Gaussian-integer arithmetic on the numerators); then
    // wu[i] = W[i, j0] and wv[j] = W[0, j] / W[0, j0].
    {
      auto num = [&](int i, int j) {
        const Entry& en = s.entries[ent[size_t(i) * X.n_src + j]];
        return std::make_pair(en.w_re, en.w_im);
      };
      int j0 = 0;
      __int128 best = -1;
      for (int j = 0; j < X.n_src; ++j) {
        const auto w = num(0, j);
        const __int128 n2 = __int128(w.first) * w.first + __int128(w.second) * w.second;
        if (n2 > best) {
          best = n2;
          j0 = j;
        }
      }
      const auto p = num(0, j0);
      bool prod = best > 0;
      for (int i = 0; i < X.n_snk && prod; ++i) {
        const auto a = num(i, j0);
        for (int j = 0; j < X.n_src; ++j) {
          const auto w = num(i, j), b = num(0, j);
          const __int128 lre = __int128(w.first) * p.first - __int128(w.second) * p.second;
          const __int128 lim = __int128(w.first) * p.second + __int128(w.second) * p.first;
          const __int128 rre = __int128(a.first) * b.first - __int128(a.second) * b.second;
          const __int128 rim = __int128(a.first) * b.second + __int128(a.second) * b.first;
          if (lre != rre || lim != rim) {
            prod = false;
            break;
          }
        }
      }
      P.rank1 = P.rank1 && prod;
      const double den = double(s.w_den[c]);
      const double pr = double(p.first), pi = double(p.second), pn = pr * pr + pi * pi;
      for (int i = 0; i < X.n_snk; ++i) {
        const auto a = num(i, j0);
        P.wu.push_back(double(a.first) / den);
        P.wu.push_back(double(a.second) / den);
      }
      for (int j = 0; j < X.n_src; ++j) {
        const auto b = num(0, j);
        const double br = double(b.first), bi = double(b.second);
        P.wv.push_back(prod ? (br * pr + bi * pi) / pn : 0.0);  // b / p
        P.wv.push_back(prod ? (bi * pr - br * pi) / pn : 0.0);
      }
    }
    // column levels per flavour: all k-subsets of the source tuples
    std::vector<Key> top_cols[2];
    for (auto& k : X.src) {
      top_cols[0].push_back(k.first);
      top_cols[1].push_back(k.second);
    }
    X.lev[0] = column_levels(top_cols[0], X.nf[0]);
    X.lev[1] = column_levels(top_cols[1], X.nf[1]);
    for (int f = 0; f < 2; ++f)
      for (int k = 1; k <= X.nf[f]; ++k) {
        const auto& cols = X.lev[f].cols[k];
        X.tab_off[f][k] = int(P.tabs.size());
        cr[8 + 2 * (6 * f + k - 1)] = int32_t(cols.size());
        cr[8 + 2 * (6 * f + k - 1) + 1] = int32_t(P.tabs.size());
        for (const Key& C : cols) {
          if (k == 1) {
            P.tabs.push_back(uint16_t(C.v[0]));
            continue;
          }
          for (int j = 0; j < k; ++j) {
            const Key rest = drop(C, j);
            const int sub = (k == 2) ? rest.v[0] : X.lev[f].index[k - 1].at(rest);
            if (sub >= 4096) throw std::runtime_error("column list too long");
            P.tabs.push_back(uint16_t((sub << 4) | C.v[j]));
          }
        }
      }
    cr[0] = X.n_src;
    cr[2] = X.n_snk;
    for (auto& k : X.src) {
      P.src_cu.push_back(X.lev[0].index[X.nf[0]].at(k.first));
      P.src_cd.push_back(X.lev[1].index[X.nf[1]].at(k.second));
    }
    P.max_src = std::max(P.max_src, X.n_src);
    for (int f = 0; f < 2; ++f)
      for (int k = 1; k <= X.nf[f]; ++k) P.max_ncol = std::max(P.max_ncol, X.ncol(f, k));
    backward_tables(X, cr, P.btab);

    // algorithmic flops (global minor DAG + leaves + (r_u, c_u) groups);
    // backward: the minors once more, the reverse sweep (k complex products
    // for the parent adjoint and k for the S adjoint per minor), both leaf
    // adjoint sums (dS); the minors and one product per entry (dW)
    double minors = 0, rev = 0;
    for (int f = 0; f < 2; ++f)
      for (int k = 2; k <= X.nf[f]; ++k) {
        std::set<Key> suf;
        for (auto& kk : X.snk) suf.insert(tail(f == 0 ? kk.first : kk.second, k));
        minors += double(suf.size()) * X.ncol(f, k) * (8.0 * k - 2.0);
        rev += double(suf.size()) * X.ncol(f, k) * 16.0 * k;
      }
    alg += minors;
    ds_alg += minors + rev + 16.0 * double(X.n_snk) * X.n_src;
    dw_alg += minors + 8.0 * double(X.n_snk) * X.n_src;
    {
      std::set<Key> ru, cu;
      for (auto& kk : X.snk) ru.insert(kk.first);
      for (auto& kk : X.src) cu.insert(kk.first);
      alg += 8.0 * double(X.n_snk) * X.n_src + 8.0 * double(ru.size()) * cu.size();
      // factored weights, per run (distinct u-tuple): L[c_d] = sum_b u[b] Dd,
      // H[c_d] = sum_s v[s] Du, and sum_c_d L H (forward); the u-leaf adjoints
      // take one product per entry and one per (run, source key), the d-leaf
      // adjoints H per run and u[b] H per (key, d column) (dS)
      const double nru = double(ru.size()), ncd = double(X.ncol(1, X.nf[1]));
      fact_alg += minors + 8.0 * (double(X.n_snk) * ncd + nru * X.n_src + nru * ncd);
      fact_ds_alg += minors + rev + 8.0 * (double(X.n_snk) * X.n_src + 2.0 * nru * X.n_src + double(X.n_snk) * ncd);
    }

    auto ft = make_tiles(X, budget, kMaxB, fwd_model);
    P.lds_bytes = std::max(P.lds_bytes, emit_tiles(X, ft, fwd_model, fo));
    cr[4] = P.n_tiles;
    auto bt = make_tiles(X, bbudget, kMaxB, bwd_model);
    P.b_lds_ds = std::max(P.b_lds_ds, emit_tiles(X, bt, bwd_model, bo));
    cr[7] = P.b_n_tiles;
    auto wt = make_tiles(X, budget, dw_keys, dw_model);
    P.b_lds_dw = std::max(P.b_lds_dw, emit_tiles(X, wt, dw_model, wo));
    {
      // the factored tiles serve the factored dS where ds_factored admits it,
      // else only the factored forward, and are then sized for its LDS
      // (D_I F32C: 139 tiles of at most 25 KB, five workgroups per CU)
      const bool for_ds = ds_factored(s.n_u, s.n_d, precision);
      const LdsModel ffwd_model{false, csz, true, true};
      auto ftl = for_ds ? make_tiles(X, bbudget, kMaxB, bwdf_model) : make_tiles(X, budget, kMaxB, ffwd_model);
      P.f_lds_ds = std::max(P.f_lds_ds, emit_tiles(X, ftl, bwdf_model, fo2));
    }
    cr[34] = P.f_n_tiles;
  }
  if (w_pos != P.nnz) throw std::logic_error("plan does not cover the index set");
  for (int c = 0; c < s.n_corr; ++c) {
    const int32_t* cr = &P.corr[size_t(c) * kCorrInts];
    P.max_csr = std::max({P.max_csr, int(cr[80]), int(cr[81])});
    for (int f = 0; f < 2; ++f)
      for (int k = 1; k <= 6; ++k) P.max_bin[k] = std::max(P.max_bin[k], int(cr[82 + 6 * f + k - 1]));
  }
  // the factored forward on the f_* tiles: S, the source factors (and a zero
  // behind them), the tile's sink factors, rows, op records and key records;
  // one top d column per thread, lists within the kernels' limit
  int max_ncd = 0;
  for (int c = 0; c < s.n_corr; ++c) {
    const int32_t* cr = &P.corr[size_t(c) * kCorrInts];
    max_ncd = std::max(max_ncd, int(cr[8 + 2 * (6 + s.n_d - 1)]));
    for (int t = cr[33]; t < cr[34]; ++t) {
      const int32_t* tr = &P.f_tiles[size_t(t) * kTileInts];
      const int64_t bytes = (576 + int64_t(cr[0]) + 1 + tr[1] + tr[6]) * csz;
      P.f_lds_fwd = std::max(P.f_lds_fwd, ((bytes + 15) & ~int64_t(15)) + int64_t(tr[4]) * 16 + int64_t(tr[1]) * 16);
    }
  }
  int max_dlist = 0;
  for (int c = 0; c < s.n_corr; ++c) max_dlist = std::max(max_dlist, int(P.corr[size_t(c) * kCorrInts + 81]));
  P.fwd_fact = P.rank1 && P.f_n_tiles > 0 && max_ncd <= P.threads && max_dlist <= top_list_max(s.n_u, s.n_d) &&
               P.max_src < 2048 && P.f_lds_fwd <= 160 * 1024;
  P.fact_alg_flops_per_site = fact_alg;
  P.fact_ds_alg_flops_per_site = fact_ds_alg;
  P.alg_flops_per_site = alg;
  P.exec_flops_per_site = exec;
  P.ds_alg_flops_per_site = ds_alg;
  P.dw_alg_flops_per_site = dw_alg;
}

}  // namespace mbc
