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

Levels column_levels(const std::vector<Key>& top, int n) {
  Levels L;
  L.n = n;
  L.cols.resize(n + 1);
  L.index.resize(n + 1);
  for (int k = 1; k <= n; ++k) {
    std::set<Key> s;
    for (const Key& c : top) k_subsets(c, k, &s);
    L.cols[k].assign(s.begin(), s.end());
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
  P.threads = 256;
  const int csz = precision == MBC_F64 ? 16 : 8;
  // local-memory budget per workgroup for the S, W and row areas
  const int64_t budget = precision == MBC_F64 ? 76 * 1024 : 52 * 1024;
  const int kMaxB = 16;
  P.corr.assign(size_t(s.n_corr) * kCorrInts, 0);
  P.w_exact.assign(size_t(2 * P.nnz), 0.0);
  P.perm.assign(size_t(P.nnz), 0);
  int64_t w_pos = 0;
  double alg = 0, exec = 0;
  const int nf[2] = {s.n_u, s.n_d};

  for (int c = 0; c < s.n_corr; ++c) {
    int32_t* cr = &P.corr[size_t(c) * kCorrInts];
    const int64_t e0 = s.corr_begin[c], e1 = s.corr_begin[c + 1];
    cr[3] = P.n_tiles;
    cr[5] = int32_t(e0);
    if (e0 == e1) {  // empty correlator: C = 0, no tiles
      cr[4] = P.n_tiles;
      cr[1] = int32_t(P.src_cu.size());
      continue;
    }
    // sink and source keys
    std::map<std::pair<Key, Key>, int> snk_id, src_id;
    for (int64_t e = e0; e < e1; ++e) {
      snk_id.emplace(std::make_pair(s.entries[e].ru, s.entries[e].rd), 0);
      src_id.emplace(std::make_pair(s.entries[e].cu, s.entries[e].cd), 0);
    }
    const int n_snk = int(snk_id.size()), n_src = int(src_id.size());
    if (int64_t(n_snk) * n_src != e1 - e0)
      throw std::domain_error("index set of a correlator is not a Cartesian product of sink and source keys");
    std::vector<std::pair<Key, Key>> snk, src;
    for (auto& kv : snk_id) snk.push_back(kv.first);
    for (auto& kv : src_id) src.push_back(kv.first);
    // plan order of sink keys: by reversed u-tuple, then d-tuple
    std::sort(snk.begin(), snk.end(), [](const std::pair<Key, Key>& a, const std::pair<Key, Key>& b) {
      if (!(a.first == b.first)) return rev_less(a.first, b.first);
      return a.second < b.second;
    });
    for (int i = 0; i < n_snk; ++i) snk_id[snk[i]] = i;
    for (int i = 0; i < n_src; ++i) src_id[src[i]] = i;
    // entry of (sink i, source j)
    std::vector<int64_t> ent(size_t(n_snk) * n_src, -1);
    for (int64_t e = e0; e < e1; ++e) {
      const int i = snk_id[{s.entries[e].ru, s.entries[e].rd}];
      const int j = src_id[{s.entries[e].cu, s.entries[e].cd}];
      int64_t& slot = ent[size_t(i) * n_src + j];
      if (slot >= 0) throw std::domain_error("duplicate index-set entry");
      slot = e;
    }
    // column levels per flavour: all k-subsets of the source tuples
    std::vector<Key> top_cols[2];
    for (auto& k : src) {
      top_cols[0].push_back(k.first);
      top_cols[1].push_back(k.second);
    }
    Levels lev[2] = {column_levels(top_cols[0], nf[0]), column_levels(top_cols[1], nf[1])};
    int tab_off_fk[2][kMaxQuarks + 1] = {};
    for (int f = 0; f < 2; ++f)
      for (int k = 1; k <= nf[f]; ++k) {
        const auto& cols = lev[f].cols[k];
        tab_off_fk[f][k] = int(P.tabs.size());
        cr[8 + 2 * (6 * f + k - 1)] = int32_t(cols.size());
        cr[8 + 2 * (6 * f + k - 1) + 1] = int32_t(P.tabs.size());
        for (const Key& C : cols) {
          if (k == 1) {
            P.tabs.push_back(uint16_t(C.v[0]));
            continue;
          }
          for (int j = 0; j < k; ++j) {
            const Key rest = drop(C, j);
            const int sub = (k == 2) ? rest.v[0] : lev[f].index[k - 1].at(rest);
            if (sub >= 4096) throw std::runtime_error("column list too long");
            P.tabs.push_back(uint16_t((sub << 4) | C.v[j]));
          }
        }
      }
    auto ncol = [&](int f, int k) { return int(lev[f].cols[k].size()); };
    // source keys -> top-level column indices
    cr[0] = n_src;
    cr[1] = int32_t(P.src_cu.size());
    cr[2] = n_snk;
    for (auto& k : src) {
      P.src_cu.push_back(lev[0].index[nf[0]].at(k.first));
      P.src_cd.push_back(lev[1].index[nf[1]].at(k.second));
    }
    P.maxs = std::max(P.maxs, (n_src + P.threads - 1) / P.threads);
    for (int f = 0; f < 2; ++f)
      for (int k = 1; k <= nf[f]; ++k) P.qmax = std::max(P.qmax, (ncol(f, k) + P.threads - 1) / P.threads);

    // algorithmic flops (global minor DAG + leaves + (r_u, c_u) groups)
    {
      for (int f = 0; f < 2; ++f)
        for (int k = 2; k <= nf[f]; ++k) {
          std::set<Key> suf;
          for (auto& kk : snk) suf.insert(tail(f == 0 ? kk.first : kk.second, k));
          alg += double(suf.size()) * ncol(f, k) * (8.0 * k - 2.0);
        }
      std::set<Key> ru, cu;
      for (auto& kk : snk) ru.insert(kk.first);
      for (auto& kk : src) cu.insert(kk.first);
      alg += 8.0 * double(n_snk) * n_src + 8.0 * double(ru.size()) * cu.size();
    }

    // runs of equal u-tuples
    std::vector<std::pair<int, int>> runs;  // [begin, end)
    for (int i = 0; i < n_snk;) {
      int j = i + 1;
      while (j < n_snk && snk[j].first == snk[i].first) ++j;
      runs.push_back({i, j});
      i = j;
    }
    auto tile_lds = [&](const std::vector<int>& sk) {
      std::set<RowId> rows;
      for (int i : sk) {
        add_chain(0, snk[i].first, &rows);
        add_chain(1, snk[i].second, &rows);
      }
      int64_t units = 576 + int64_t(sk.size()) * n_src;
      for (auto& r : rows) units += ncol(r.f, r.k);
      return units * csz + int64_t(rows.size()) * 16;
    };
    // greedy tiling over whole runs (a run longer than a tile is split)
    std::vector<std::vector<int>> tiles;
    std::vector<int> cur;
    for (auto& rn : runs) {
      std::vector<int> run;
      for (int i = rn.first; i < rn.second; ++i) run.push_back(i);
      std::vector<int> trial = cur;
      trial.insert(trial.end(), run.begin(), run.end());
      if (!cur.empty() && (int(trial.size()) > kMaxB || tile_lds(trial) > budget)) {
        tiles.push_back(cur);
        cur.clear();
      }
      for (int i : run) {
        std::vector<int> t2 = cur;
        t2.push_back(i);
        if (!cur.empty() && (int(t2.size()) > kMaxB || tile_lds(t2) > budget)) {
          tiles.push_back(cur);
          cur.clear();
        }
        cur.push_back(i);
      }
    }
    if (!cur.empty()) tiles.push_back(cur);

    for (auto& sk : tiles) {
      const int B = int(sk.size());
      std::set<RowId> rowset;
      for (int i : sk) {
        add_chain(0, snk[i].first, &rowset);
        add_chain(1, snk[i].second, &rowset);
      }
      // slots in (level, flavour, tuple) order; phases = levels
      std::map<RowId, int> slot;
      int units = 0;
      for (auto& r : rowset) {
        slot[r] = units;
        units += ncol(r.f, r.k);
      }
      // double-buffered S, the tile's weights, row slots, staged (r0, in, out) ops
      const int64_t lds = int64_t(576 + int64_t(B) * n_src + units) * csz + int64_t(rowset.size()) * 16;
      if (lds > 160 * 1024) throw std::runtime_error("a tile exceeds the 160 KiB local memory of a CU");
      P.lds_bytes = std::max(P.lds_bytes, lds);
      std::vector<int32_t> tr(kTileInts, 0);
      tr[0] = c;
      tr[1] = B;
      tr[2] = int32_t(w_pos);
      tr[3] = int32_t(P.ops.size() / kOpInts);
      tr[5] = int32_t(P.meta.size() / kMetaInts);
      tr[6] = units;
      tr[16] = sk[0];
      int n_ops = 0, phase = -1, cur_level = 0, item = 0;
      for (auto& r : rowset) {
        if (r.k != cur_level) {
          ++phase;
          if (phase >= kMaxPhases) throw std::runtime_error("too many phases");
          tr[8 + phase] = n_ops;
          cur_level = r.k;
          item = 0;
        }
        int in = 0;
        if (r.k == 2) in = r.t.v[1];
        if (r.k >= 3) in = slot.at({r.f, r.k - 1, tail(r.t, r.k - 1)});
        const int nc = ncol(r.f, r.k);
        if (tr[21 + 2 * (7 * r.f + r.k)] == 0) tr[20 + 2 * (7 * r.f + r.k)] = n_ops;
        ++tr[21 + 2 * (7 * r.f + r.k)];
        const int32_t op[kOpInts] = {r.f, r.k, r.t.v[0], in, slot.at(r), tab_off_fk[r.f][r.k], nc, item};
        P.ops.insert(P.ops.end(), op, op + kOpInts);
        item += nc;
        ++n_ops;
        if (r.k >= 2) exec += double(nc) * (8.0 * r.k - 2.0);
      }
      tr[4] = n_ops;
      tr[7] = phase + 1;
      tr[8 + phase + 1] = n_ops;
      P.max_ops = std::max(P.max_ops, n_ops);
      // per sink key metadata and the tile's weights (b-major)
      int pieces = 0;
      for (int b = 0; b < B; ++b) {
        const int i = sk[b];
        const bool run_end = (b + 1 == B) || !(snk[sk[b + 1]].first == snk[i].first);
        pieces += run_end;
        const int u_slot = slot.at({0, nf[0], snk[i].first});
        const int d_slot = slot.at({1, nf[1], snk[i].second});
        const int32_t m[kMetaInts] = {u_slot, d_slot, run_end ? 1 : 0, i};
        P.meta.insert(P.meta.end(), m, m + kMetaInts);
        for (int j = 0; j < n_src; ++j) {
          const int64_t e = ent[size_t(i) * n_src + j];
          P.perm[size_t(w_pos)] = e;
          const double den = double(s.w_den[c]);
          P.w_exact[size_t(2 * w_pos)] = double(s.entries[e].w_re) / den;
          P.w_exact[size_t(2 * w_pos + 1)] = double(s.entries[e].w_im) / den;
          ++w_pos;
        }
      }
      exec += 8.0 * double(B) * n_src + 8.0 * double(pieces) * n_src;
      P.max_b = std::max(P.max_b, B);
      P.tiles.insert(P.tiles.end(), tr.begin(), tr.end());
      ++P.n_tiles;
    }
    cr[4] = P.n_tiles;
  }
  if (w_pos != P.nnz) throw std::logic_error("plan does not cover the index set");
  P.alg_flops_per_site = alg;
  P.exec_flops_per_site = exec;
}

}  // namespace mbc
