// Operator algebra and canonical index sets (host, exact integer arithmetic).
//
// Builds, for a batch of correlators, the index set I of eq. 1 together with
// its exact weights W: the sink operator of each correlator (a single baryon
// or one of the multi-baryon operators of eq. "ops") is expanded into ordered
// Grassmann products of quark fields, each term is brought to the flavour
// order u..u d..d with its sign, tuples are sorted (times the permutation
// parity), terms with a repeated index are dropped, equal keys are merged and
// zero sums removed (the canonical ordering with multiplicities of Sec. 3,
// applied at the quark level).  The source operator carries the conjugate
// coefficients in the same written order, so W_{r,c} = sigma s^2 w_r conj(w_c)
// on the Cartesian product of sink and source keys.
//
// Conventions: quark index a = 4*colour + spin; Euclidean Dirac basis with
// C = gamma_2 gamma_4; Gamma = C gamma_5 (P_+- = (1 +- gamma_4)/2 for the
// non-relativistic baryons).  sigma = (-1)^(n_u n_d + n_u(n_u-1)/2 + n_d(n_d-1)/2).
#include "mbc_internal.hpp"

#include <algorithm>
#include <array>
#include <map>
#include <stdexcept>

namespace mbc {

namespace {

struct G {  // Gaussian integer
  int64_t re = 0, im = 0;
};
inline G gmul(G a, G b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
inline G gadd(G a, G b) { return {a.re + b.re, a.im + b.im}; }
inline G gneg(G a) { return {-a.re, -a.im}; }
inline G gconj(G a) { return {a.re, -a.im}; }
inline bool gzero(G a) { return a.re == 0 && a.im == 0; }

using M4 = std::array<std::array<G, 4>, 4>;

M4 mmul(const M4& a, const M4& b) {
  M4 c{};
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      G s{};
      for (int k = 0; k < 4; ++k) s = gadd(s, gmul(a[i][k], b[k][j]));
      c[i][j] = s;
    }
  return c;
}

// gamma_k = [[0, -i sigma_k], [i sigma_k, 0]], gamma_4 = diag(1, 1, -1, -1).
M4 dirac_gamma(int mu) {
  M4 g{};
  if (mu == 4) {
    g[0][0] = {1, 0}; g[1][1] = {1, 0}; g[2][2] = {-1, 0}; g[3][3] = {-1, 0};
    return g;
  }
  // Pauli matrices as Gaussian-integer 2x2 blocks
  G s[2][2];
  if (mu == 1) { s[0][0] = {0, 0}; s[0][1] = {1, 0}; s[1][0] = {1, 0}; s[1][1] = {0, 0}; }
  if (mu == 2) { s[0][0] = {0, 0}; s[0][1] = {0, -1}; s[1][0] = {0, 1}; s[1][1] = {0, 0}; }
  if (mu == 3) { s[0][0] = {1, 0}; s[0][1] = {0, 0}; s[1][0] = {0, 0}; s[1][1] = {-1, 0}; }
  const G mi{0, -1}, pi{0, 1};
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      g[a][2 + b] = gmul(mi, s[a][b]);
      g[2 + a][b] = gmul(pi, s[a][b]);
    }
  return g;
}

// C gamma_5 (proj 0) or C gamma_5 P_+- (proj +-1).
M4 cg5(int proj) {
  M4 C = mmul(dirac_gamma(2), dirac_gamma(4));
  M4 g5 = mmul(mmul(dirac_gamma(1), dirac_gamma(2)), mmul(dirac_gamma(3), dirac_gamma(4)));
  M4 m = mmul(C, g5);
  if (proj != 0) {
    M4 g4 = dirac_gamma(4), p{};
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) {
        int64_t v = (i == j ? 1 : 0) + proj * g4[i][j].re;  // gamma_4 is real diagonal
        if (v % 2 != 0 || g4[i][j].im != 0) throw std::logic_error("non-integral projector");
        p[i][j] = {v / 2, 0};
      }
    m = mmul(m, p);
  }
  return m;
}

constexpr int kMaxFields = 12;
enum : uint8_t { kU = 0, kD = 1 };

struct Term {
  G coef;
  int n = 0;
  uint8_t flav[kMaxFields];
  uint8_t idx[kMaxFields];
};

int parity(const uint8_t* v, int n) {
  int inv = 0;
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) inv += v[i] > v[j];
  return (inv & 1) ? -1 : 1;
}

// Single baryon at open spin `spin`: eps_abc Gamma_{beta gamma} q1(4a+beta) q2(4b+gamma) q1(4c+spin),
// (q1, q2) = (u, d) for the proton family and (d, u) for the neutron family.
std::vector<Term> baryon(bool proton, int proj, int spin) {
  const M4 gm = cg5(proj);
  const uint8_t f1 = proton ? kU : kD, f2 = proton ? kD : kU;
  static const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  std::vector<Term> out;
  for (const auto& p : perms) {
    uint8_t pp[3] = {uint8_t(p[0]), uint8_t(p[1]), uint8_t(p[2])};
    const int eps = parity(pp, 3);
    for (int be = 0; be < 4; ++be)
      for (int ga = 0; ga < 4; ++ga) {
        G g = gm[be][ga];
        if (gzero(g)) continue;
        Term t;
        t.coef = eps > 0 ? g : gneg(g);
        t.n = 3;
        t.flav[0] = f1; t.idx[0] = uint8_t(4 * p[0] + be);
        t.flav[1] = f2; t.idx[1] = uint8_t(4 * p[1] + ga);
        t.flav[2] = f1; t.idx[2] = uint8_t(4 * p[2] + spin);
        out.push_back(t);
      }
  }
  return out;
}

struct BaryonName {
  bool proton;
  int proj;
};
constexpr BaryonName P{true, 0}, N{false, 0}, PP{true, 1}, PM{true, -1}, NP{false, 1};

struct Product {
  int sign;
  int nb;
  BaryonName b[3];
};

Term concat(const Term& a, const Term& b, G extra) {
  Term t;
  t.coef = gmul(extra, gmul(a.coef, b.coef));
  t.n = a.n + b.n;
  for (int i = 0; i < a.n; ++i) { t.flav[i] = a.flav[i]; t.idx[i] = a.idx[i]; }
  for (int i = 0; i < b.n; ++i) { t.flav[a.n + i] = b.flav[i]; t.idx[a.n + i] = b.idx[i]; }
  return t;
}

// The written products X^T (C gamma5) Y [Z^j] of a multi-baryon operator of
// eq. "ops" with their relative signs, and the s^2 denominator.
std::vector<Product> written_products(int op, int* den) {
  *den = 1;
  switch (op) {
    case MBC_OP_DI: return {{+1, 2, {N, P}}};
    case MBC_OP_DII: *den = 2; return {{+1, 2, {N, P}}, {-1, 2, {P, N}}};
    case MBC_OP_HE3_I: return {{+1, 3, {PM, NP, PP}}};
    case MBC_OP_HE3_II:
      *den = 6;
      return {{+1, 3, {PM, NP, PP}}, {-1, 3, {PP, NP, PM}}, {+1, 3, {NP, PP, PM}},
              {-1, 3, {NP, PM, PP}}, {+1, 3, {PP, PM, NP}}, {-1, 3, {PM, PP, NP}}};
    default: throw std::invalid_argument("unknown operator");
  }
}

// Written terms of an operator (before flavour separation) and s^2 denominator.
std::vector<Term> operator_terms(int op, int spin, int sign_mode, int* den) {
  *den = 1;
  if (op == MBC_OP_PROTON) return baryon(true, 0, spin);
  if (op == MBC_OP_NEUTRON) return baryon(false, 0, spin);
  const std::vector<Product> prods = written_products(op, den);
  const M4 gm = cg5(0);
  std::vector<Term> out;
  for (const Product& pr : prods) {
    const int rel = (sign_mode == MBC_SIGNS_R2) ? 1 : pr.sign;
    std::vector<Term> third;
    if (pr.nb == 3) third = baryon(pr.b[2].proton, pr.b[2].proj, spin);
    for (int al = 0; al < 4; ++al)
      for (int be = 0; be < 4; ++be) {
        G g = gm[al][be];
        if (gzero(g)) continue;
        if (rel < 0) g = gneg(g);
        const auto X = baryon(pr.b[0].proton, pr.b[0].proj, al);
        const auto Y = baryon(pr.b[1].proton, pr.b[1].proj, be);
        for (const Term& x : X)
          for (const Term& y : Y) {
            Term xy = concat(x, y, g);
            if (pr.nb == 2) {
              out.push_back(xy);
            } else {
              for (const Term& z : third) out.push_back(concat(xy, z, G{1, 0}));
            }
          }
      }
  }
  return out;
}

struct SepTerm {
  G coef;
  Key u, d;
};

// Stable partition into u..u d..d with the Grassmann sign (one transposition
// for every d written before a u).
std::vector<SepTerm> separate(const std::vector<Term>& terms, int* nu, int* nd) {
  std::vector<SepTerm> out;
  out.reserve(terms.size());
  for (const Term& t : terms) {
    SepTerm s;
    int swaps = 0, seen_d = 0;
    s.u.n = s.d.n = 0;
    for (int i = 0; i < t.n; ++i) {
      if (t.flav[i] == kD) {
        ++seen_d;
        s.d.v[s.d.n++] = t.idx[i];
      } else {
        swaps += seen_d;
        s.u.v[s.u.n++] = t.idx[i];
      }
    }
    s.coef = (swaps & 1) ? gneg(t.coef) : t.coef;
    *nu = s.u.n;
    *nd = s.d.n;
    out.push_back(s);
  }
  return out;
}

bool has_repeat(const Key& k) {
  for (int i = 0; i < k.n; ++i)
    for (int j = i + 1; j < k.n; ++j)
      if (k.v[i] == k.v[j]) return true;
  return false;
}

// Canonical sink tensor: sorted keys, exact merged coefficients, zeros dropped.
std::vector<std::pair<std::pair<Key, Key>, G>> canonical(const std::vector<SepTerm>& raw) {
  std::map<std::pair<Key, Key>, G> acc;
  for (const SepTerm& s : raw) {
    if (has_repeat(s.u) || has_repeat(s.d)) continue;
    const int par = parity(s.u.v, s.u.n) * parity(s.d.v, s.d.n);
    Key su = s.u, sd = s.d;
    std::sort(su.v, su.v + su.n);
    std::sort(sd.v, sd.v + sd.n);
    G c = par > 0 ? s.coef : gneg(s.coef);
    auto it = acc.find({su, sd});
    if (it == acc.end())
      acc.emplace(std::make_pair(su, sd), c);
    else
      it->second = gadd(it->second, c);
  }
  std::vector<std::pair<std::pair<Key, Key>, G>> out;
  for (auto& kv : acc)
    if (!gzero(kv.second)) out.push_back(kv);
  return out;  // std::map iteration = lexicographic (u, d) order
}

int grassmann_sigma(int nu, int nd) {
  const int e = nu * nd + nu * (nu - 1) / 2 + nd * (nd - 1) / 2;
  return (e & 1) ? -1 : 1;
}

struct KeyList {
  std::vector<Key> u, d;
  std::vector<G> w;
};

KeyList make_keys(int op, int spin, int sign_mode, bool sym, int* nu, int* nd, int* den) {
  auto terms = operator_terms(op, spin, sign_mode, den);
  auto raw = separate(terms, nu, nd);
  KeyList kl;
  if (sym) {
    for (auto& kv : canonical(raw)) {
      kl.u.push_back(kv.first.first);
      kl.d.push_back(kv.first.second);
      kl.w.push_back(kv.second);
    }
  } else {
    for (auto& s : raw) {
      kl.u.push_back(s.u);
      kl.d.push_back(s.d);
      kl.w.push_back(s.coef);
    }
  }
  return kl;
}

BaryonSlot slot_of(BaryonName b, int spin) {
  BaryonSlot x;
  x.family = b.proton ? MBC_FAMILY_P : MBC_FAMILY_N;
  x.proj = b.proj;
  x.spin = spin;
  return x;
}

}  // namespace

std::vector<SinkProduct> sink_products(int op, int spin, int sign_mode, int* den) {
  if (sign_mode != MBC_SIGNS_EXACT && sign_mode != MBC_SIGNS_R2) throw std::invalid_argument("sign_mode");
  if (spin < 0 || spin > 3) throw std::invalid_argument("spin index out of range");
  std::vector<SinkProduct> out;
  *den = 1;
  if (op == MBC_OP_PROTON || op == MBC_OP_NEUTRON) {
    SinkProduct p;
    p.coef = {1, 0};
    p.nb = 1;
    p.b[0] = slot_of(op == MBC_OP_PROTON ? P : N, spin);
    out.push_back(p);
    return out;
  }
  const std::vector<Product> prods = written_products(op, den);
  const M4 gm = cg5(0);
  for (const Product& pr : prods) {
    const int rel = (sign_mode == MBC_SIGNS_R2) ? 1 : pr.sign;
    for (int al = 0; al < 4; ++al)
      for (int be = 0; be < 4; ++be) {
        G g = gm[al][be];
        if (gzero(g)) continue;
        if (rel < 0) g = gneg(g);
        SinkProduct sp;
        sp.coef = {g.re, g.im};
        sp.nb = pr.nb;
        sp.b[0] = slot_of(pr.b[0], al);
        sp.b[1] = slot_of(pr.b[1], be);
        if (pr.nb == 3) sp.b[2] = slot_of(pr.b[2], spin);
        out.push_back(sp);
      }
  }
  return out;
}

std::vector<WrittenProduct> written_baryon_products(int op, int sign_mode, int* den) {
  if (sign_mode != MBC_SIGNS_EXACT && sign_mode != MBC_SIGNS_R2) throw std::invalid_argument("sign_mode");
  *den = 1;
  std::vector<WrittenProduct> out;
  if (op == MBC_OP_PROTON || op == MBC_OP_NEUTRON) {
    WrittenProduct w;
    w.nb = 1;
    w.b[0] = slot_of(op == MBC_OP_PROTON ? P : N, 0);
    out.push_back(w);
    return out;
  }
  for (const Product& pr : written_products(op, den)) {
    WrittenProduct w;
    w.sign = (sign_mode == MBC_SIGNS_R2) ? 1 : pr.sign;
    w.nb = pr.nb;
    for (int i = 0; i < pr.nb; ++i) w.b[i] = slot_of(pr.b[i], 0);
    out.push_back(w);
  }
  return out;
}

std::vector<FieldTerm> source_terms(int op, int spin, int sign_mode, bool canonical_form, const int32_t* pts) {
  if (sign_mode != MBC_SIGNS_EXACT && sign_mode != MBC_SIGNS_R2) throw std::invalid_argument("sign_mode");
  if (spin < 0 || spin > 3) throw std::invalid_argument("spin index out of range");
  int den = 1;
  std::vector<Term> terms = operator_terms(op, spin, sign_mode, &den);
  // field i of slot i / 3 at point pts[i / 3], carried as index 12 * point + a
  // so that sorting orders the fields of one flavour by (point, index)
  for (Term& t : terms)
    for (int i = 0; i < t.n; ++i) {
      const int p = pts ? pts[i / 3] : 0;
      if (p < 0 || p > 2) throw std::invalid_argument("source point out of range (0..2)");
      t.idx[i] = uint8_t(12 * p + t.idx[i]);
    }
  std::vector<FieldTerm> out;
  auto split = [](FieldTerm& f, int i, int v) {
    f.idx[i] = uint8_t(v % 12);
    f.pt[i] = uint8_t(v / 12);
  };
  if (!canonical_form) {
    out.reserve(terms.size());
    for (const Term& t : terms) {
      FieldTerm f;
      f.coef = {t.coef.re, t.coef.im};
      f.n = t.n;
      for (int i = 0; i < t.n; ++i) {
        f.flav[i] = t.flav[i];
        split(f, i, t.idx[i]);
      }
      out.push_back(f);
    }
    return out;
  }
  int nu = 0, nd = 0;
  for (auto& kv : canonical(separate(terms, &nu, &nd))) {
    FieldTerm f;
    f.coef = {kv.second.re, kv.second.im};
    const Key& u = kv.first.first;
    const Key& d = kv.first.second;
    f.n = u.n + d.n;
    for (int i = 0; i < u.n; ++i) {
      f.flav[i] = kFlavU;
      split(f, i, u.v[i]);
    }
    for (int i = 0; i < d.n; ++i) {
      f.flav[u.n + i] = kFlavD;
      split(f, u.n + i, d.v[i]);
    }
    out.push_back(f);
  }
  return out;
}

void gamma_cg5(int proj, int64_t re[16], int64_t im[16]) {
  const M4 m = cg5(proj);
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      re[4 * i + j] = m[i][j].re;
      im[4 * i + j] = m[i][j].im;
    }
}

bool operator<(const Key& a, const Key& b) {
  if (a.n != b.n) return a.n < b.n;
  for (int i = 0; i < a.n; ++i)
    if (a.v[i] != b.v[i]) return a.v[i] < b.v[i];
  return false;
}
bool operator==(const Key& a, const Key& b) {
  if (a.n != b.n) return false;
  for (int i = 0; i < a.n; ++i)
    if (a.v[i] != b.v[i]) return false;
  return true;
}

void build_index_set(const mbc_op_desc* ops, int n_corr, IndexSet* out) {
  out->n_u = out->n_d = -1;
  out->n_corr = n_corr;
  out->w_den.assign(n_corr, 1);
  out->entries.clear();
  out->corr_begin.assign(n_corr + 1, 0);
  for (int c = 0; c < n_corr; ++c) {
    const mbc_op_desc& od = ops[c];
    if (od.sign_mode != MBC_SIGNS_EXACT && od.sign_mode != MBC_SIGNS_R2)
      throw std::invalid_argument("sign_mode");
    if (od.snk_spin < 0 || od.snk_spin > 3 || od.src_spin < 0 || od.src_spin > 3)
      throw std::invalid_argument("spin index out of range");
    int nu = 0, nd = 0, den = 1, nu2 = 0, nd2 = 0, den2 = 1;
    const bool sym = od.symmetrise != 0;
    KeyList snk = make_keys(od.op, od.snk_spin, od.sign_mode, sym, &nu, &nd, &den);
    KeyList src = make_keys(od.op, od.src_spin, od.sign_mode, sym, &nu2, &nd2, &den2);
    if (out->n_u < 0) {
      out->n_u = nu;
      out->n_d = nd;
    } else if (out->n_u != nu || out->n_d != nd) {
      throw std::invalid_argument("correlators of one index set must share (n_u, n_d)");
    }
    out->w_den[c] = den;
    const int sig = grassmann_sigma(nu, nd);
    const size_t base = out->entries.size();
    for (size_t i = 0; i < snk.u.size(); ++i)
      for (size_t j = 0; j < src.u.size(); ++j) {
        Entry e;
        e.ru = snk.u[i]; e.rd = snk.d[i];
        e.cu = src.u[j]; e.cd = src.d[j];
        G w = gmul(snk.w[i], gconj(src.w[j]));
        if (sig < 0) w = gneg(w);
        e.w_re = w.re;
        e.w_im = w.im;
        e.corr = c;
        out->entries.push_back(e);
      }
    if (sym) {
      std::sort(out->entries.begin() + base, out->entries.end(), [](const Entry& a, const Entry& b) {
        if (!(a.ru == b.ru)) return a.ru < b.ru;
        if (!(a.cu == b.cu)) return a.cu < b.cu;
        if (!(a.rd == b.rd)) return a.rd < b.rd;
        return a.cd < b.cd;
      });
    }
    out->corr_begin[c + 1] = static_cast<int64_t>(out->entries.size());
    out->canonical = out->canonical && sym;
  }
  if (n_corr == 0) out->n_u = out->n_d = 0;
}

}  // namespace mbc
