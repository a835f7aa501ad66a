// Host walk of a compiled plan (checking aid for the plan compiler; see
// include/mbc_debug.h).  Mirrors the device kernel's loops in FP64.
#include <complex>
#include <stdexcept>
#include <vector>

#include "../../include/mbc_debug.h"
#include "mbc_internal.hpp"

namespace mbc {
mbc_status debug_eval(const mbc_index_set* s, int precision, const double* S_u, const double* S_d, int T,
                      int64_t V, const double* W, double* C, mbc_plan_stats* stats) {
  using cd = std::complex<double>;
  PlanHost h;
  compile_plan(s->s, precision, &h);
  std::vector<cd> Wp(size_t(h.nnz));
  for (int64_t i = 0; i < h.nnz; ++i) {
    if (W)
      Wp[i] = cd(W[2 * h.perm[i]], W[2 * h.perm[i] + 1]);
    else
      Wp[i] = cd(h.w_exact[2 * i], h.w_exact[2 * i + 1]);
  }
  std::vector<cd> out(size_t(h.n_corr) * T, cd(0, 0));
  std::vector<cd> S(288), R;
  for (int tile = 0; tile < h.n_tiles; ++tile) {
    const int32_t* tr = &h.tiles[size_t(tile) * kTileInts];
    const int corr = tr[0], B = tr[1], w_off = tr[2], op0 = tr[3], meta0 = tr[5], units = tr[6], nph = tr[7];
    const int32_t* cr = &h.corr[size_t(corr) * kCorrInts];
    const int n_src = cr[0], src_off = cr[1];
    R.assign(size_t(units), cd(0, 0));
    for (int t = 0; t < T; ++t)
      for (int64_t v = 0; v < V; ++v) {
        const int64_t site = int64_t(t) * V + v;
        for (int i = 0; i < 144; ++i) {
          S[i] = cd(S_u[2 * (site * 144 + i)], S_u[2 * (site * 144 + i) + 1]);
          S[144 + i] = cd(S_d[2 * (site * 144 + i)], S_d[2 * (site * 144 + i) + 1]);
        }
        for (int ph = 0; ph < nph; ++ph)
          for (int o = tr[8 + ph]; o < tr[9 + ph]; ++o) {
            const int32_t* op = &h.ops[size_t(op0 + o) * kOpInts];
            const int f = op[0], k = op[1], r0 = op[2], in = op[3], outs = op[4], toff = op[5], nc = op[6];
            const cd* Sf = &S[144 * f];
            for (int i = 0; i < nc; ++i) {
              cd val(0, 0);
              if (k == 1) {
                val = Sf[12 * r0 + h.tabs[toff + i]];
              } else {
                for (int j = 0; j < k; ++j) {
                  const int e = h.tabs[toff + i * k + j];
                  const cd x = Sf[12 * r0 + (e & 15)];
                  const cd y = (k == 2) ? Sf[12 * in + (e >> 4)] : R[in + (e >> 4)];
                  val += (j & 1) ? -x * y : x * y;
                }
              }
              R[outs + i] = val;
            }
          }
        cd acc(0, 0);
        for (int sidx = 0; sidx < n_src; ++sidx) {
          const int cu = h.src_cu[src_off + sidx], cdx = h.src_cd[src_off + sidx];
          cd L(0, 0);
          for (int b = 0; b < B; ++b) {
            const int32_t* mb = &h.meta[size_t(meta0 + b) * kMetaInts];
            L += Wp[size_t(w_off) + size_t(b) * n_src + sidx] * R[mb[1] + cdx];
            if (mb[2]) {
              acc += R[mb[0] + cu] * L;
              L = cd(0, 0);
            }
          }
        }
        out[size_t(corr) * T + t] += acc;
      }
  }
  for (size_t i = 0; i < out.size(); ++i) {
    C[2 * i] = out[i].real();
    C[2 * i + 1] = out[i].imag();
  }
  if (stats) {
    stats->nnz = h.nnz;
    stats->n_corr = h.n_corr;
    stats->n_u = h.n_u;
    stats->n_d = h.n_d;
    stats->precision = h.precision;
    stats->n_tiles = h.n_tiles;
    stats->threads = h.threads;
    stats->lds_bytes = h.lds_bytes;
    stats->alg_flops_per_site = h.alg_flops_per_site;
    stats->exec_flops_per_site = h.exec_flops_per_site;
    stats->in_bytes_per_site = 2.0 * 144.0 * 16.0;
  }
  return MBC_OK;
}
}  // namespace mbc
