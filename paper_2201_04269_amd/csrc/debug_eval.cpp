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
  // the exact weights go through the factored forward, as mbc_contract does:
  // per run of the factored tiles, sum over top d columns c of
  // (sum_b u[b] Dd_b[c]) (sum over the source keys of column c of v[s] Du[c_u(s)])
  const bool fact = (W == nullptr) && h.fwd_fact;
  for (int tile = 0; fact && tile < h.f_n_tiles; ++tile) {
    const int32_t* tr = &h.f_tiles[size_t(tile) * kTileInts];
    const int corr = tr[0], B = tr[1], op0 = tr[3], meta0 = tr[5], units = tr[6], nreal = tr[17];
    const int32_t* cr = &h.corr[size_t(corr) * kCorrInts];
    const int src_off = cr[1];
    const int ncd = cr[8 + 2 * (6 + h.n_d - 1)];
    const int32_t* csrd = &h.btab[size_t(cr[65])];
    auto cx = [](const std::vector<double>& v, size_t i) { return cd(v[2 * i], v[2 * i + 1]); };
    R.assign(size_t(units), cd(0, 0));
    for (int t = 0; t < T; ++t)
      for (int64_t v = 0; v < V; ++v) {
        const int64_t site = int64_t(t) * V + v;
        for (int i = 0; i < 144; ++i) {
          S[i] = cd(S_u[2 * (site * 144 + i)], S_u[2 * (site * 144 + i) + 1]);
          S[144 + i] = cd(S_d[2 * (site * 144 + i)], S_d[2 * (site * 144 + i) + 1]);
        }
        for (int o = 0; o < nreal; ++o) {  // rows (backward op records, level order)
          const int32_t* p = &h.f_ops[size_t(op0 + o) * kOpInts];
          const int f = p[0], k = p[1], r0 = p[2], in = p[3], outs = p[4];
          const int nc = cr[8 + 2 * (6 * f + k - 1)], toff = cr[8 + 2 * (6 * f + k - 1) + 1];
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
        for (int c = 0; c < ncd; ++c) {
          cd L(0, 0);
          for (int b = 0; b < B; ++b) {
            const int32_t* mb = &h.f_meta[size_t(meta0 + b) * kMetaInts];
            L += cx(h.wu, size_t(cr[32] + tr[16] + b)) * R[mb[1] + c];
            if (mb[2] & 1) {
              cd H(0, 0);
              for (int q = csrd[c]; q < csrd[c + 1]; ++q) {
                const int sidx = csrd[q];
                H += cx(h.wv, size_t(src_off + sidx)) * R[mb[0] + h.src_cu[src_off + sidx]];
              }
              acc += L * H;
              L = cd(0, 0);
            }
          }
        }
        out[size_t(corr) * T + t] += acc;
      }
  }
  for (int tile = 0; !fact && tile < h.n_tiles; ++tile) {
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
    stats->b_n_tiles = h.b_n_tiles;
    stats->b_lds_bytes_ds = h.b_lds_ds;
    stats->b_lds_bytes_dw = h.b_lds_dw;
    stats->w_n_tiles = h.w_n_tiles;
    stats->ds_alg_flops_per_site = h.ds_alg_flops_per_site;
    stats->dw_alg_flops_per_site = h.dw_alg_flops_per_site;
    stats->rank1 = h.rank1 ? 1 : 0;
    stats->f_n_tiles = h.f_n_tiles;
    stats->f_lds_bytes_ds = h.f_lds_ds;
    stats->fwd_factored = h.fwd_fact ? 1 : 0;
    stats->ds_factored = (h.rank1 && ds_factored(h.n_u, h.n_d, h.precision)) ? 1 : 0;
    stats->f_lds_bytes_fwd = h.f_lds_fwd;
    stats->fact_alg_flops_per_site = h.fact_alg_flops_per_site;
    stats->fact_ds_alg_flops_per_site = h.fact_ds_alg_flops_per_site;
  }
  return MBC_OK;
}

// Backward walk: gradients in PyTorch's convention (see mbc_contract_backward),
// through the backward tiling exactly as the dS and dW kernels traverse it.
mbc_status debug_backward(const mbc_index_set* s, int precision, const double* S_u, const double* S_d, int T,
                          int64_t V, const double* W, const double* grad_C, double* grad_W, double* grad_Su,
                          double* grad_Sd) {
  using cd = std::complex<double>;
  PlanHost h;
  compile_plan(s->s, precision, &h);
  std::vector<cd> Wp(size_t(h.nnz));
  for (int64_t i = 0; i < h.nnz; ++i)
    Wp[i] = W ? cd(W[2 * h.perm[i]], W[2 * h.perm[i] + 1]) : cd(h.w_exact[2 * i], h.w_exact[2 * i + 1]);
  std::vector<cd> gW(size_t(h.nnz), cd(0, 0));
  const int nS = 2 * 144;
  std::vector<cd> S(nS), R, A, part, adj1, Sbar(size_t(T) * V * nS, cd(0, 0));
  // the exact weights go through the factored dS tiling, as mbc_contract_backward does
  const bool fact = (W == nullptr) && h.rank1 && ds_factored(h.n_u, h.n_d, h.precision);
  const std::vector<int32_t>& btiles = fact ? h.f_tiles : h.b_tiles;
  const std::vector<int32_t>& bops = fact ? h.f_ops : h.b_ops;
  const std::vector<int32_t>& bmeta = fact ? h.f_meta : h.b_meta;
  const std::vector<int32_t>& bextra = fact ? h.f_extra : h.b_extra;
  const int bn_tiles = fact ? h.f_n_tiles : h.b_n_tiles;
  for (int tile = 0; tile < bn_tiles; ++tile) {
    const int32_t* tr = &btiles[size_t(tile) * kTileInts];
    const int corr = tr[0], B = tr[1], w_off = tr[2], op0 = tr[3], meta0 = tr[5], units = tr[6];
    const int nreal = tr[17], nvirt = tr[18];
    const int32_t* cr = &h.corr[size_t(corr) * kCorrInts];
    const int n_src = cr[0], src_off = cr[1];
    const int nf[2] = {h.n_u, h.n_d};
    const int32_t* ex = &bextra[size_t(tr[19])];
    const int n_runs = ex[0], n_dg = ex[1];
    const int32_t* runs = ex + 3;
    const int32_t* dgs = runs + 3 * n_runs;
    const int32_t* child = dgs + 2 * n_dg;
    auto op = [&](int o) { return &bops[size_t(op0 + o) * kOpInts]; };
    auto metab = [&](int b) { return &bmeta[size_t(meta0 + b) * kMetaInts]; };
    // W[b, s] of the tile's key b: the weight, or the product of its factors
    auto weight = [&](int b, int sidx) {
      if (!fact) return Wp[size_t(w_off) + size_t(b) * n_src + sidx];
      const size_t iu = size_t(cr[32] + tr[16] + b), iv = size_t(src_off + sidx);
      return cd(h.wu[2 * iu], h.wu[2 * iu + 1]) * cd(h.wv[2 * iv], h.wv[2 * iv + 1]);
    };
    R.assign(size_t(units), cd(0, 0));
    A.assign(size_t(units), cd(0, 0));
    for (int t = 0; t < T; ++t) {
      const cd gbar = std::conj(cd(grad_C[2 * (size_t(corr) * T + t)], grad_C[2 * (size_t(corr) * T + t) + 1]));
      for (int64_t v = 0; v < V; ++v) {
        const int64_t site = int64_t(t) * V + v;
        for (int i = 0; i < 144; ++i) {
          S[i] = cd(S_u[2 * (site * 144 + i)], S_u[2 * (site * 144 + i) + 1]);
          S[144 + i] = cd(S_d[2 * (site * 144 + i)], S_d[2 * (site * 144 + i) + 1]);
        }
        // forward rows (real ops, level order)
        for (int o = 0; o < nreal; ++o) {
          const int32_t* p = op(o);
          const int f = p[0], k = p[1], r0 = p[2], in = p[3], outs = p[4];
          const int nc = cr[8 + 2 * (6 * f + k - 1)], toff = cr[8 + 2 * (6 * f + k - 1) + 1];
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
        // leaf adjoints of the top rows (holomorphic, seeded with conj(grad_C))
        const int ncu = cr[8 + 2 * (6 * 0 + nf[0] - 1)], ncd = cr[8 + 2 * (6 * 1 + nf[1] - 1)];
        const int32_t* csru = &h.btab[size_t(cr[64])];
        const int32_t* csrd = &h.btab[size_t(cr[65])];
        for (int r = 0; r < n_runs; ++r) {
          const int us = runs[3 * r], b0 = runs[3 * r + 1], b1 = runs[3 * r + 2];
          for (int c = 0; c < ncu; ++c) {
            cd sum(0, 0);
            for (int q = csru[c]; q < csru[c + 1]; ++q) {
              const int sidx = csru[q];
              for (int b = b0; b < b1; ++b)
                sum += weight(b, sidx) * R[metab(b)[1] + h.src_cd[src_off + sidx]];
            }
            A[us + c] = gbar * sum;
          }
        }
        for (int g = 0; g < n_dg; ++g) {
          const int ds = dgs[2 * g], mask = dgs[2 * g + 1];
          for (int c = 0; c < ncd; ++c) {
            cd sum(0, 0);
            for (int q = csrd[c]; q < csrd[c + 1]; ++q) {
              const int sidx = csrd[q];
              for (int b = 0; b < B; ++b)
                if (mask & (1 << b))
                  sum += weight(b, sidx) * R[metab(b)[0] + h.src_cu[src_off + sidx]];
            }
            A[ds + c] = gbar * sum;
          }
        }
        // reverse sweep, top level down
        part.assign(size_t(nreal) * 12, cd(0, 0));
        adj1.assign(size_t(nvirt) * 12, cd(0, 0));
        const int kmax = std::max(nf[0], nf[1]);
        for (int k = kmax; k >= 1; --k) {
          for (int o = 0; o < nreal; ++o) {  // (ii) S-bar parts of the level-k rows
            const int32_t* p = op(o);
            if (p[1] != k) continue;
            const int f = p[0];
            const int32_t* jl = &h.btab[size_t(cr[40 + 6 * f + k - 1])];
            const cd* Sf = &S[144 * f];
            for (int j = 0; j < 12; ++j) {
              cd sum(0, 0);
              for (int q = jl[j]; q < jl[j + 1]; ++q) {
                const int e = jl[q], C = e & 4095;
                if (k == 1) {
                  sum += A[p[4] + C];
                } else {
                  const int sub = (e >> 12) & 4095, pos = e >> 24;
                  const cd y = (k == 2) ? Sf[12 * p[3] + sub] : R[p[3] + sub];
                  sum += (pos & 1) ? -A[p[4] + C] * y : A[p[4] + C] * y;
                }
              }
              part[size_t(o) * 12 + j] = sum;
            }
          }
          if (k == 1) continue;
          // (i) adjoints of the parents (level k-1 rows, or S rows for k = 2)
          for (int o = 0; o < nreal + nvirt; ++o) {
            const int32_t* p = op(o);
            const bool virt = p[7] != 0;
            if (virt ? (k != 2) : (p[1] != k - 1)) continue;
            if (p[6] == 0) continue;  // a top row: its adjoint came from the leaves
            const int f = p[0];
            const int ncp = cr[8 + 2 * (6 * f + k - 2)];
            const int32_t* ut = &h.btab[size_t(cr[67 + 6 * f + k - 2])];
            const int toff1 = cr[8 + 2 * (6 * f + 0) + 1];
            const cd* Sf = &S[144 * f];
            for (int c = 0; c < ncp; ++c) {
              cd sum(0, 0);
              for (int ci = 0; ci < p[6]; ++ci) {
                const int ce = child[p[5] + ci];  // child row: slot << 4 | r0
                const int ch_slot = ce >> 4, ch_r0 = ce & 15;
                for (int j = 0; j < 12; ++j) {
                  const int ent = (ut[6 * c + j / 2] >> (16 * (j % 2))) & 0xffff;
                  if (ent == 0xffff) continue;
                  const cd term = A[ch_slot + (ent & 4095)] * Sf[12 * ch_r0 + j];
                  sum += ((ent >> 12) & 1) ? -term : term;
                }
              }
              if (virt)
                adj1[size_t(p[4]) + h.tabs[toff1 + c]] = sum;
              else
                A[p[4] + c] = sum;
            }
          }
        }
        cd* sb = &Sbar[size_t(site) * nS];
        for (int f = 0; f < 2; ++f)
          for (int a = 0; a < 12; ++a)
            for (int bb = 0; bb < 12; ++bb) {
              cd sum(0, 0);
              for (int o = 0; o < nreal + nvirt; ++o) {
                const int32_t* p = op(o);
                if (p[0] != f || p[2] != a) continue;
                sum += p[7] ? adj1[size_t(p[4]) + bb] : part[size_t(o) * 12 + bb];
              }
              sb[144 * f + 12 * a + bb] += sum;
            }
      }
    }
  }
  // dW through its own tiling: per-entry products summed over each timeslice
  for (int tile = 0; tile < h.w_n_tiles; ++tile) {
    const int32_t* tr = &h.w_tiles[size_t(tile) * kTileInts];
    const int corr = tr[0], B = tr[1], w_off = tr[2], op0 = tr[3], nops = tr[4], meta0 = tr[5], units = tr[6];
    const int32_t* cr = &h.corr[size_t(corr) * kCorrInts];
    const int n_src = cr[0], src_off = cr[1];
    R.assign(size_t(units), cd(0, 0));
    for (int t = 0; t < T; ++t) {
      std::vector<cd> Q(size_t(B) * n_src, cd(0, 0));
      for (int64_t v = 0; v < V; ++v) {
        const int64_t site = int64_t(t) * V + v;
        for (int i = 0; i < 144; ++i) {
          S[i] = cd(S_u[2 * (site * 144 + i)], S_u[2 * (site * 144 + i) + 1]);
          S[144 + i] = cd(S_d[2 * (site * 144 + i)], S_d[2 * (site * 144 + i) + 1]);
        }
        for (int o = 0; o < nops; ++o) {
          const int32_t* p = &h.w_ops[size_t(op0 + o) * kOpInts];
          const int f = p[0], k = p[1], r0 = p[2], in = p[3], outs = p[4];
          const int nc = cr[8 + 2 * (6 * f + k - 1)], toff = cr[8 + 2 * (6 * f + k - 1) + 1];
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
        for (int b = 0; b < B; ++b) {
          const int32_t* mb = &h.w_meta[size_t(meta0 + b) * kMetaInts];
          for (int sidx = 0; sidx < n_src; ++sidx)
            Q[size_t(b) * n_src + sidx] += R[mb[0] + h.src_cu[src_off + sidx]] * R[mb[1] + h.src_cd[src_off + sidx]];
        }
      }
      const cd g(grad_C[2 * (size_t(corr) * T + t)], grad_C[2 * (size_t(corr) * T + t) + 1]);
      for (int b = 0; b < B; ++b)
        for (int sidx = 0; sidx < n_src; ++sidx)
          gW[size_t(w_off) + size_t(b) * n_src + sidx] += g * std::conj(Q[size_t(b) * n_src + sidx]);
    }
  }
  if (grad_W)
    for (int64_t i = 0; i < h.nnz; ++i) {
      grad_W[2 * h.perm[i]] = gW[i].real();
      grad_W[2 * h.perm[i] + 1] = gW[i].imag();
    }
  for (int64_t site = 0; site < int64_t(T) * V; ++site)
    for (int i = 0; i < 144; ++i) {
      const cd u = std::conj(Sbar[size_t(site) * nS + i]), d = std::conj(Sbar[size_t(site) * nS + 144 + i]);
      if (grad_Su) {
        grad_Su[2 * (site * 144 + i)] = u.real();
        grad_Su[2 * (site * 144 + i) + 1] = u.imag();
      }
      if (grad_Sd) {
        grad_Sd[2 * (site * 144 + i)] = d.real();
        grad_Sd[2 * (site * 144 + i) + 1] = d.imag();
      }
    }
  return MBC_OK;
}
}  // namespace mbc
