// dS kernel of the adjoint (backward) contraction for gfx950: device code
// and its launch template, shared by the units that instantiate it.
//
// dS kernel (one workgroup = one site, all tiles): per tile, rebuilds the
// rows (minors recomputed, none stored), forms the adjoints of the top rows
// from the factor-tree leaves, then sweeps the Laplace recursion backwards:
//   adjoint of a parent row:  A_{k-1}(r', C') = sum_j (-1)^pos S[r0, j] A_k(r, C' + j)
//   adjoint of S row r0:      Sbar[r0, j]   += sum_{C contains j} (-1)^pos A_k(r, C) M_{k-1}(r', C \ j)
// (Jacobi's formula applied level by level).  The S-bar contributions of
// each row are reduced over 16-lane groups into per-row partials and summed
// by the thread that owns each S-bar entry in a fixed order, so the result
// is deterministic.  Seeded with conj(grad_C), the holomorphic adjoint is
// conjugated on output (PyTorch's convention).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "device_common.hpp"
#include "kernels.hpp"

namespace mbc {

struct BwdArgs {
  const int32_t* corr;
  const int32_t* tiles;
  const int32_t* ops;
  const int32_t* meta;
  const int32_t* extra;
  const int32_t* btab;
  const int32_t* src_cu;
  const int32_t* src_cd;
  const uint16_t* tabs;
  const void* W;
  const void* S_u;
  const void* S_d;
  int s_c64;
  int n_tiles;
  int T;
  int64_t V;
  const double* grad_C;
  void* grad_S_u;
  void* grad_S_d;
  int chunk, nc;
  double* partial;  // dW partials [T * nc][nnz][2] (plan order)
  int64_t nnz;
  const void* wu;   // factored dS: sink and source factors of the exact weights
  const void* wv;
};

namespace {

using namespace dev;

// Rows of one site for one tile (no propagator prefetch): one barrier per level.
template <int K, int KMAX, int NU, int ND, int QMAX, int NT, typename C>
__device__ __forceinline__ void tile_levels(const FlavTabs<NU, QMAX, NT>& tu, const FlavTabs<ND, QMAX, NT>& td,
                                            const int32_t* tr, const int4* sOps, const C* sS, C* sR) {
  if constexpr (K <= KMAX) {
    if constexpr (K <= NU && (K >= 2 || NU == 1)) run_level<K>(tu, tr, 0, sOps, sS, sR);
    if constexpr (K <= ND && (K >= 2 || ND == 1)) run_level<K>(td, tr, 1, sOps, sS + 144, sR);
    __syncthreads();
    tile_levels<K + 1, KMAX, NU, ND, QMAX, NT, C>(tu, td, tr, sOps, sS, sR);
  }
}

// ---------------------------------------------------------------------------
// dS
// ---------------------------------------------------------------------------
// Register tables of the reverse sweep, loaded once per correlator.
//
// S-bar partials of a level-K row: bin j collects the columns C that contain
// j.  Levels K <= 2 have short bins (at most 11 entries): one lane per bin,
// thread t takes bin t % 12 of row group t / 12 (21 rows side by side).
// Levels K >= 3: L = 16 lanes per bin (workgroups of fewer than 384 threads)
// or 32 (384 threads or more), thread t takes bin t / L (t < 12 L) of one
// row, lane t % L holds entries l, l + L, ...; 32 lanes halve the entries
// per lane, so the 3He rows' bins (up to 224 entries) take 7 registers.
// Level 2 with 384 threads or more: 4 lanes per bin (3 entries each).
__host__ __device__ constexpr int bin_lanes(int k, int nt) {
  return k == 1 ? 1 : (k == 2 ? (nt >= 384 ? 4 : 1) : (nt >= 384 ? 32 : 16));
}
__host__ __device__ constexpr int bin_regs(int k, int nt) {
  return k == 1 ? 1 : (k == 2 ? (nt >= 384 ? 3 : 11) : (nt >= 384 ? (k == 3 ? 2 : (k == 4 ? 6 : 7)) : (k == 3 ? 4 : (k == 4 ? 11 : 14))));
}

// Sum over the 4 lanes of each quad (every lane receives the quad's sum).
__device__ __forceinline__ float quad4_sum(float x) {
  x += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0xB1, 0xf, 0xf, false));
  x += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x4E, 0xf, 0xf, false));
  return x;
}
__device__ __forceinline__ double quad4_sum(double x) {
  x += dpp_f64<0xB1>(x);
  x += dpp_f64<0x4E>(x);
  return x;
}

template <int K, int NT>
struct BinTab {
  static constexpr int kRegs = bin_regs(K, NT), kLanes = bin_lanes(K, NT);
  int e[kRegs];
  __device__ __forceinline__ void load(const int32_t* cr, int f, const int32_t* __restrict__ btab, int t) {
    // unused slots read column ncol of the row: its zero element
    const int pad = cr[8 + 2 * (6 * f + K - 1)];
#pragma unroll
    for (int m = 0; m < kRegs; ++m) e[m] = pad;
    const int32_t* jl = btab + cr[40 + 6 * f + K - 1];
    int j, l;
    if constexpr (kLanes == 1) {
      if (t >= 12 * (NT / 12)) return;
      j = t % 12;
      l = 0;
    } else {
      if (t >= 12 * kLanes * (NT / (12 * kLanes))) return;
      j = (t % (12 * kLanes)) / kLanes;
      l = t % kLanes;
    }
    const int q0 = jl[j], q1 = jl[j + 1];
#pragma unroll
    for (int m = 0; m < kRegs; ++m) {
      const int q = q0 + l + kLanes * m;
      if (q < q1) e[m] = jl[q];
    }
  }
};

// Parent adjoints: the (parent, column) items of a level are spread like the
// forward row items: with ncol <= NT, G = NT / ncol parents side by side
// (thread t: item t % ncol of parent group t / ncol); else items t, t + NT.
// Item i takes column col = order[i] of the level's columns ordered by their
// count of supersets, so a wave's columns have similar counts; nw is the
// wave's largest count (uniform).  Entries: index of C' + {j} one level up |
// parity of the position of j << 11 | j << 12, compacted and padded to
// 12 - K entries (the most a K-column can have) with the child row's zero
// element (index ncol one level up), two per int32.
__host__ __device__ constexpr int up_len(int k) { return 12 - k; }

// Parent-table entries per uniform bound check: the loads of a step issue
// together (a level-K parent column has up to 12 - K entries: two steps of
// six for K <= 5).
constexpr int kUpStep = 6;

template <int K, int QMAX, int NT>
struct UpTab {
  int ncol = 0, G = 1, g = 0, i0 = 0;
  unsigned up[QMAX][6];
  int col[QMAX];     // the item's column, ncol if none
  int nw[QMAX];      // entries the wave runs
  int colnum[QMAX];
  __device__ __forceinline__ void load(const int32_t* cr, int f, const int32_t* __restrict__ btab,
                                       const uint16_t* __restrict__ tabs, int t) {
    ncol = cr[8 + 2 * (6 * f + K - 1)];
    const unsigned pad = unsigned(cr[8 + 2 * (6 * f + K)]) & 2047u;  // ncol one level up
    const int32_t* ut = btab + cr[67 + 6 * f + K - 1];
    const int32_t* order = ut + 6 * ncol;
    const int toff = cr[8 + 2 * (6 * f + K - 1) + 1];
    if (ncol > 0 && ncol <= NT) {
      G = NT / ncol;
      g = t / ncol;
      i0 = t % ncol;
    } else {
      G = 1;
      g = 0;
      i0 = t;
    }
#pragma unroll
    for (int q = 0; q < QMAX; ++q) {
      const int i = i0 + NT * q;
      const bool ok = i < ncol && g < G;
      const int c = ok ? order[i] : 0;
      col[q] = ok ? c : ncol;
      int cnt = 0;
#pragma unroll
      for (int w = 0; w < 6; ++w) up[q][w] = 0;
#pragma unroll
      for (int j = 0; j < 12; ++j) {
        const unsigned ent = ok ? ((unsigned(ut[6 * c + (j >> 1)]) >> (16 * (j & 1))) & 0xffffu) : 0xffffu;
        if (ent != 0xffffu) {
          const unsigned packed = (ent & 2047u) | (((ent >> 12) & 1u) << 11) | (unsigned(j) << 12);
          // compact: entry cnt goes to half (cnt & 1) of word cnt >> 1
#pragma unroll
          for (int w = 0; w < 6; ++w)
            if ((cnt >> 1) == w) up[q][w] |= packed << (16 * (cnt & 1));
          ++cnt;
        }
      }
#pragma unroll
      for (int m = 0; m < up_len(K); ++m)
        if (m >= cnt) up[q][m >> 1] |= pad << (16 * (m & 1));
      colnum[q] = (K == 1 && ok) ? int(tabs[toff + c]) : 0;
      for (int off = 32; off > 0; off >>= 1) cnt = max(cnt, __shfl_xor(cnt, off));
      nw[q] = __builtin_amdgcn_readfirstlane(cnt);
    }
  }
};

// Leaf adjoints: thread owns top columns c = t, t + NT and keeps the source
// keys of each (s | other-flavour column << 11).
// Unused slots pair source key 0 with the zero element of the other
// flavour's top row; nw[q] is the largest list length in the wave.
template <int QMAX, int MC, int NT>
struct CsrTab {
  int ncol = 0;
  int nw[QMAX];
  int e[QMAX][MC];
  __device__ __forceinline__ void load(const int32_t* cr, int f, int nf, int nf_other,
                                       const int32_t* __restrict__ btab, const int32_t* __restrict__ other_col,
                                       int t) {
    ncol = cr[8 + 2 * (6 * f + nf - 1)];
    const int pad = cr[8 + 2 * (6 * (1 - f) + nf_other - 1)] << 11;
    const int32_t* lists = btab + cr[64 + f];
    const int src_off = cr[1];
#pragma unroll
    for (int q = 0; q < QMAX; ++q) {
      const int c = t + NT * q;
      int n = 0, q0 = 0;
      if (c < ncol) {
        q0 = lists[c];
        n = lists[c + 1] - q0;
      }
#pragma unroll
      for (int m = 0; m < MC; ++m) {
        int v = pad;
        if (m < n) {
          const int sidx = lists[q0 + m];
          v = sidx | (other_col[src_off + sidx] << 11);
        }
        e[q][m] = v;
      }
      for (int off = 32; off > 0; off >>= 1) n = max(n, __shfl_xor(n, off));
      nw[q] = __builtin_amdgcn_readfirstlane(n);
    }
  }
};

// Leaf adjoint of one top column: sum over the group's sink keys b and the
// first NM entries (s, oc) of the column's source-key list of
// W[b, s] * (other flavour's top minor at b's row slot, column oc).  The u
// leaves take the run [lo, hi) and the d slots of its keys; the d leaves take
// the sink keys in the bit mask lo and their u slots.
template <int NM, int MC, bool MASK, typename C>
__device__ __forceinline__ C leaf_terms(const int (&e)[MC], int lo, int hi, const C* sW, int n_src, const C* sR,
                                        const int2* sMeta) {
  C sum = cmake<C>(0, 0);
  int sidx[NM], oc[NM];
#pragma unroll
  for (int m = 0; m < NM; ++m) {
    sidx[m] = e[m] & 2047;
    oc[m] = e[m] >> 11;
  }
  auto key = [&](int b) {
    const C* wrow = sW + b * n_src;
    const C* orow = sR + (MASK ? sMeta[b].x : sMeta[b].y);
#pragma unroll
    for (int m = 0; m < NM; ++m) sum = cmac(wrow[sidx[m]], orow[oc[m]], sum);
  };
  if constexpr (MASK) {
    for (int mm = lo; mm; mm &= mm - 1) key(__ffs(mm) - 1);
  } else {
    for (int b = lo; b < hi; ++b) key(b);
  }
  return sum;
}

// Dispatch on the wave's longest list (nw, uniform), in steps of two entries;
// the padded entries of shorter lists read the zero element.  (This form
// keeps all of a key's loads in flight; the factored leaves below use
// predicated steps instead, where this dispatch was compiled into loops
// indexing their entry arrays in scratch memory.)
template <int N, int MC, bool MASK, typename C>
__device__ __forceinline__ C leaf_sum(int nw, const int (&e)[MC], int lo, int hi, const C* sW, int n_src,
                                      const C* sR, const int2* sMeta) {
  if constexpr (N >= MC) {
    return leaf_terms<MC, MC, MASK>(e, lo, hi, sW, n_src, sR, sMeta);
  } else {
    if (nw <= N) return leaf_terms<N, MC, MASK>(e, lo, hi, sW, n_src, sR, sMeta);
    return leaf_sum<N + 2, MC, MASK>(nw, e, lo, hi, sW, n_src, sR, sMeta);
  }
}

// Factored weights W[b, s] = u[b] v[s] (v = sW[0, n_src), u = sW[n_src, n_src + B)).
// Slot field of a staged key record; bit 30 of the d slot marks the first key
// of the tile with its d-tuple.
constexpr int kSlotMask = (1 << 30) - 1;

// u top column of a run [b0, b1): sum over the first nw (the wave's longest
// list, uniform) entries of the column's source-key list of
// v[s] sum_b u[b] Dd_b[c_d(s)], in groups of G entries with the keys inside,
// so that a key's gathers of a group are in flight together; padded entries
// read the zero element.
template <int MC, typename C>
__device__ __forceinline__ C leaf_u_fact(int nw, const int (&e)[MC], int b0, int b1, const C* sW, int n_src,
                                         const C* sR, const int2* sMeta) {
  constexpr int G = 2;
  const C* sU = sW + n_src;
  C sum = cmake<C>(0, 0);
#pragma unroll
  for (int m0 = 0; m0 < MC; m0 += G) {
    if (m0 < nw) {
      C t[G];
#pragma unroll
      for (int j = 0; j < G; ++j) t[j] = cmake<C>(0, 0);
      for (int b = b0; b < b1; ++b) {
        const C u = sU[b];
        const C* orow = sR + (sMeta[b].y & kSlotMask);
#pragma unroll
        for (int j = 0; j < G; ++j)
          if (m0 + j < MC) t[j] = cmac(u, orow[e[m0 + j] >> 11], t[j]);
      }
#pragma unroll
      for (int j = 0; j < G; ++j)
        if (m0 + j < MC) sum = cmac(sW[e[m0 + j] & 2047], t[j], sum);
    }
  }
  return sum;
}

// d top column, one run: H = sum over the first nw entries of the column's
// source-key list of v[s] Du[c_u(s)] (du: the run's u top row).  The run's
// keys b then add u[b] H to the adjoint of their d top row.
template <int MC, typename C>
__device__ __forceinline__ C leaf_h_fact(int nw, const int (&e)[MC], const C* sW, const C* du) {
  C sum = cmake<C>(0, 0);
#pragma unroll
  for (int m0 = 0; m0 < MC; m0 += 2)
    if (m0 < nw) {
#pragma unroll
      for (int m = m0; m < m0 + 2 && m < MC; ++m) sum = cmac(sW[e[m] & 2047], du[e[m] >> 11], sum);
    }
  return sum;
}

template <int NF, int QMAX, int NT>
struct RevTabs {
  BinTab<1, NT> b1;
  BinTab<2, NT> b2;
  BinTab<3, NT> b3;
  BinTab<4, NT> b4;
  BinTab<5, NT> b5;
  UpTab<1, QMAX, NT> u1;
  UpTab<2, QMAX, NT> u2;
  UpTab<3, QMAX, NT> u3;
  UpTab<4, QMAX, NT> u4;
  int tb = 0;  // lane order of the S-bar bins; the parent tables take their own
  __device__ __forceinline__ void load(const int32_t* cr, int f, const int32_t* btab, const uint16_t* tabs,
                                       int t_bins, int t_ups) {
    tb = t_bins;
    if constexpr (NF == 1) b1.load(cr, f, btab, t_bins);
    if constexpr (NF >= 2) b2.load(cr, f, btab, t_bins);
    if constexpr (NF >= 3) b3.load(cr, f, btab, t_bins);
    if constexpr (NF >= 4) b4.load(cr, f, btab, t_bins);
    if constexpr (NF >= 5) b5.load(cr, f, btab, t_bins);
    if constexpr (NF >= 2) u1.load(cr, f, btab, tabs, t_ups);
    if constexpr (NF >= 3) u2.load(cr, f, btab, tabs, t_ups);
    if constexpr (NF >= 4) u3.load(cr, f, btab, tabs, t_ups);
    if constexpr (NF >= 5) u4.load(cr, f, btab, tabs, t_ups);
  }
};

template <int K, int NF, int QMAX, int NT>
__device__ __forceinline__ const BinTab<K, NT>& bins_of(const RevTabs<NF, QMAX, NT>& rt) {
  if constexpr (K == 1) return rt.b1;
  else if constexpr (K == 2) return rt.b2;
  else if constexpr (K == 3) return rt.b3;
  else if constexpr (K == 4) return rt.b4;
  else return rt.b5;
}
template <int K, int NF, int QMAX, int NT>
__device__ __forceinline__ const UpTab<K, QMAX, NT>& ups_of(const RevTabs<NF, QMAX, NT>& rt) {
  if constexpr (K == 1) return rt.u1;
  else if constexpr (K == 2) return rt.u2;
  else if constexpr (K == 3) return rt.u3;
  else return rt.u4;
}

template <int K, int NT, typename C>
__device__ __forceinline__ C bin_sum(const BinTab<K, NT>& bt, int4 ov, const C* Sf, const C* sR, const C* sA) {
  C sum = cmake<C>(0, 0);
#pragma unroll
  for (int m = 0; m < BinTab<K, NT>::kRegs; ++m) {
    const int e = bt.e[m];
    const C av = sA[ov.z + (e & 4095)];
    if constexpr (K == 1) {
      sum.x += av.x;
      sum.y += av.y;
    } else {
      const int sub = (e >> 12) & 4095;
      const C y = (K == 2) ? Sf[12 * ov.y + sub] : sR[ov.y + sub];
      sum = cmac(cneg_if(av, (e >> 24) & 1), y, sum);
    }
  }
  return sum;
}

// (ii) S-bar partials of the level-K rows [o0, o0 + cnt) of one flavour:
// part[o][j] = sum over columns C containing j of (-1)^pos A(C) M_{K-1}(C \ j).
// One lane per bin (L = 1): NT / 12 rows side by side.  Otherwise NT / (12 L)
// groups of 12 bins x L lanes, each taking two rows per trip.
template <int K, int NT, typename C>
__device__ __forceinline__ void rev_part(const BinTab<K, NT>& bt, int tid, int o0, int cnt, const int4* sOpv,
                                         const C* Sf, const C* sR, const C* sA, C* sPart) {
  if constexpr (BinTab<K, NT>::kLanes == 1) {
    constexpr int RB = NT / 12;
    if (tid >= 12 * RB) return;
    const int j = tid % 12;
    for (int o = o0 + tid / 12; o < o0 + cnt; o += RB) sPart[12 * o + j] = bin_sum<K>(bt, sOpv[o], Sf, sR, sA);
  } else {
    constexpr int L = BinTab<K, NT>::kLanes;
    constexpr int GW = 12 * L;
    constexpr int NG = NT / GW;
    if (tid >= GW * NG) return;
    const int lt = tid % GW;
    for (int o = o0 + 2 * (tid / GW); o < o0 + cnt; o += 2 * NG) {
      const bool two = o + 1 < o0 + cnt;
      C s0 = bin_sum<K>(bt, sOpv[o], Sf, sR, sA);
      C s1 = two ? bin_sum<K>(bt, sOpv[o + 1], Sf, sR, sA) : cmake<C>(0, 0);
      if constexpr (L == 4) {
        s0.x = quad4_sum(s0.x);
        s0.y = quad4_sum(s0.y);
        s1.x = quad4_sum(s1.x);
        s1.y = quad4_sum(s1.y);
      } else {
        s0.x = row16_sum(s0.x);
        s0.y = row16_sum(s0.y);
        s1.x = row16_sum(s1.x);
        s1.y = row16_sum(s1.y);
      }
      // 32-lane bins are aligned halves of the wave: the upper 16-lane row
      // adds the lower row's sum and its first lane writes
      if constexpr (L == 32) {
        s0.x = upper_row_pair_sum(s0.x);
        s0.y = upper_row_pair_sum(s0.y);
        s1.x = upper_row_pair_sum(s1.x);
        s1.y = upper_row_pair_sum(s1.y);
      }
      if (lt % L == (L == 32 ? 16 : 0)) {
        sPart[12 * o + lt / L] = s0;
        if (two) sPart[12 * (o + 1) + lt / L] = s1;
      }
    }
  }
}

// One child row's terms of a parent column: sum over the first nw up entries
// (superset C' + j: its index in the child row, the parity of j's position,
// j) of (-1)^pos S[r0, j] A_K(child, C' + j); ce = child slot << 4 | r0.
template <int KP, bool BOUND, typename C>
__device__ __forceinline__ C child_terms(const unsigned (&up)[6], int nw, int ce, const C* Sf, const C* sA) {
  const C* srow = Sf + 12 * (ce & 15);
  const C* arow = sA + (ce >> 4);
  C sum = cmake<C>(0, 0);
#pragma unroll
  for (int m0 = 0; m0 < up_len(KP); m0 += kUpStep) {
    if (!BOUND || m0 < nw) {  // entries past a lane's count read the zero element
#pragma unroll
      for (int m = m0; m < m0 + kUpStep && m < up_len(KP); ++m) {
        const unsigned ent = (up[m >> 1] >> (16 * (m & 1))) & 0xffffu;
        const C av = arow[int(ent & 2047u)];
        sum = cmac(cneg_if(av, int((ent >> 11) & 1u)), srow[ent >> 12], sum);
      }
    }
  }
  return sum;
}

// (i) adjoints of the parents of level K-1 (real rows; S rows for K = 2):
// A_{K-1}(C') = sum over children, over j not in C', of (-1)^pos S[r0, j] A_K(C' + j).
// The first child (most parents have one) is summed straight-line.
template <int K, bool BOUND, int QMAX, int NT, typename C>
__device__ __forceinline__ void rev_parents(const UpTab<K - 1, QMAX, NT>& ut, int p0, int pcnt, const int4* sOpx,
                                            const int4* sOpv, const int32_t* children, const C* Sf, C* sA,
                                            C* sAdj1) {
  if (ut.g >= ut.G) return;
  for (int p = p0 + ut.g; p < p0 + pcnt; p += ut.G) {
    const int4 ox = sOpx[p];
    const int nch = ox.w & 0xffff;
    if (nch == 0) continue;  // a top row: its adjoint came from the leaves
    const int4 ov = sOpv[p];
    const int c1 = children[ox.z];
#pragma unroll
    for (int q = 0; q < QMAX; ++q) {
      const int c = ut.col[q];
      if (c < ut.ncol) {
        C sum = child_terms<K - 1, BOUND>(ut.up[q], ut.nw[q], c1, Sf, sA);
        for (int ci = 1; ci < nch; ++ci) {
          const C t = child_terms<K - 1, BOUND>(ut.up[q], ut.nw[q], children[ox.z + ci], Sf, sA);
          sum.x += t.x;
          sum.y += t.y;
        }
        if (K == 2)
          sAdj1[ov.z + ut.colnum[q]] = sum;
        else
          sA[ov.z + c] = sum;
      }
    }
  }
}

template <int K, bool BOUND, int NU, int ND, int QMAX, int NT, typename C>
__device__ __forceinline__ void rev_levels(const RevTabs<NU, QMAX, NT>& ru, const RevTabs<ND, QMAX, NT>& rd,
                                           const int32_t* tr, const int4* sOpx, const int4* sOpv,
                                           const int32_t* children, const C* sS, const C* sR, C* sA, C* sAdj1,
                                           C* sPart) {
  if constexpr (K >= 1) {
    if constexpr (K <= NU)
      rev_part<K>(bins_of<K>(ru), ru.tb, tr[20 + 2 * K], tr[21 + 2 * K], sOpv, sS, sR, sA, sPart);
    if constexpr (K <= ND)
      rev_part<K>(bins_of<K>(rd), rd.tb, tr[20 + 2 * (7 + K)], tr[21 + 2 * (7 + K)], sOpv, sS + 144, sR, sA, sPart);
    if constexpr (K >= 2) {
      // parents: real rows of level K-1, or the level-1 records for K = 2
      if constexpr (K <= NU) {
        const int p0 = (K == 2) ? tr[17] : tr[20 + 2 * (K - 1)];
        const int pc = (K == 2) ? tr[14] : tr[21 + 2 * (K - 1)];
        rev_parents<K, BOUND>(ups_of<K - 1>(ru), p0, pc, sOpx, sOpv, children, sS, sA, sAdj1);
      }
      if constexpr (K <= ND) {
        const int p0 = (K == 2) ? tr[17] + tr[14] : tr[20 + 2 * (7 + K - 1)];
        const int pc = (K == 2) ? tr[18] - tr[14] : tr[21 + 2 * (7 + K - 1)];
        rev_parents<K, BOUND>(ups_of<K - 1>(rd), p0, pc, sOpx, sOpv, children, sS + 144, sA, sAdj1);
      }
    }
    __syncthreads();
    rev_levels<K - 1, BOUND, NU, ND, QMAX, NT, C>(ru, rd, tr, sOpx, sOpv, children, sS, sR, sA, sAdj1, sPart);
  }
}

template <typename R, int NU, int ND, int QMAX, int MC, int NT, bool FACT>
__global__ __launch_bounds__(NT) void ds_kernel(BwdArgs a) {
  using C = typename cx<R>::T;
  constexpr int KMIN = (NU == 1 || ND == 1) ? 1 : 2;
  constexpr int KMAX = NU > ND ? NU : ND;
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x;
  const int64_t site = blockIdx.x;
  const int t = int(site / a.V);
  C* sS = reinterpret_cast<C*>(smem);
  for (int i = tid; i < 288; i += NT)
    sS[i] = load_site<C>(i < 144 ? a.S_u : a.S_d, a.s_c64, site * 144 + (i % 144));

  // Lane orders: the workgroup's lanes are rotated by a multiple of a wave
  // (so that co-resident workgroups put their busiest wave on different
  // SIMDs), and the u and d flavours and the parent tables start half a
  // workgroup / a quarter apart, so that small per-flavour tasks of one
  // level run on different waves side by side.
  constexpr int NQ = (288 + NT - 1) / NT;  // S-bar entries per thread
  const int vt = rotated_lane<NT>();
  const int vt_u = vt, vt_d = (vt + NT / 2) & (NT - 1);
  const int vt_pu = (vt + NT / 4) & (NT - 1), vt_pd = (vt + 3 * NT / 4) & (NT - 1);
  CompAcc<R> sb[NQ];  // S-bar entries vt + NT q (< 288)
  int cur_corr = -1;
  FlavTabs<NU, QMAX, NT> tu;
  FlavTabs<ND, QMAX, NT> td;
  RevTabs<NU, QMAX, NT> ru;
  RevTabs<ND, QMAX, NT> rd;
  CsrTab<QMAX, MC, NT> cu_tab, cd_tab;
  const int4* meta_all = reinterpret_cast<const int4*>(a.meta);

  for (int tile = 0; tile < a.n_tiles; ++tile) {
    const int32_t* tr = a.tiles + tile * kTileInts;
    const int corr = tr[0], B = tr[1], w_off = tr[2], op0 = tr[3], nops = tr[4];
    const int meta0 = tr[5], units = tr[6], nreal = tr[17], nvirt = tr[18], ex_off = tr[19], ex_len = tr[15];
    const int32_t* cr = a.corr + corr * kCorrInts;
    const int n_src = cr[0];
    if (corr != cur_corr) {
      tu.load(cr, 0, a.tabs, vt_u);
      td.load(cr, 1, a.tabs, vt_d);
      ru.load(cr, 0, a.btab, a.tabs, vt_u, vt_pu);
      rd.load(cr, 1, a.btab, a.tabs, vt_d, vt_pd);
      cu_tab.load(cr, 0, NU, ND, a.btab, a.src_cd, vt_u);
      cd_tab.load(cr, 1, ND, NU, a.btab, a.src_cu, vt_d);
      cur_corr = corr;
    }
    C gbar;
    gbar.x = R(a.grad_C[2 * (int64_t(corr) * a.T + t)]);
    gbar.y = R(-a.grad_C[2 * (int64_t(corr) * a.T + t) + 1]);
    C* sW = sS + 288;  // W (B x n_src), or FACT: the factors v (n_src) and u (B)
    C* sR = sW + (FACT ? n_src + B : B * n_src);
    C* sA = sR + units;
    C* sAdj1 = sA + units;
    C* sPart = sAdj1 + 12 * nvirt;
    int4* sOps = lds_align16<int4>(smem, sPart + 12 * nreal);
    int4* sOpx = sOps + nreal;  // (f, k, child_begin, n_children | virt << 16)
    int4* sOpv = sOpx + nops;   // (r0, in, out, 0)
    int32_t* sEx = reinterpret_cast<int32_t*>(sOpv + nops);
    int2* sMeta = reinterpret_cast<int2*>(sEx + ((ex_len + 1) & ~1));  // (u slot, d slot) of each sink key
    __syncthreads();  // the previous tile's LDS is no longer read
    if constexpr (FACT) {
      stage_lds<NT>(sW, reinterpret_cast<const C*>(a.wv) + cr[1], n_src);
      if (tid < B) sW[n_src + tid] = reinterpret_cast<const C*>(a.wu)[cr[32] + tr[16] + tid];
    } else {
      stage_lds<NT>(sW, reinterpret_cast<const C*>(a.W) + w_off, B * n_src);
    }
    if (tid < B) {
      const int4 mb = meta_all[meta0 + tid];
      sMeta[tid] = make_int2(mb.x, FACT ? (mb.y | ((mb.z & 2) << 29)) : mb.y);
    }
    for (int i = tid; i < nops; i += NT) {
      const int4* op = reinterpret_cast<const int4*>(a.ops + int64_t(op0 + i) * kOpInts);
      const int4 lo = op[0], hi = op[1];  // (f, k, r0, in), (out, child_begin, n_children, virt)
      if (i < nreal) {
        sOps[i] = make_int4(lo.z, lo.w, hi.x, 0);
        const int pad = hi.x + cr[8 + 2 * (6 * lo.x + lo.y - 1)];
        sR[pad] = cmake<C>(0, 0);
        sA[pad] = cmake<C>(0, 0);
      }
      sOpv[i] = make_int4(lo.z, lo.w, hi.x, 0);
      sOpx[i] = make_int4(lo.x, lo.y, hi.y, hi.z | (hi.w << 16));
    }
    for (int i = tid; i < ex_len; i += NT) sEx[i] = a.extra[ex_off + i];
    for (int i = tid; i < 12 * nvirt; i += NT) sAdj1[i] = cmake<C>(0, 0);
    __syncthreads();

    tile_levels<KMIN, KMAX, NU, ND, QMAX, NT, C>(tu, td, tr, sOps, sS, sR);

    // adjoints of the top rows from the factor-tree leaves
    if constexpr (FACT) {
      // per run: u top row adjoint (u columns), and u[b] H added to the d top
      // row adjoint of each key b of the run (d columns; the first key of a
      // d-tuple writes, later ones add, in key order)
      const int n_runs = sEx[0];
      const int32_t* runs = sEx + 3;
      const C* sU = sW + n_src;
      for (int r = 0; r < n_runs; ++r) {
        const int us = runs[3 * r], b0 = runs[3 * r + 1], b1 = runs[3 * r + 2];
#pragma unroll
        for (int q = 0; q < QMAX; ++q) {
          const int c = vt_u + NT * q;
          if (c < cu_tab.ncol) {
            const C sum = leaf_u_fact<MC>(cu_tab.nw[q], cu_tab.e[q], b0, b1, sW, n_src, sR, sMeta);
            sA[us + c] = cmul(gbar, sum);
          }
        }
#pragma unroll
        for (int q = 0; q < QMAX; ++q) {
          const int c = vt_d + NT * q;
          if (c < cd_tab.ncol) {
            const C h = cmul(gbar, leaf_h_fact<MC>(cd_tab.nw[q], cd_tab.e[q], sW, sR + us));
            for (int b = b0; b < b1; ++b) {
              const int dy = sMeta[b].y;
              C* dst = sA + (dy & kSlotMask) + c;
              C v = cmul(sU[b], h);
              if (!(dy >> 30)) {
                const C o = *dst;
                v.x += o.x;
                v.y += o.y;
              }
              *dst = v;
            }
          }
        }
      }
    } else {
      const int n_runs = sEx[0], n_dg = sEx[1];
      const int32_t* runs = sEx + 3;
      const int32_t* dgs = runs + 3 * n_runs;
      for (int r = 0; r < n_runs; ++r) {
        const int us = runs[3 * r], b0 = runs[3 * r + 1], b1 = runs[3 * r + 2];
#pragma unroll
        for (int q = 0; q < QMAX; ++q) {
          const int c = vt_u + NT * q;
          if (c < cu_tab.ncol) {
            const C sum = leaf_sum<2, MC, false>(cu_tab.nw[q], cu_tab.e[q], b0, b1, sW, n_src, sR, sMeta);
            sA[us + c] = cmul(gbar, sum);
          }
        }
      }
      for (int g = 0; g < n_dg; ++g) {
        const int ds = dgs[2 * g], mask = dgs[2 * g + 1];
#pragma unroll
        for (int q = 0; q < QMAX; ++q) {
          const int c = vt_d + NT * q;
          if (c < cd_tab.ncol) {
            const C sum = leaf_sum<2, MC, true>(cd_tab.nw[q], cd_tab.e[q], mask, 0, sW, n_src, sR, sMeta);
            sA[ds + c] = cmul(gbar, sum);
          }
        }
      }
    }
    __syncthreads();

    const int32_t* children = sEx + 3 + 3 * sEx[0] + 2 * sEx[1];
    const int32_t* rsum = sEx + sEx[2];
    // the wave's superset count bounds the parent sums, except in the
    // unfactored FP32-comp schedule of the dinucleons, which measured faster
    // running every padded entry (D_I F32C 310 vs 333 ms; in FP64, and for
    // the proton and neutron, the unbounded sums take registers enough to
    // cost waves per SIMD)
    constexpr bool kBound = FACT || (NU + ND != 6) || std::is_same<R, double>::value;
    rev_levels<KMAX, kBound, NU, ND, QMAX, NT, C>(ru, rd, tr, sOpx, sOpv, children, sS, sR, sA, sAdj1, sPart);

    // fixed-order accumulation of this tile's S-bar contributions
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int e = vt + NT * q;
      if (e < 288) {
        const int row = e / 12, bc = e % 12;  // row = 12 f + r0
        C sum = cmake<C>(0, 0);
        const int l1 = rsum[row + 1];
        for (int l = rsum[row]; l < l1; ++l) {
          const int o = rsum[l];
          const C v = (o >= nreal) ? sAdj1[sOpv[o].z + bc] : sPart[12 * o + bc];
          sum.x += v.x;
          sum.y += v.y;
        }
        sb[q].add(sum.x, sum.y);
      }
    }
  }

  // grad_S = conj(S-bar)
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int e = vt + NT * q;
    if (e < 288) {
      const double x = double(sb[q].hx) + double(sb[q].lx);
      const double y = -(double(sb[q].hy) + double(sb[q].ly));
      void* base = e < 144 ? a.grad_S_u : a.grad_S_d;
      if (base) {
        const int64_t idx = site * 144 + (e % 144);
        if (a.s_c64) {
          reinterpret_cast<float2*>(base)[idx] = make_float2(float(x), float(y));
        } else {
          reinterpret_cast<double2*>(base)[idx] = make_double2(x, y);
        }
      }
    }
  }
}

template <typename K>
hipError_t launch_k(K k, int nt, int nblocks, size_t lds, hipStream_t st, const BwdArgs& a) {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(nblocks), dim3(nt), lds, st, a);
  return hipGetLastError();
}

// dS launch with the factored (FACT) or the weight-staging schedule, for at
// most MAXCOL columns per level and MC source keys per top column.
template <typename R, int NU, int ND, int MAXCOL, int MC, bool FACT>
hipError_t launch_ds_one(const mbc_plan* p, const BwdArgs& a, int nb, size_t lds, hipStream_t st) {
  constexpr int NT = ds_threads(NU, ND, std::is_same<R, double>::value ? MBC_F64 : MBC_F32C);
  constexpr int QMAX = (MAXCOL + NT - 1) / NT;
  if (p->h.max_ncol > MAXCOL || p->h.max_csr > MC) return hipErrorNotSupported;
  return launch_k(ds_kernel<R, NU, ND, QMAX, MC, NT, FACT>, NT, nb, lds, st, a);
}

template <typename R, int NU, int ND, int MAXCOL, int MC>
hipError_t launch_ds_f(const mbc_plan* p, const BwdArgs& a, int nb, size_t lds, bool factored, hipStream_t st) {
  if (factored) return launch_ds_one<R, NU, ND, MAXCOL, MC, true>(p, a, nb, lds, st);
  return launch_ds_one<R, NU, ND, MAXCOL, MC, false>(p, a, nb, lds, st);
}

}  // namespace

// Factored FP32-comp dS launch of the (5, 4) family (3He), compiled in a unit
// of its own whose instruction scheduler favours instruction-level
// parallelism: the kernel runs two waves per SIMD at its register limit, so
// its LDS gathers' latency is hidden only by keeping many of them in flight.
hipError_t launch_ds_5_4_factored_f32(const mbc_plan* p, const BwdArgs& a, int nb, size_t lds, hipStream_t st);

}  // namespace mbc
