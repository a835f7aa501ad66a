// HIP kernels of the adjoint (backward) contraction for gfx950.
//
// dW kernel (one workgroup = one tile of sink keys x the sites of one
// timeslice chunk): rebuilds the tile's determinant rows per site exactly as
// the forward kernel does, and accumulates Q[b,s] = sum_x Du Dd per index
// entry (C is linear in W, eq. 1) in compensated accumulators in LDS; the
// chunk's grad_C[t] conj(Q) is written in FP64 and the chunks are summed in
// a fixed order by dw_reduce_kernel.
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
#include <hip/hip_runtime.h>

#include <cstdint>

#include "device_common.hpp"
#include "kernels.hpp"

namespace mbc {

namespace {

using namespace dev;

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
};

template <typename C>
__device__ __forceinline__ C cconj(C a) {
  a.y = -a.y;
  return a;
}

// Rows of one site for one tile (no propagator prefetch): one barrier per level.
template <int K, int KMAX, int NU, int ND, int QMAX, typename C>
__device__ __forceinline__ void tile_levels(const FlavTabs<NU, QMAX>& tu, const FlavTabs<ND, QMAX>& td,
                                            const int32_t* tr, const int4* sOps, const C* sS, C* sR) {
  if constexpr (K <= KMAX) {
    if constexpr (K <= NU && (K >= 2 || NU == 1)) run_level<K>(tu, tr, 0, sOps, sS, sR);
    if constexpr (K <= ND && (K >= 2 || ND == 1)) run_level<K>(td, tr, 1, sOps, sS + 144, sR);
    __syncthreads();
    tile_levels<K + 1, KMAX, NU, ND, QMAX, C>(tu, td, tr, sOps, sS, sR);
  }
}

// Same with the next site's propagators stored during the top level.
template <int K, int KMAX, int NU, int ND, int QMAX, typename C>
__device__ __forceinline__ void site_levels_pf(const FlavTabs<NU, QMAX>& tu, const FlavTabs<ND, QMAX>& td,
                                               const int32_t* tr, const int4* sOps, const C* sS, C* sR, C* sSnext,
                                               const C* pre, bool have_next) {
  if constexpr (K <= KMAX) {
    if constexpr (K <= NU && (K >= 2 || NU == 1)) run_level<K>(tu, tr, 0, sOps, sS, sR);
    if constexpr (K <= ND && (K >= 2 || ND == 1)) run_level<K>(td, tr, 1, sOps, sS + 144, sR);
    if constexpr (K == KMAX) {
      if (have_next) {
        sSnext[threadIdx.x] = pre[0];
        if (threadIdx.x < 288 - kNT) sSnext[kNT + threadIdx.x] = pre[1];
      }
    }
    __syncthreads();
    site_levels_pf<K + 1, KMAX, NU, ND, QMAX, C>(tu, td, tr, sOps, sS, sR, sSnext, pre, have_next);
  }
}

// ---------------------------------------------------------------------------
// dW
// ---------------------------------------------------------------------------
template <typename R, int NU, int ND, int MAXS, int QMAX>
__global__ __launch_bounds__(kNT) void dw_kernel(BwdArgs a) {
  using C = typename cx<R>::T;
  constexpr int KMIN = (NU == 1 || ND == 1) ? 1 : 2;
  constexpr int KMAX = NU > ND ? NU : ND;
  constexpr bool kOverlapLeaves = (NU >= 3 && ND >= 3);
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x;
  const int lin = xcd_linear(blockIdx.x, gridDim.x);
  const int tile = lin % a.n_tiles;
  const int tc = lin / a.n_tiles;
  const int32_t* tr = a.tiles + tile * kTileInts;
  const int corr = tr[0], B = tr[1], w_off = tr[2], op0 = tr[3], nreal = tr[17];
  const int meta0 = tr[5], row_units = tr[6];
  const int32_t* cr = a.corr + corr * kCorrInts;
  const int n_src = cr[0], src_off = cr[1];

  C* sS0 = reinterpret_cast<C*>(smem);
  C* sR = sS0 + 576;
  int4* sOps = reinterpret_cast<int4*>((reinterpret_cast<uintptr_t>(sR + row_units) + 15) & ~uintptr_t(15));
  R* sAcc = reinterpret_cast<R*>(sOps + nreal);  // [B * n_src][4]: hx, lx, hy, ly

  for (int i = tid; i < nreal; i += kNT) {
    const int32_t* op = a.ops + int64_t(op0 + i) * kOpInts;
    sOps[i] = make_int4(op[2], op[3], op[4], 0);
  }
  for (int i = tid; i < 4 * B * n_src; i += kNT) sAcc[i] = R(0);
  const int4* meta = reinterpret_cast<const int4*>(a.meta) + meta0;
  FlavTabs<NU, QMAX> tu;
  FlavTabs<ND, QMAX> td;
  tu.load(cr, 0, a.tabs);
  td.load(cr, 1, a.tabs);
  int cu[MAXS], cd[MAXS];
#pragma unroll
  for (int m = 0; m < MAXS; ++m) {
    const int s = tid + kNT * m;
    cu[m] = s < n_src ? a.src_cu[src_off + s] : 0;
    cd[m] = s < n_src ? a.src_cd[src_off + s] : 0;
  }
  const int t = tc / a.nc, ch = tc % a.nc;
  const int64_t v0 = int64_t(ch) * a.chunk;
  const int64_t v1 = (v0 + a.chunk < a.V) ? v0 + a.chunk : a.V;
  auto fetch = [&](int64_t v, C* pre) {
    const int64_t site = int64_t(t) * a.V + v;
    pre[0] = load_site<C>(tid < 144 ? a.S_u : a.S_d, a.s_c64, site * 144 + (tid % 144));
    if (tid < 288 - kNT) pre[1] = load_site<C>(a.S_d, a.s_c64, site * 144 + (kNT + tid - 144));
  };
  C pre[2];
  fetch(v0, pre);
  sS0[tid] = pre[0];
  if (tid < 288 - kNT) sS0[kNT + tid] = pre[1];
  __syncthreads();
  for (int64_t v = v0; v < v1; ++v) {
    const int buf = int((v - v0) & 1);
    C* sS = sS0 + 288 * buf;
    C* sSn = sS0 + 288 * (buf ^ 1);
    const bool have_next = v + 1 < v1;
    if (have_next) fetch(v + 1, pre);
    site_levels_pf<KMIN, KMAX, NU, ND, QMAX, C>(tu, td, tr, sOps, sS, sR, sSn, pre, have_next);
    for (int b = 0; b < B; ++b) {
      const int4 mb = meta[b];
#pragma unroll
      for (int m = 0; m < MAXS; ++m) {
        const int s = tid + kNT * m;
        if (s < n_src) {
          const C p = cmul(sR[mb.x + cu[m]], sR[mb.y + cd[m]]);
          R* acc = sAcc + 4 * (b * n_src + s);
          R sx, ex, sy, ey;
          two_sum(acc[0], p.x, sx, ex);
          two_sum(acc[2], p.y, sy, ey);
          acc[0] = sx;
          acc[1] += ex;
          acc[2] = sy;
          acc[3] += ey;
        }
      }
    }
    if constexpr (!kOverlapLeaves) __syncthreads();
  }
  __syncthreads();
  const double gx = a.grad_C[2 * (int64_t(corr) * a.T + t)], gy = a.grad_C[2 * (int64_t(corr) * a.T + t) + 1];
  double* out = a.partial + 2 * (int64_t(tc) * a.nnz + w_off);
  for (int i = tid; i < B * n_src; i += kNT) {
    const R* acc = sAcc + 4 * i;
    const double qx = double(acc[0]) + double(acc[1]);
    const double qy = -(double(acc[2]) + double(acc[3]));  // conj(Q)
    out[2 * i] = gx * qx - gy * qy;
    out[2 * i + 1] = gx * qy + gy * qx;
  }
}

__global__ __launch_bounds__(256) void dw_reduce_kernel(const double* __restrict__ partial, int ntc, int64_t nnz,
                                                        const int64_t* __restrict__ perm, double* __restrict__ gW) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nnz) return;
  CompAcc<double> acc;
  for (int tc = 0; tc < ntc; ++tc) {
    const double* p = partial + 2 * (int64_t(tc) * nnz + i);
    acc.add(p[0], p[1]);
  }
  const int64_t k = perm[i];
  gW[2 * k] = acc.hx + acc.lx;
  gW[2 * k + 1] = acc.hy + acc.ly;
}

// ---------------------------------------------------------------------------
// dS
// ---------------------------------------------------------------------------
template <typename R, int NU, int ND, int QMAX>
__global__ __launch_bounds__(kNT) void ds_kernel(BwdArgs a) {
  using C = typename cx<R>::T;
  constexpr int KMIN = (NU == 1 || ND == 1) ? 1 : 2;
  constexpr int KMAX = NU > ND ? NU : ND;
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x;
  const int64_t site = blockIdx.x;
  const int t = int(site / a.V);
  C* sS = reinterpret_cast<C*>(smem);
  for (int i = tid; i < 288; i += kNT)
    sS[i] = load_site<C>(i < 144 ? a.S_u : a.S_d, a.s_c64, site * 144 + (i % 144));

  // S-bar entries owned by this thread: e = tid and tid + NT (< 288)
  CompAcc<R> sb[2];
  int cur_corr = -1;
  FlavTabs<NU, QMAX> tu;
  FlavTabs<ND, QMAX> td;
  const int4* meta_all = reinterpret_cast<const int4*>(a.meta);

  for (int tile = 0; tile < a.n_tiles; ++tile) {
    const int32_t* tr = a.tiles + tile * kTileInts;
    const int corr = tr[0], B = tr[1], w_off = tr[2], op0 = tr[3], nops = tr[4];
    const int meta0 = tr[5], units = tr[6], nreal = tr[17], nvirt = tr[18], ex_off = tr[19], ex_len = tr[15];
    const int32_t* cr = a.corr + corr * kCorrInts;
    const int n_src = cr[0], src_off = cr[1];
    if (corr != cur_corr) {
      tu.load(cr, 0, a.tabs);
      td.load(cr, 1, a.tabs);
      cur_corr = corr;
    }
    C gbar;
    gbar.x = R(a.grad_C[2 * (int64_t(corr) * a.T + t)]);
    gbar.y = R(-a.grad_C[2 * (int64_t(corr) * a.T + t) + 1]);
    C* sW = sS + 288;
    C* sR = sW + B * n_src;
    C* sA = sR + units;
    C* sAdj1 = sA + units;
    C* sPart = sAdj1 + 12 * nvirt;
    int4* sOps = reinterpret_cast<int4*>((reinterpret_cast<uintptr_t>(sPart + 12 * nreal) + 15) & ~uintptr_t(15));
    int4* sOpx = sOps + nreal;                                  // (f, k, child_begin, n_children | virt << 16)
    int4* sOpv = sOpx + nops;                                   // (r0, in, out, 0) of all ops
    int32_t* sEx = reinterpret_cast<int32_t*>(sOpv + nops);
    __syncthreads();  // the previous tile's LDS is no longer read
    const C* Wg = reinterpret_cast<const C*>(a.W) + w_off;
    for (int i = tid; i < B * n_src; i += kNT) sW[i] = Wg[i];
    for (int i = tid; i < nops; i += kNT) {
      const int32_t* op = a.ops + int64_t(op0 + i) * kOpInts;
      if (i < nreal) sOps[i] = make_int4(op[2], op[3], op[4], 0);
      sOpv[i] = make_int4(op[2], op[3], op[4], 0);
      sOpx[i] = make_int4(op[0], op[1], op[5], op[6] | (op[7] << 16));
    }
    for (int i = tid; i < ex_len; i += kNT) sEx[i] = a.extra[ex_off + i];
    for (int i = tid; i < 12 * nvirt; i += kNT) sAdj1[i] = cmake<C>(0, 0);
    __syncthreads();

    tile_levels<KMIN, KMAX, NU, ND, QMAX, C>(tu, td, tr, sOps, sS, sR);

    // adjoints of the top rows from the factor-tree leaves
    {
      const int n_runs = sEx[0], n_dg = sEx[1];
      const int32_t* runs = sEx + 2;
      const int32_t* dgs = runs + 3 * n_runs;
      const int4* meta = meta_all + meta0;
      const int ncu = cr[8 + 2 * (NU - 1)], ncd = cr[8 + 2 * (6 + ND - 1)];
      const int32_t* csru = a.btab + cr[64];
      const int32_t* csrd = a.btab + cr[65];
      for (int r = 0; r < n_runs; ++r) {
        const int us = runs[3 * r], b0 = runs[3 * r + 1], b1 = runs[3 * r + 2];
        for (int c = tid; c < ncu; c += kNT) {
          C sum = cmake<C>(0, 0);
          const int q1 = csru[c + 1];
          for (int q = csru[c]; q < q1; ++q) {
            const int s = csru[q];
            const int cds = a.src_cd[src_off + s];
            for (int b = b0; b < b1; ++b) sum = cmac(sW[b * n_src + s], sR[meta[b].y + cds], sum);
          }
          sA[us + c] = cmul(gbar, sum);
        }
      }
      for (int g = 0; g < n_dg; ++g) {
        const int ds = dgs[2 * g], mask = dgs[2 * g + 1];
        for (int c = tid; c < ncd; c += kNT) {
          C sum = cmake<C>(0, 0);
          const int q1 = csrd[c + 1];
          for (int q = csrd[c]; q < q1; ++q) {
            const int s = csrd[q];
            const int cus = a.src_cu[src_off + s];
            for (int b = 0; b < B; ++b)
              if (mask & (1 << b)) sum = cmac(sW[b * n_src + s], sR[meta[b].x + cus], sum);
          }
          sA[ds + c] = cmul(gbar, sum);
        }
      }
    }
    __syncthreads();

    // reverse sweep of the Laplace recursion
    const int32_t* children = sEx + 2 + 3 * sEx[0] + 2 * sEx[1];
    for (int k = KMAX; k >= 1; --k) {
      // (ii) per-row partials of S-bar[r0, j], 16 lanes per (row, j)
      {
        int lo = 0, cnt = 0;
        const int cu_ = (k <= NU) ? tr[21 + 2 * k] : 0, cd_ = (k <= ND) ? tr[21 + 2 * (7 + k)] : 0;
        if (cu_ > 0) lo = tr[20 + 2 * k];
        else if (cd_ > 0) lo = tr[20 + 2 * (7 + k)];
        cnt = cu_ + cd_;
        const int lane16 = tid & 15;
        for (int pg = tid >> 4; pg < cnt * 12; pg += kNT / 16) {
          const int o = lo + pg / 12, j = pg % 12;
          const int4 ox = sOpx[o];
          const int4 ov = sOpv[o];
          const int f = ox.x;
          const C* Sf = sS + 144 * f;
          const int32_t* jl = a.btab + cr[40 + 6 * f + k - 1];
          const int q0 = jl[j], q1 = jl[j + 1];
          C sum = cmake<C>(0, 0);
          for (int q = q0 + lane16; q < q1; q += 16) {
            const int e = jl[q];
            const C av = sA[ov.z + (e & 4095)];
            if (k == 1) {
              sum.x += av.x;
              sum.y += av.y;
            } else {
              const int sub = (e >> 12) & 4095;
              const C y = (k == 2) ? Sf[12 * ov.y + sub] : sR[ov.y + sub];
              sum = ((e >> 24) & 1) ? cmsub(av, y, sum) : cmac(av, y, sum);
            }
          }
#pragma unroll
          for (int off = 8; off > 0; off >>= 1) {
            sum.x += __shfl_xor(sum.x, off, 16);
            sum.y += __shfl_xor(sum.y, off, 16);
          }
          if (lane16 == 0) sPart[12 * o + j] = sum;
        }
      }
      // (i) adjoints of the parents at level k-1 (S rows for k = 2)
      if (k >= 2) {
        for (int o = 0; o < nops; ++o) {
          const int4 ox = sOpx[o];
          const int virt = ox.w >> 16, nch = ox.w & 0xffff;
          if (nch == 0) continue;                           // a top row
          if (virt ? (k != 2) : (ox.y != k - 1)) continue;  // not a parent of level k
          const int f = ox.x;
          const int4 ov = sOpv[o];
          const C* Sf = sS + 144 * f;
          const int ncp = cr[8 + 2 * (6 * f + k - 2)];
          const int32_t* sup = a.btab + cr[52 + 6 * f + k - 2];
          const int toff1 = cr[8 + 2 * (6 * f) + 1];
          for (int c = tid; c < ncp; c += kNT) {
            C sum = cmake<C>(0, 0);
            const int q0 = sup[c], q1 = sup[c + 1];
            for (int ci = 0; ci < nch; ++ci) {
              const int4 chv = sOpv[children[ox.z + ci]];
              for (int q = q0; q < q1; ++q) {
                const int e = sup[q];
                const C av = sA[chv.z + (e & 4095)];
                const C x = Sf[12 * chv.x + ((e >> 12) & 15)];
                sum = ((e >> 16) & 1) ? cmsub(av, x, sum) : cmac(av, x, sum);
              }
            }
            if (virt)
              sAdj1[ov.z + a.tabs[toff1 + c]] = sum;
            else
              sA[ov.z + c] = sum;
          }
        }
      }
      __syncthreads();
    }

    // fixed-order accumulation of this tile's S-bar contributions
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int e = tid + kNT * q;
      if (e < 288) {
        const int f = e / 144, ar = (e % 144) / 12, bc = e % 12;
        C sum = cmake<C>(0, 0);
        for (int o = 0; o < nops; ++o) {
          const int4 ox = sOpx[o];
          if (ox.x != f || sOpv[o].x != ar) continue;
          const C v = (ox.w >> 16) ? sAdj1[sOpv[o].z + bc] : sPart[12 * o + bc];
          sum.x += v.x;
          sum.y += v.y;
        }
        sb[q].add(sum.x, sum.y);
      }
    }
  }

  // grad_S = conj(S-bar)
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int e = tid + kNT * q;
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

BwdArgs make_args(const mbc_plan* p, const void* S_u, const void* S_d, int s_c64, const Launch& L,
                  const void* W_plan) {
  BwdArgs a;
  a.corr = p->d.corr;
  a.tiles = p->d.b_tiles;
  a.ops = p->d.b_ops;
  a.meta = p->d.b_meta;
  a.extra = p->d.b_extra;
  a.btab = p->d.btab;
  a.src_cu = p->d.src_cu;
  a.src_cd = p->d.src_cd;
  a.tabs = p->d.tabs;
  a.W = W_plan;
  a.S_u = S_u;
  a.S_d = S_d;
  a.s_c64 = s_c64;
  a.n_tiles = p->h.b_n_tiles;
  a.T = L.T;
  a.V = L.V;
  a.chunk = L.chunk;
  a.nc = L.nc;
  a.nnz = p->h.nnz;
  a.grad_C = nullptr;
  a.grad_S_u = nullptr;
  a.grad_S_d = nullptr;
  a.partial = nullptr;
  return a;
}

template <typename K>
hipError_t launch_k(K k, int nblocks, size_t lds, hipStream_t st, const BwdArgs& a) {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(nblocks), dim3(kNT), lds, st, a);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_dw_r(const mbc_plan* p, const BwdArgs& a, int nb, size_t lds, hipStream_t st) {
  const int nu = p->h.n_u, nd = p->h.n_d, ms = p->h.maxs, qm = p->h.qmax;
  if (nu == 2 && nd == 1 && ms <= 1 && qm <= 1) return launch_k(dw_kernel<R, 2, 1, 1, 1>, nb, lds, st, a);
  if (nu == 1 && nd == 2 && ms <= 1 && qm <= 1) return launch_k(dw_kernel<R, 1, 2, 1, 1>, nb, lds, st, a);
  if (nu == 3 && nd == 3 && ms <= 4 && qm <= 1) return launch_k(dw_kernel<R, 3, 3, 4, 1>, nb, lds, st, a);
  if (nu == 5 && nd == 4 && ms <= 8 && qm <= 2) return launch_k(dw_kernel<R, 5, 4, 8, 2>, nb, lds, st, a);
  return hipErrorNotSupported;
}

template <typename R>
hipError_t launch_ds_r(const mbc_plan* p, const BwdArgs& a, int nb, size_t lds, hipStream_t st) {
  const int nu = p->h.n_u, nd = p->h.n_d, qm = p->h.qmax;
  if (nu == 2 && nd == 1 && qm <= 1) return launch_k(ds_kernel<R, 2, 1, 1>, nb, lds, st, a);
  if (nu == 1 && nd == 2 && qm <= 1) return launch_k(ds_kernel<R, 1, 2, 1>, nb, lds, st, a);
  if (nu == 3 && nd == 3 && qm <= 1) return launch_k(ds_kernel<R, 3, 3, 1>, nb, lds, st, a);
  if (nu == 5 && nd == 4 && qm <= 2) return launch_k(ds_kernel<R, 5, 4, 2>, nb, lds, st, a);
  return hipErrorNotSupported;
}

}  // namespace

Launch backward_dw_launch_shape(const PlanHost& h, int T, int64_t V) {
  Launch L;
  L.T = T;
  L.V = V;
  // whole timeslices per workgroup unless the grid would be too small
  const int64_t want = 4096;
  int64_t nc = 1;
  const int64_t base = int64_t(std::max(1, h.b_n_tiles)) * T;
  if (base < want) nc = (want + base - 1) / base;
  if (nc > V) nc = V;
  L.chunk = int((V + nc - 1) / nc);
  L.nc = int((V + L.chunk - 1) / L.chunk);
  return L;
}

hipError_t launch_backward_dw(const mbc_plan* p, const void* S_u, const void* S_d, int s_c64, const Launch& L,
                              const void* W_plan, const double* grad_C, double* partial, double* grad_W,
                              hipStream_t st) {
  if (p->h.nnz == 0) return hipSuccess;
  BwdArgs a = make_args(p, S_u, S_d, s_c64, L, W_plan);
  a.grad_C = grad_C;
  a.partial = partial;
  const int64_t nb = int64_t(p->h.b_n_tiles) * L.T * L.nc;
  if (nb > 0x7fffffff) return hipErrorInvalidValue;
  const size_t lds = size_t(p->h.b_lds_dw);
  hipError_t e = (p->h.precision == MBC_F64) ? launch_dw_r<double>(p, a, int(nb), lds, st)
                                             : launch_dw_r<float>(p, a, int(nb), lds, st);
  if (e != hipSuccess) return e;
  const int rb = int((p->h.nnz + 255) / 256);
  hipLaunchKernelGGL(dw_reduce_kernel, dim3(rb), dim3(256), 0, st, partial, L.T * L.nc, p->h.nnz, p->d.perm,
                     grad_W);
  return hipGetLastError();
}

hipError_t launch_backward_ds(const mbc_plan* p, const void* S_u, const void* S_d, int s_c64, int T, int64_t V,
                              const void* W_plan, const double* grad_C, void* grad_S_u, void* grad_S_d,
                              hipStream_t st) {
  Launch L;
  L.T = T;
  L.V = V;
  BwdArgs a = make_args(p, S_u, S_d, s_c64, L, W_plan);
  a.grad_C = grad_C;
  a.grad_S_u = grad_S_u;
  a.grad_S_d = grad_S_d;
  const int64_t nb = int64_t(T) * V;
  if (nb > 0x7fffffff) return hipErrorInvalidValue;
  const size_t lds = size_t(p->h.b_lds_ds);
  if (p->h.precision == MBC_F64) return launch_ds_r<double>(p, a, int(nb), lds, st);
  return launch_ds_r<float>(p, a, int(nb), lds, st);
}

}  // namespace mbc
