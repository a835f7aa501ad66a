// HIP kernels of the adjoint (backward) contraction for gfx950.
//
// dW kernel (one workgroup = one tile of sink keys x the sites of one
// timeslice chunk): rebuilds the tile's determinant rows per site exactly as
// the forward kernel does, and accumulates Q[b,s] = sum_x Du Dd per index
// entry (C is linear in W, eq. 1) in compensated accumulators in LDS; the
// chunk's grad_C[t] conj(Q) is written in FP64 and the chunks are summed in
// a fixed order by dw_reduce_kernel.
//
// The dS kernel is in ds_kernel.hpp; this unit instantiates it for every
// family and precision except the factored FP32-comp (5, 4) kernel, which
// kernels_ds_5_4.hip instantiates with its own scheduling.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "device_common.hpp"
#include "ds_kernel.hpp"
#include "kernels.hpp"

namespace mbc {

namespace {

using namespace dev;

// Rows of one site for one tile with the next site's propagators stored
// during the top level: one barrier per level.
template <int K, int KMAX, int NU, int ND, int QMAX, int NT, typename C>
__device__ __forceinline__ void site_levels_pf(const FlavTabs<NU, QMAX, NT>& tu, const FlavTabs<ND, QMAX, NT>& td,
                                               const int32_t* tr, const int4* sOps, const C* sS, C* sR, C* sSnext,
                                               const C* pre, bool have_next) {
  if constexpr (K <= KMAX) {
    if constexpr (K <= NU && (K >= 2 || NU == 1)) run_level<K>(tu, tr, 0, sOps, sS, sR);
    if constexpr (K <= ND && (K >= 2 || ND == 1)) run_level<K>(td, tr, 1, sOps, sS + 144, sR);
    if constexpr (K == KMAX) {
      if (have_next) store_site<NT>(sSnext, pre);
    }
    __syncthreads();
    site_levels_pf<K + 1, KMAX, NU, ND, QMAX, NT, C>(tu, td, tr, sOps, sS, sR, sSnext, pre, have_next);
  }
}

// ---------------------------------------------------------------------------
// dW
// ---------------------------------------------------------------------------
// Products of one site for the tile's NB sink keys and the thread's source
// slots: acc[b][m] += Du[b, s_m] Dd[b, s_m].  A wave skips the slots past its
// last source key (uniform); lanes past n_src read key n_src - 1 and are
// never written out.
template <int NB, int BW, int MAXS, typename R, typename C>
__device__ __forceinline__ void dw_products(const C* sR, const int (&us)[BW], const int (&dsl)[BW],
                                            const int (&cu)[MAXS], const int (&cd)[MAXS], int nlive,
                                            CompAcc<R> (&acc)[BW][MAXS]) {
#pragma unroll
  for (int m = 0; m < MAXS; ++m) {
    if (m < nlive) {
      C p[NB];
#pragma unroll
      for (int b = 0; b < NB; ++b) p[b] = cmul(sR[us[b] + cu[m]], sR[dsl[b] + cd[m]]);
#pragma unroll
      for (int b = 0; b < NB; ++b) acc[b][m].add(p[b].x, p[b].y);
    }
  }
}

// dW: one workgroup per (dW tile, chunk of sites of one timeslice).  Per site
// the tile's rows are built (propagators double-buffered), then every
// (sink key, source key) product of the tile is added to its compensated
// accumulator, held in registers across the chunk; the chunk's sums,
// times grad_C, go to partial[t * nc + chunk][entry].
template <typename R, int NU, int ND, int MAXS, int QMAX, int BW, int NT>
__global__ __launch_bounds__(NT) void dw_kernel(BwdArgs a) {
  using C = typename cx<R>::T;
  constexpr int KMIN = (NU == 1 || ND == 1) ? 1 : 2;
  constexpr int KMAX = NU > ND ? NU : ND;
  constexpr bool kOverlapLeaves = (NU >= 3 && ND >= 3);
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x;
  const int vt = rotated_lane<NT>();
  const int lin = xcd_linear(blockIdx.x, gridDim.x);
  const int tile = lin % a.n_tiles;
  const int tc = lin / a.n_tiles;
  const int32_t* tr = a.tiles + tile * kTileInts;
  const int corr = tr[0], B = tr[1], w_off = tr[2], op0 = tr[3], nops = tr[4];
  const int meta0 = tr[5], row_units = tr[6];
  const int32_t* cr = a.corr + corr * kCorrInts;
  const int n_src = cr[0], src_off = cr[1];

  C* sS0 = reinterpret_cast<C*>(smem);
  C* sR = sS0 + 576;
  int4* sOps = lds_align16<int4>(smem, sR + row_units);
  for (int i = tid; i < nops; i += NT) {
    const int32_t* op = a.ops + int64_t(op0 + i) * kOpInts;
    sOps[i] = make_int4(op[2], op[3], op[4], 0);
  }
  int us[BW], dsl[BW];
#pragma unroll
  for (int b = 0; b < BW; ++b) {
    const int4 mb = reinterpret_cast<const int4*>(a.meta)[meta0 + (b < B ? b : 0)];
    us[b] = mb.x;
    dsl[b] = mb.y;
  }
  FlavTabs<NU, QMAX, NT> tu;
  FlavTabs<ND, QMAX, NT> td;
  tu.load(cr, 0, a.tabs);
  td.load(cr, 1, a.tabs);
  int cu[MAXS], cd[MAXS];
  bool live[MAXS];
#pragma unroll
  for (int m = 0; m < MAXS; ++m) {
    const int s = vt + NT * m;
    live[m] = s < n_src;
    const int sl = live[m] ? s : n_src - 1;
    cu[m] = a.src_cu[src_off + sl];
    cd[m] = a.src_cd[src_off + sl];
  }
  const int nlive = (n_src - (vt & ~63) + NT - 1) / NT;  // slots the wave runs
  CompAcc<R> acc[BW][MAXS];

  const int t = tc / a.nc, ch = tc % a.nc;
  const int64_t v0 = int64_t(ch) * a.chunk;
  const int64_t v1 = (v0 + a.chunk < a.V) ? v0 + a.chunk : a.V;
  C pre[2];
  fetch_site<NT>(a.S_u, a.S_d, a.s_c64, int64_t(t) * a.V + v0, pre);
  store_site<NT>(sS0, pre);
  __syncthreads();
  for (int64_t v = v0; v < v1; ++v) {
    const int buf = int((v - v0) & 1);
    C* sS = sS0 + 288 * buf;
    C* sSn = sS0 + 288 * (buf ^ 1);
    const bool have_next = v + 1 < v1;
    if (have_next) fetch_site<NT>(a.S_u, a.S_d, a.s_c64, int64_t(t) * a.V + v + 1, pre);
    site_levels_pf<KMIN, KMAX, NU, ND, QMAX, NT, C>(tu, td, tr, sOps, sS, sR, sSn, pre, have_next);
    // dispatch on the tile's number of sink keys (uniform; written out so
    // that the accumulators stay in registers)
    if (nlive > 0) {
#define MBC_DW_CASE(N)                                                            \
  else if (B <= (N)) dw_products<((N) < BW ? (N) : BW), BW, MAXS>(sR, us, dsl, cu, cd, nlive, acc);
      if (B <= 1) dw_products<1, BW, MAXS>(sR, us, dsl, cu, cd, nlive, acc);
      MBC_DW_CASE(2) MBC_DW_CASE(3) MBC_DW_CASE(4) MBC_DW_CASE(5) MBC_DW_CASE(6) MBC_DW_CASE(7)
      else dw_products<BW, BW, MAXS>(sR, us, dsl, cu, cd, nlive, acc);
#undef MBC_DW_CASE
    }
    if constexpr (!kOverlapLeaves) __syncthreads();
  }
  const double gx = a.grad_C[2 * (int64_t(corr) * a.T + t)], gy = a.grad_C[2 * (int64_t(corr) * a.T + t) + 1];
  double* out = a.partial + 2 * (int64_t(tc) * a.nnz + w_off);
#pragma unroll
  for (int b = 0; b < BW; ++b) {
#pragma unroll
    for (int m = 0; m < MAXS; ++m) {
      if (b < B && live[m]) {
        const int i = b * n_src + vt + NT * m;
        const double qx = double(acc[b][m].hx) + double(acc[b][m].lx);
        const double qy = -(double(acc[b][m].hy) + double(acc[b][m].ly));  // conj(Q)
        out[2 * i] = gx * qx - gy * qy;
        out[2 * i + 1] = gx * qy + gy * qx;
      }
    }
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
  a.wu = p->d.wu;
  a.wv = p->d.wv;
  return a;
}

template <typename R, int NU, int ND, int QMAX>
hipError_t launch_dw_f(const mbc_plan* p, const BwdArgs& a, int nb, size_t lds, hipStream_t st) {
  constexpr int NT = family_threads(NU, ND);
  constexpr int MS = dw_src_per_thread(NU, ND);
  constexpr int BW = dw_keys_per_tile(NU, ND, std::is_same<R, double>::value ? MBC_F64 : MBC_F32C);
  if ((p->h.max_src + NT - 1) / NT > MS || (p->h.max_ncol + NT - 1) / NT > QMAX || p->h.w_max_b > BW)
    return hipErrorNotSupported;
  return launch_k(dw_kernel<R, NU, ND, MS, QMAX, BW, NT>, NT, nb, lds, st, a);
}

template <typename R>
hipError_t launch_dw_r(const mbc_plan* p, const BwdArgs& a, int nb, size_t lds, hipStream_t st) {
  const int nu = p->h.n_u, nd = p->h.n_d;
  if (nu == 2 && nd == 1) return launch_dw_f<R, 2, 1, 1>(p, a, nb, lds, st);
  if (nu == 1 && nd == 2) return launch_dw_f<R, 1, 2, 1>(p, a, nb, lds, st);
  if (nu == 3 && nd == 3) return launch_dw_f<R, 3, 3, 1>(p, a, nb, lds, st);
  if (nu == 5 && nd == 4) return launch_dw_f<R, 5, 4, 1>(p, a, nb, lds, st);
  return hipErrorNotSupported;
}

bool bins_fit(const PlanHost& h, int nt) {
  for (int k = 1; k <= 5; ++k)
    if (h.max_bin[k] > bin_lanes(k, nt) * bin_regs(k, nt)) return false;
  return h.max_bin[6] == 0;
}

template <typename R>
hipError_t launch_ds_r(const mbc_plan* p, const BwdArgs& a, int nb, size_t lds, bool factored, hipStream_t st) {
  const int nu = p->h.n_u, nd = p->h.n_d;
  if (!bins_fit(p->h, ds_threads(nu, nd, p->h.precision))) return hipErrorNotSupported;
  // instantiated for at most MAXCOL columns per level and MC source keys per top column
  if (nu == 2 && nd == 1) return launch_ds_f<R, 2, 1, 256, 2>(p, a, nb, lds, factored, st);
  if (nu == 1 && nd == 2) return launch_ds_f<R, 1, 2, 256, 2>(p, a, nb, lds, factored, st);
  if (nu == 3 && nd == 3) return launch_ds_f<R, 3, 3, 256, 6>(p, a, nb, lds, factored, st);
  if (nu == 5 && nd == 4) {
    if constexpr (std::is_same<R, float>::value) {
      if (factored) return launch_ds_5_4_factored_f32(p, a, nb, lds, st);
      return launch_ds_one<R, 5, 4, 512, 10, false>(p, a, nb, lds, st);
    } else {
      return launch_ds_f<R, 5, 4, 512, 10>(p, a, nb, lds, factored, st);
    }
  }
  return hipErrorNotSupported;
}

}  // namespace

bool backward_supports(const PlanHost& h, std::string* why) {
  const int nu = h.n_u, nd = h.n_d;
  const bool fam = (nu == 2 && nd == 1) || (nu == 1 && nd == 2) || (nu == 3 && nd == 3) || (nu == 5 && nd == 4);
  if (!fam) {
    *why = "no backward kernels for (n_u, n_d) = (" + std::to_string(nu) + ", " + std::to_string(nd) + ")";
    return false;
  }
  // dW: source slots per thread, one column per thread, keys per tile
  const int nt = family_threads(nu, nd);
  if (h.max_src > dw_src_per_thread(nu, nd) * nt || h.max_ncol > nt ||
      h.w_max_b > dw_keys_per_tile(nu, nd, h.precision)) {
    *why = "the dW kernel is not instantiated for this plan's source keys, columns or keys per tile";
    return false;
  }
  // dS: columns per level, source keys per top column, j-list bins
  const int maxcol = nu + nd >= 8 ? 512 : 256, mc = nu + nd >= 8 ? 10 : (nu + nd >= 6 ? 6 : 2);
  if (h.max_ncol > maxcol || h.max_csr > mc || !bins_fit(h, ds_threads(nu, nd, h.precision))) {
    *why = "the dS kernel is not instantiated for this plan's columns, source-key lists or j-lists";
    return false;
  }
  return true;
}

Launch backward_dw_launch_shape(const PlanHost& h, int T, int64_t V) {
  Launch L;
  L.T = T;
  L.V = V;
  // whole timeslices per workgroup unless the grid would have fewer than
  // 32k workgroups: shorter workgroups even out the tail of the launch
  // (one 32^3 timeslice of the 3He batch: 2402 tiles x 14 chunks, 1.20 ->
  // 1.10 s; more chunks gain little and cost partial sums, nnz x 16 B each)
  const int64_t want = 32768;
  int64_t nc = 1;
  const int64_t base = int64_t(std::max(1, h.w_n_tiles)) * T;
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
  a.tiles = p->d.w_tiles;
  a.ops = p->d.w_ops;
  a.meta = p->d.w_meta;
  a.n_tiles = p->h.w_n_tiles;
  a.grad_C = grad_C;
  a.partial = partial;
  const int64_t nb = int64_t(p->h.w_n_tiles) * L.T * L.nc;
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
                              bool factored, hipStream_t st) {
  Launch L;
  L.T = T;
  L.V = V;
  BwdArgs a = make_args(p, S_u, S_d, s_c64, L, W_plan);
  a.grad_C = grad_C;
  a.grad_S_u = grad_S_u;
  a.grad_S_d = grad_S_d;
  factored = factored && p->h.rank1;
  size_t lds = size_t(p->h.b_lds_ds);
  if (factored) {
    a.tiles = p->d.f_tiles;
    a.ops = p->d.f_ops;
    a.meta = p->d.f_meta;
    a.extra = p->d.f_extra;
    a.n_tiles = p->h.f_n_tiles;
    lds = size_t(p->h.f_lds_ds);
  }
  const int64_t nb = int64_t(T) * V;
  if (nb > 0x7fffffff) return hipErrorInvalidValue;
  if (p->h.precision == MBC_F64) return launch_ds_r<double>(p, a, int(nb), lds, factored, st);
  return launch_ds_r<float>(p, a, int(nb), lds, factored, st);
}

}  // namespace mbc
