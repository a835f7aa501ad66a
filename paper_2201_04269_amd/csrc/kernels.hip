// HIP kernels for gfx950 (CDNA4): forward correlator contraction, weight
// gather, and the per-timeslice FP64 reduction.
//
// Forward kernel (one workgroup = one tile of sink keys x one chunk of sites
// of one timeslice):
//   1. stage the tile's row program, per-sink-key metadata and weights W in
//      LDS once;
//   2. for each site of the chunk: load S_u(x), S_d(x) (12x12 complex each)
//      into LDS, then build the tile's compound-matrix rows level by level
//      with the Laplace expansion along the first row (every thread takes
//      (row, column-subset) work items of the level; one barrier per level);
//   3. factor-tree leaves: each thread owns source keys s and, for every sink
//      key b of the tile, accumulates L_s += W[b,s] Dd[r_d(b), c_d(s)]; at the
//      end of a run of equal u-tuples it adds Du[r_u, c_u(s)] L_s to its
//      compensated (TwoSum) accumulator;
//   4. after the chunk, a fixed-order FP64 workgroup reduction writes the
//      chunk's partial sum for the tile.
// No MFMA: the work is gathers and small-determinant recursions, not a dense
// contraction.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "device_common.hpp"
#include "kernels.hpp"

namespace mbc {

namespace {

using namespace dev;

struct FwdArgs {
  const int32_t* corr;
  const int32_t* tiles;
  const int32_t* ops;
  const int32_t* meta;
  const int32_t* src_cu;
  const int32_t* src_cd;
  const uint16_t* tabs;
  const void* W;     // plan-ordered weights, plan precision
  const void* wu;    // factored: sink and source factors of the exact weights
  const void* wv;
  const int32_t* btab;
  const void* S_u;
  const void* S_d;
  int s_c64;
  int n_tiles;
  int T;
  int64_t V;
  int chunk;
  int nc;
  double* partial;   // [n_tiles][T][nc][2]
};

// All levels of one site, one barrier after each level.  During the top
// level the next site's propagators (prefetched in registers) are stored in
// the other S buffer.
template <int K, int KMAX, int NU, int ND, int QMAX, int NT, typename C>
__device__ __forceinline__ void site_levels(const FlavTabs<NU, QMAX, NT>& tu, const FlavTabs<ND, QMAX, NT>& td,
                                            const int32_t* tr, const int4* sOps, const C* sS, C* sR,
                                            C* sSnext, const C* pre, bool have_next) {
  if constexpr (K <= KMAX) {
    if constexpr (K <= NU && (K >= 2 || NU == 1)) run_level<K>(tu, tr, 0, sOps, sS, sR);
    if constexpr (K <= ND && (K >= 2 || ND == 1)) run_level<K>(td, tr, 1, sOps, sS + 144, sR);
    if constexpr (K == KMAX) {
      if (have_next) store_site<NT>(sSnext, pre);
    }
    __syncthreads();
    site_levels<K + 1, KMAX, NU, ND, QMAX, NT, C>(tu, td, tr, sOps, sS, sR, sSnext, pre, have_next);
  }
}

// Factor-tree leaves of one site for the first NL source-key slots of the
// thread: L_s = sum over a run's keys b of W[b, s] Dd[b, s], then
// acc += Du[run, s] L_s at the end of the run (compensated).
template <int NL, int MAXS, typename R, typename C>
__device__ __forceinline__ void leaf_site(int B, const int4* meta, const C* sW, const C* sR, int n_src,
                                          const int (&sl)[MAXS], const bool (&live)[MAXS], const int (&cu)[MAXS],
                                          const int (&cd)[MAXS], CompAcc<R>& acc) {
  C L[NL];
#pragma unroll
  for (int m = 0; m < NL; ++m) L[m] = cmake<C>(0, 0);
  for (int b = 0; b < B; ++b) {
    const int4 mb = meta[b];
    const C* Wb = sW + b * n_src;
    const C* Dd = sR + mb.y;
#pragma unroll
    for (int m = 0; m < NL; ++m) L[m] = cmac(Wb[sl[m]], Dd[cd[m]], L[m]);
    if (mb.z) {
      const C* Du = sR + mb.x;
#pragma unroll
      for (int m = 0; m < NL; ++m) {
        C p = cmul(Du[cu[m]], L[m]);
        if (!live[m]) p = cmake<C>(0, 0);
        acc.add(p.x, p.y);
        L[m] = cmake<C>(0, 0);
      }
    }
  }
}

// Dispatch on the wave's number of live slots (uniform).
template <int NL, int MAXS, typename R, typename C>
__device__ __forceinline__ void leaf_dispatch(int nlive, int B, const int4* meta, const C* sW, const C* sR,
                                              int n_src, const int (&sl)[MAXS], const bool (&live)[MAXS],
                                              const int (&cu)[MAXS], const int (&cd)[MAXS], CompAcc<R>& acc) {
  if (nlive <= 0) return;
  if constexpr (NL >= MAXS) {
    leaf_site<MAXS, MAXS>(B, meta, sW, sR, n_src, sl, live, cu, cd, acc);
  } else {
    if (nlive == NL) {
      leaf_site<NL, MAXS>(B, meta, sW, sR, n_src, sl, live, cu, cd, acc);
      return;
    }
    leaf_dispatch<NL + 1, MAXS>(nlive, B, meta, sW, sR, n_src, sl, live, cu, cd, acc);
  }
}

// Factored leaves (W[b, s] = u[b] v[s]): thread t owns top d column t and
// the source keys s of that column (list entries s | c_u(s) << 11, padded with
// the zero weight at slot n_src).  Per key b of a run it accumulates
// L += u[b] Dd_b[t]; at the run's end it adds L * H to its compensated
// accumulator, H = sum over its source keys of v[s] Du[c_u(s)].
template <int MC, typename C>
__device__ __forceinline__ C fact_group(int nw, const int (&e)[MC], const C* sV, const C* du) {
  C h = cmake<C>(0, 0);
#pragma unroll
  for (int m0 = 0; m0 < MC; m0 += 2)
    if (m0 < nw) {
#pragma unroll
      for (int m = m0; m < m0 + 2 && m < MC; ++m) h = cmac(sV[e[m] & 2047], du[e[m] >> 11], h);
    }
  return h;
}

template <typename R, int NU, int ND, int MAXS, int QMAX, int NT, bool FACT, int MC>
__global__ __launch_bounds__(NT, (FACT && NT >= 512 && sizeof(R) == 4) ? 4 : 1) void fwd_kernel(FwdArgs a) {
  using C = typename cx<R>::T;
  constexpr int KMIN = (NU == 1 || ND == 1) ? 1 : 2;
  constexpr int KMAX = NU > ND ? NU : ND;
  // With both flavours' top level above 2, the first level of the next site
  // writes no slot the leaves read, so the leaves need no closing barrier.
  constexpr bool kOverlapLeaves = (NU >= 3 && ND >= 3);
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x;
  const int vt = rotated_lane<NT>();
  const int lin = xcd_linear(blockIdx.x, gridDim.x);
  const int tile = lin % a.n_tiles;
  const int tc = lin / a.n_tiles;  // t * nc + chunk
  const int32_t* tr = a.tiles + tile * kTileInts;
  const int corr = tr[0], B = tr[1], w_off = tr[2], op0 = tr[3], nops = tr[4];
  const int meta0 = tr[5], row_units = tr[6];
  const int32_t* cr = a.corr + corr * kCorrInts;
  const int n_src = cr[0], src_off = cr[1];

  C* sS0 = reinterpret_cast<C*>(smem);
  C* sW = sS0 + 576;  // W (B x n_src), or FACT: v (n_src), a zero, u (B)
  C* sR = sW + (FACT ? n_src + 1 + B : B * n_src);
  int4* sOps = lds_align16<int4>(smem, sR + row_units);
  int4* meta = sOps + nops;  // (u slot, d slot, run end (bit 0), key) of each sink key

  for (int i = tid; i < nops; i += NT) {
    const int32_t* op = a.ops + int64_t(op0 + i) * kOpInts;
    sOps[i] = make_int4(op[2], op[3], op[4], 0);
  }
  if constexpr (FACT) {
    stage_lds<NT>(sW, reinterpret_cast<const C*>(a.wv) + src_off, n_src);
    if (tid == 0) sW[n_src] = cmake<C>(0, 0);
    if (tid < B) sW[n_src + 1 + tid] = reinterpret_cast<const C*>(a.wu)[cr[32] + tr[16] + tid];
  } else {
    stage_lds<NT>(sW, reinterpret_cast<const C*>(a.W) + w_off, B * n_src);
  }
  if (tid < B) meta[tid] = reinterpret_cast<const int4*>(a.meta)[meta0 + tid];

  FlavTabs<NU, QMAX, NT> tu;
  FlavTabs<ND, QMAX, NT> td;
  tu.load(cr, 0, a.tabs);
  td.load(cr, 1, a.tabs);

  // source keys s = vt + NT m (vt: rotated lane); lanes past the last key read key n_src - 1
  // and drop their products; the wave runs the slots its first lane has
  constexpr int NS = FACT ? 1 : MAXS;
  int cu[NS], cd[NS], sl[NS];
  bool live[NS];
  int nlive = 0;
  // FACT: the thread's top d column and its source-key list
  constexpr int NE = FACT ? MC : 1;
  int le[NE];
  int lnw = 0, dcol = 0;
  bool dlive = false;
  if constexpr (FACT) {
    const int ncd = cr[8 + 2 * (6 + ND - 1)];
    dlive = vt < ncd;
    dcol = dlive ? vt : 0;
    const int32_t* lists = a.btab + cr[65];
    int n = 0, q0 = 0;
    if (dlive) {
      q0 = lists[vt];
      n = lists[vt + 1] - q0;
    }
#pragma unroll
    for (int m = 0; m < NE; ++m) {
      int v = n_src;  // the zero weight
      if (m < n) {
        const int s = lists[q0 + m];
        v = s | (a.src_cu[src_off + s] << 11);
      }
      le[m] = v;
    }
    for (int off = 32; off > 0; off >>= 1) n = max(n, __shfl_xor(n, off));
    lnw = __builtin_amdgcn_readfirstlane(n);
    nlive = (vt & ~63) < ncd ? 1 : 0;  // wave has a live column
  } else {
#pragma unroll
    for (int m = 0; m < NS; ++m) {
      const int s = vt + NT * m;
      live[m] = s < n_src;
      sl[m] = live[m] ? s : n_src - 1;
      cu[m] = a.src_cu[src_off + sl[m]];
      cd[m] = a.src_cd[src_off + sl[m]];
    }
    nlive = (n_src - (vt & ~63) + NT - 1) / NT;  // > 0 unless the wave has no key
  }

  const int t = tc / a.nc, ch = tc % a.nc;
  const int64_t v0 = int64_t(ch) * a.chunk;
  const int64_t v1 = (v0 + a.chunk < a.V) ? v0 + a.chunk : a.V;
  CompAcc<R> acc;

  // propagators of site v: thread i holds entries i and i + NT (< 288)
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
    site_levels<KMIN, KMAX, NU, ND, QMAX, NT, C>(tu, td, tr, sOps, sS, sR, sSn, pre, have_next);
    if constexpr (FACT) {
      if (nlive) {
        const C* sU = sW + n_src + 1;
        C L = cmake<C>(0, 0);
        for (int b = 0; b < B; ++b) {
          const int4 mb = meta[b];
          L = cmac(sU[b], sR[mb.y + dcol], L);
          if (mb.z & 1) {
            C p = cmul(L, fact_group<NE>(lnw, le, sW, sR + mb.x));
            if (!dlive) p = cmake<C>(0, 0);
            acc.add(p.x, p.y);
            L = cmake<C>(0, 0);
          }
        }
      }
    } else {
      leaf_dispatch<1, MAXS>(nlive, B, meta, sW, sR, n_src, sl, live, cu, cd, acc);
    }
    if constexpr (!kOverlapLeaves) __syncthreads();
  }

  // fixed-order FP64 reduction over the workgroup
  double rx = double(acc.hx) + double(acc.lx);
  double ry = double(acc.hy) + double(acc.ly);
  for (int off = 32; off > 0; off >>= 1) {
    rx += __shfl_xor(rx, off);
    ry += __shfl_xor(ry, off);
  }
  __syncthreads();
  double* red = reinterpret_cast<double*>(smem);
  const int wave = tid >> 6, lane = tid & 63;
  if (lane == 0) {
    red[2 * wave] = rx;
    red[2 * wave + 1] = ry;
  }
  __syncthreads();
  if (tid == 0) {
    double sx = 0, sy = 0;
    for (int w = 0; w < NT / 64; ++w) {
      sx += red[2 * w];
      sy += red[2 * w + 1];
    }
    double* out = a.partial + 2 * ((int64_t(tile) * a.T + t) * a.nc + ch);
    out[0] = sx;
    out[1] = sy;
  }
}

template <typename R>
__global__ void gather_w_kernel(const double2* __restrict__ Wu, const int64_t* __restrict__ perm,
                                typename cx<R>::T* __restrict__ Wp, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) {
    const double2 v = Wu[perm[i]];
    typename cx<R>::T r;
    r.x = R(v.x);
    r.y = R(v.y);
    Wp[i] = r;
  }
}

// One workgroup per (correlator, timeslice): strided per-thread compensated
// sums in a fixed order, then a fixed-order tree.
// range: index of the correlator record's (first tile, end tile) pair of the
// tiling the forward ran on.
__global__ __launch_bounds__(256) void reduce_kernel(const int32_t* __restrict__ corr, int T, int nc, int range,
                                                     const double* __restrict__ partial,
                                                     double* __restrict__ C) {
  const int c = blockIdx.x / T, t = blockIdx.x % T;
  const int32_t* cr = corr + c * kCorrInts;
  const int tb = cr[range], te = cr[range + 1];
  const int64_t n = int64_t(te - tb) * nc;
  CompAcc<double> acc;
  for (int64_t j = threadIdx.x; j < n; j += 256) {
    const int64_t tile = tb + j / nc, ch = j % nc;
    const double* p = partial + 2 * ((tile * T + t) * nc + ch);
    acc.add(p[0], p[1]);
  }
  __shared__ double sx[256], sy[256];
  sx[threadIdx.x] = acc.hx + acc.lx;
  sy[threadIdx.x] = acc.hy + acc.ly;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (int(threadIdx.x) < s) {
      sx[threadIdx.x] += sx[threadIdx.x + s];
      sy[threadIdx.x] += sy[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    C[2 * (int64_t(c) * T + t)] = sx[0];
    C[2 * (int64_t(c) * T + t) + 1] = sy[0];
  }
}

// Source-key slots per thread (MAXS) and columns per thread (QMAX) the
// forward kernel is instantiated with, per operator family; 0 if none.
constexpr int fwd_maxs(int nu, int nd) {
  return (nu == 2 && nd == 1) || (nu == 1 && nd == 2) ? 1 : ((nu == 3 && nd == 3) || (nu == 5 && nd == 4) ? 4 : 0);
}
constexpr int fwd_qmax(int nu, int nd) { return fwd_maxs(nu, nd) ? 1 : 0; }

template <typename R, int NU, int ND, int MAXS, int QMAX>
hipError_t launch_fwd_t(const mbc_plan* p, const FwdArgs& a, int nblocks, size_t lds, bool fact, hipStream_t st) {
  static_assert(MAXS == fwd_maxs(NU, ND) && QMAX == fwd_qmax(NU, ND), "instantiation table");
  constexpr int NT = family_threads(NU, ND);
  constexpr int MC = top_list_max(NU, ND);
  if ((p->h.max_ncol + NT - 1) / NT > QMAX) return hipErrorNotSupported;
  if (fact ? !p->h.fwd_fact : (p->h.max_src + NT - 1) / NT > MAXS) return hipErrorNotSupported;
  auto k = fact ? fwd_kernel<R, NU, ND, MAXS, QMAX, NT, true, MC> : fwd_kernel<R, NU, ND, MAXS, QMAX, NT, false, MC>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(nblocks), dim3(NT), lds, st, a);
  return hipGetLastError();
}

// Instantiated shapes: proton (2,1), neutron (1,2), dinucleon (3,3), 3He (5,4).
template <typename R>
hipError_t launch_fwd_r(const mbc_plan* p, const FwdArgs& a, int nblocks, size_t lds, bool fact, hipStream_t st) {
  const int nu = p->h.n_u, nd = p->h.n_d;
  if (nu == 2 && nd == 1) return launch_fwd_t<R, 2, 1, 1, 1>(p, a, nblocks, lds, fact, st);
  if (nu == 1 && nd == 2) return launch_fwd_t<R, 1, 2, 1, 1>(p, a, nblocks, lds, fact, st);
  if (nu == 3 && nd == 3) return launch_fwd_t<R, 3, 3, 4, 1>(p, a, nblocks, lds, fact, st);
  if (nu == 5 && nd == 4) return launch_fwd_t<R, 5, 4, 4, 1>(p, a, nblocks, lds, fact, st);
  return hipErrorNotSupported;
}

}  // namespace

bool forward_supports(const PlanHost& h, std::string* why) {
  const int maxs = fwd_maxs(h.n_u, h.n_d), qmax = fwd_qmax(h.n_u, h.n_d);
  const int nt = family_threads(h.n_u, h.n_d);
  if (maxs == 0) {
    *why = "no forward kernel for (n_u, n_d) = (" + std::to_string(h.n_u) + ", " + std::to_string(h.n_d) + ")";
    return false;
  }
  if ((h.max_src + nt - 1) / nt > maxs) {
    *why = "a correlator has " + std::to_string(h.max_src) + " source keys, more than the forward kernel's " +
           std::to_string(maxs * nt);
    return false;
  }
  if ((h.max_ncol + nt - 1) / nt > qmax) {
    *why = "a level has " + std::to_string(h.max_ncol) + " columns, more than the kernels' " + std::to_string(qmax * nt);
    return false;
  }
  return true;
}

Launch forward_launch_shape(const PlanHost& h, int T, int64_t V, bool fact) {
  Launch L;
  L.T = T;
  L.V = V;
  // about 32k workgroups over the grid, at least 1 site each (shorter
  // workgroups even out the tail: 3He forward per timeslice 439 -> 432 ms
  // against 16k, D_I 45.2 -> 43.9 ms)
  const double target = 32768.0;
  const double total = double(T) * double(V) * std::max(1, fact ? h.f_n_tiles : h.n_tiles);
  int64_t chunk = int64_t(total / target);
  if (chunk < 1) chunk = 1;
  if (chunk > V) chunk = V;
  L.chunk = int(chunk);
  L.nc = int((V + chunk - 1) / chunk);
  return L;
}

hipError_t launch_gather_w(const mbc_plan* p, const double* W_user, void* W_plan, hipStream_t st) {
  const int64_t n = p->h.nnz;
  if (n == 0) return hipSuccess;
  const int nb = int((n + 255) / 256);
  if (p->h.precision == MBC_F64)
    hipLaunchKernelGGL(gather_w_kernel<double>, dim3(nb), dim3(256), 0, st,
                       reinterpret_cast<const double2*>(W_user), p->d.perm,
                       reinterpret_cast<double2*>(W_plan), n);
  else
    hipLaunchKernelGGL(gather_w_kernel<float>, dim3(nb), dim3(256), 0, st,
                       reinterpret_cast<const double2*>(W_user), p->d.perm,
                       reinterpret_cast<float2*>(W_plan), n);
  return hipGetLastError();
}

hipError_t launch_forward(const mbc_plan* p, const void* S_u, const void* S_d, int s_c64,
                          const Launch& L, const void* W_plan, double* partial, bool fact, hipStream_t st) {
  const int n_tiles = fact ? p->h.f_n_tiles : p->h.n_tiles;
  if (n_tiles == 0) return hipSuccess;
  FwdArgs a;
  a.corr = p->d.corr;
  a.tiles = fact ? p->d.f_tiles : p->d.tiles;
  a.ops = fact ? p->d.f_ops : p->d.ops;
  a.meta = fact ? p->d.f_meta : p->d.meta;
  a.wu = p->d.wu;
  a.wv = p->d.wv;
  a.btab = p->d.btab;
  a.src_cu = p->d.src_cu;
  a.src_cd = p->d.src_cd;
  a.tabs = p->d.tabs;
  a.W = W_plan;
  a.S_u = S_u;
  a.S_d = S_d;
  a.s_c64 = s_c64;
  a.n_tiles = n_tiles;
  a.T = L.T;
  a.V = L.V;
  a.chunk = L.chunk;
  a.nc = L.nc;
  a.partial = partial;
  const int64_t nb = int64_t(n_tiles) * L.T * L.nc;
  if (nb > 0x7fffffff) return hipErrorInvalidValue;
  const size_t lds = size_t(fact ? p->h.f_lds_fwd : p->h.lds_bytes);
  if (p->h.precision == MBC_F64) return launch_fwd_r<double>(p, a, int(nb), lds, fact, st);
  return launch_fwd_r<float>(p, a, int(nb), lds, fact, st);
}

hipError_t launch_reduce(const mbc_plan* p, const Launch& L, const double* partial, double* C, bool fact,
                         hipStream_t st) {
  const int nb = p->h.n_corr * L.T;
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(reduce_kernel, dim3(nb), dim3(256), 0, st, p->d.corr, L.T, L.nc, fact ? 33 : 3, partial, C);
  return hipGetLastError();
}

namespace {
__global__ void zero_kernel(unsigned long long* p, size_t n) {
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x) p[i] = 0;
}
}  // namespace

// Fixed device scratch for mbc_contract_noalloc: one copy per GPU, held
// until the process ends.  In host code the array's name is not a device
// address; scratch_device_ptr() looks the address up once per device with
// hipGetSymbolAddress (with that device current) and caches it.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

hipError_t scratch_device_ptr(void** out) {
  constexpr int kMaxDevices = 64;
  static void* ptrs[kMaxDevices] = {};
  static std::mutex mu;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (ptrs[dev] == nullptr) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    ptrs[dev] = ptr;
  }
  *out = ptrs[dev];
  return hipSuccess;
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t st) {
  const size_t n = bytes / 8;
  if (n == 0) return hipSuccess;
  const size_t nb = std::min<size_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(zero_kernel, dim3(unsigned(nb)), dim3(256), 0, st, static_cast<unsigned long long*>(p), n);
  return hipGetLastError();
}

}  // namespace mbc
