// Device helpers shared by the forward and backward kernels: complex
// arithmetic, compensated sums, propagator loads, the XCD-aware block order,
// and the Laplace-row machinery (register-resident column tables, one level
// of row operations).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "mbc_internal.hpp"

namespace mbc {
namespace dev {

// Workgroup sizes are template parameters (NT, a multiple of 64) of the
// kernels and of every helper that maps work onto the workgroup's lanes.

// Next 16-byte boundary of an LDS pointer, computed as an offset from the
// dynamic LDS base: the result stays an LDS pointer for the compiler, which a
// round trip through an integer address would lose (turning every access
// through it into a flat access).  The base is 16-byte aligned.
template <typename T>
__device__ __forceinline__ T* lds_align16(unsigned char* base, const void* p) {
  const unsigned off = unsigned(reinterpret_cast<const unsigned char*>(p) - base);
  return reinterpret_cast<T*>(base + ((off + 15u) & ~15u));
}

// Copies n elements from global memory into LDS with all NT threads of the
// workgroup, four loads in flight per thread before the stores.
template <int NT, typename T>
__device__ __forceinline__ void stage_lds(T* dst, const T* __restrict__ src, int n) {
  int i = threadIdx.x;
  for (; i + 3 * NT < n; i += 4 * NT) {
    const T v0 = src[i], v1 = src[i + NT], v2 = src[i + 2 * NT], v3 = src[i + 3 * NT];
    dst[i] = v0;
    dst[i + NT] = v1;
    dst[i + 2 * NT] = v2;
    dst[i + 3 * NT] = v3;
  }
  for (; i < n; i += NT) dst[i] = src[i];
}

template <typename R>
struct cx;
template <>
struct cx<double> {
  using T = double2;
};
template <>
struct cx<float> {
  using T = float2;
};

template <typename C>
__device__ __forceinline__ C cmake(decltype(C::x) a, decltype(C::x) b) {
  C r;
  r.x = a;
  r.y = b;
  return r;
}

// acc + a*b and acc - a*b (complex, FMA-contracted)
template <typename C>
__device__ __forceinline__ C cmac(C a, C b, C acc) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
  return acc;
}
template <typename C>
__device__ __forceinline__ C cmsub(C a, C b, C acc) {
  acc.x = fma(-a.x, b.x, acc.x);
  acc.x = fma(a.y, b.y, acc.x);
  acc.y = fma(-a.x, b.y, acc.y);
  acc.y = fma(-a.y, b.x, acc.y);
  return acc;
}
template <typename C>
__device__ __forceinline__ C cmul(C a, C b) {
  C r;
  r.x = fma(a.x, b.x, -a.y * b.y);
  r.y = fma(a.x, b.y, a.y * b.x);
  return r;
}

// Sum over the 16 lanes of each DPP row (every lane receives the row sum):
// rotations by 8, 4, 2, 1 within the row double the covered lanes each step.
__device__ __forceinline__ float row16_sum(float x) {
  x += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x128, 0xf, 0xf, false));
  x += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x124, 0xf, 0xf, false));
  x += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x122, 0xf, 0xf, false));
  x += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x121, 0xf, 0xf, false));
  return x;
}
// Sum of the two 16-lane rows of each 32-lane half of the wave, valid in the
// upper row of the half (lanes 16..31 and 48..63) once every lane holds its
// row's sum: row_bcast:15 hands lane 15 of rows 0 and 2 to rows 1 and 3
// (row mask 0b1010; the lower rows keep their own sum).
__device__ __forceinline__ float upper_row_pair_sum(float x) {
  return x + __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x142, 0xa, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
  const long long v = __builtin_bit_cast(long long, x);
  const int lo = __builtin_amdgcn_update_dpp(0, int(v & 0xffffffff), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, int(v >> 32), CTRL, 0xf, 0xf, false);
  return __builtin_bit_cast(double, (static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}
__device__ __forceinline__ double row16_sum(double x) {
  x += dpp_f64<0x128>(x);
  x += dpp_f64<0x124>(x);
  x += dpp_f64<0x122>(x);
  x += dpp_f64<0x121>(x);
  return x;
}
__device__ __forceinline__ double upper_row_pair_sum(double x) {
  const long long v = __builtin_bit_cast(long long, x);
  const int lo = __builtin_amdgcn_update_dpp(0, int(v & 0xffffffff), 0x142, 0xa, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, int(v >> 32), 0x142, 0xa, 0xf, false);
  return x + __builtin_bit_cast(double, (static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// Negates a complex value when `odd` is 1 (flips both sign bits).
__device__ __forceinline__ float2 cneg_if(float2 v, int odd) {
  const unsigned m = unsigned(odd) << 31;
  v.x = __uint_as_float(__float_as_uint(v.x) ^ m);
  v.y = __uint_as_float(__float_as_uint(v.y) ^ m);
  return v;
}
__device__ __forceinline__ double2 cneg_if(double2 v, int odd) {
  const unsigned long long m = static_cast<unsigned long long>(odd) << 63;
  v.x = __longlong_as_double(static_cast<long long>(static_cast<unsigned long long>(__double_as_longlong(v.x)) ^ m));
  v.y = __longlong_as_double(static_cast<long long>(static_cast<unsigned long long>(__double_as_longlong(v.y)) ^ m));
  return v;
}

// Knuth's TwoSum: s + e == a + b exactly (round-to-nearest, no reassociation).
template <typename R>
__device__ __forceinline__ void two_sum(R a, R b, R& s, R& e) {
  s = a + b;
  R bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// Compensated complex accumulator.
template <typename R>
struct CompAcc {
  R hx = 0, lx = 0, hy = 0, ly = 0;
  __device__ __forceinline__ void add(R x, R y) {
    R s, e;
    two_sum(hx, x, s, e);
    hx = s;
    lx += e;
    two_sum(hy, y, s, e);
    hy = s;
    ly += e;
  }
};

template <typename C>
__device__ __forceinline__ C load_site(const void* base, int c64, int64_t idx) {
  C r;
  if (c64) {
    const float2 v = reinterpret_cast<const float2*>(base)[idx];
    r.x = v.x;
    r.y = v.y;
  } else {
    const double2 v = reinterpret_cast<const double2*>(base)[idx];
    r.x = v.x;
    r.y = v.y;
  }
  return r;
}

// Propagators of one site: thread i < 288 holds entry i of the 288 (the u
// block, then the d block); with NT < 288, threads i < 288 - NT also hold
// entry NT + i.
template <int NT, typename C>
__device__ __forceinline__ void fetch_site(const void* S_u, const void* S_d, int c64, int64_t site, C* pre) {
  const int i = threadIdx.x;
  if (NT <= 288 || i < 288) pre[0] = load_site<C>(i < 144 ? S_u : S_d, c64, site * 144 + (i % 144));
  if constexpr (NT < 288)
    if (i < 288 - NT) pre[1] = load_site<C>(S_d, c64, site * 144 + (NT + i - 144));
}
template <int NT, typename C>
__device__ __forceinline__ void store_site(C* dst, const C* pre) {
  const int i = threadIdx.x;
  if (NT <= 288 || i < 288) dst[i] = pre[0];
  if constexpr (NT < 288)
    if (i < 288 - NT) dst[NT + i] = pre[1];
}

// A rotation of the workgroup's lane order by a multiple of a wave, varied
// between workgroups, so that the wave given the most work (for instance an
// extra source slot) falls on different SIMDs in co-resident workgroups.
template <int NT>
__device__ __forceinline__ int rotated_lane() {
  const int rot = int(((blockIdx.x >> 3) + (blockIdx.x >> 8)) & (NT / 64 - 1)) * 64;
  return (int(threadIdx.x) + rot) & (NT - 1);
}

// Blocks are dispatched round-robin over the 8 XCDs (block id mod 8).  Map
// them so that each XCD receives a contiguous range of logical ids, which
// keeps all tiles of a chunk of sites (same propagators) in one L2.
__device__ __forceinline__ int xcd_linear(int bid, int nb) {
  const int per = nb / 8, rem = nb % 8;
  const int xcd = bid % 8, loc = bid / 8;
  return (xcd < rem) ? xcd * (per + 1) + loc : rem * (per + 1) + (xcd - rem) * per + loc;
}

// Column-subset table entries of one (flavour, level) for the columns this
// thread owns, kept in registers for the whole tile.  With ncol <= NT the
// workgroup runs G = NT / ncol row ops of the level side by side (thread t
// takes column t % ncol of op group t / ncol); otherwise each thread takes
// columns t, t + NT, ... of one op at a time.
template <int K, int QMAX, int NT>
struct LevelTab {
  int ncol = 0, G = 1, g = 0, i0 = 0;
  int e[QMAX][K > 0 ? K : 1];

  // t: the thread's index in the workgroup's (possibly rotated) lane order
  __device__ __forceinline__ void load(const int32_t* cr, int f, const uint16_t* __restrict__ tabs, int t) {
    ncol = cr[8 + 2 * (6 * f + K - 1)];
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
      const int i = i0 + q * NT;
#pragma unroll
      for (int j = 0; j < K; ++j) e[q][j] = (i < ncol && g < G) ? int(tabs[toff + i * (K == 1 ? 1 : K) + (K == 1 ? 0 : j)]) : 0;
    }
  }
};

template <int K, typename C>
__device__ __forceinline__ C minor_entry(const int* e, const C* srow, const C* inr) {
  if constexpr (K == 1) {
    return srow[e[0]];
  } else {
    C val = cmake<C>(0, 0);
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const C x = srow[e[j] & 15];
      const C y = inr[e[j] >> 4];
      val = (j & 1) ? cmsub(x, y, val) : cmac(x, y, val);
    }
    return val;
  }
}

// One (flavour, level) phase: rows of the tile's ops [o0, o0 + nops).
// Two ops are processed per trip so that their LDS loads overlap.
template <int K, int QMAX, int NT, typename C>
__device__ __forceinline__ void level_phase(const LevelTab<K, QMAX, NT>& tb, const int4* sOps, int o0, int nops,
                                            const C* Sf, C* sR) {
  if (tb.g >= tb.G) return;
  for (int jb = tb.g; jb < nops; jb += 2 * tb.G) {
    const int j2 = jb + tb.G;
    const int4 opa = sOps[o0 + jb];
    const int4 opb = sOps[o0 + (j2 < nops ? j2 : jb)];
    const C* sa = Sf + 12 * opa.x;
    const C* sb = Sf + 12 * opb.x;
    const C* ia = (K == 2) ? (Sf + 12 * opa.y) : (sR + opa.y);
    const C* ib = (K == 2) ? (Sf + 12 * opb.y) : (sR + opb.y);
#pragma unroll
    for (int q = 0; q < QMAX; ++q) {
      const int i = tb.i0 + q * NT;
      if (i < tb.ncol) {
        const C va = minor_entry<K>(tb.e[q], sa, ia);
        const C vb = minor_entry<K>(tb.e[q], sb, ib);
        sR[opa.z + i] = va;
        if (j2 < nops) sR[opb.z + i] = vb;
      }
    }
  }
}

template <int NF, int QMAX, int NT>
struct FlavTabs {
  LevelTab<1, QMAX, NT> l1;
  LevelTab<2, QMAX, NT> l2;
  LevelTab<3, QMAX, NT> l3;
  LevelTab<4, QMAX, NT> l4;
  LevelTab<5, QMAX, NT> l5;
  LevelTab<6, QMAX, NT> l6;
  __device__ __forceinline__ void load(const int32_t* cr, int f, const uint16_t* __restrict__ tabs,
                                       int t = threadIdx.x) {
    if constexpr (NF == 1) l1.load(cr, f, tabs, t);
    if constexpr (NF >= 2) l2.load(cr, f, tabs, t);
    if constexpr (NF >= 3) l3.load(cr, f, tabs, t);
    if constexpr (NF >= 4) l4.load(cr, f, tabs, t);
    if constexpr (NF >= 5) l5.load(cr, f, tabs, t);
    if constexpr (NF >= 6) l6.load(cr, f, tabs, t);
  }
};

template <int K, int NF, int QMAX, int NT, typename C>
__device__ __forceinline__ void run_level(const FlavTabs<NF, QMAX, NT>& ft, const int32_t* tr, int f,
                                          const int4* sOps, const C* Sf, C* sR) {
  const int o0 = tr[20 + 2 * (7 * f + K)], n = tr[21 + 2 * (7 * f + K)];
  if constexpr (K == 1) level_phase<1>(ft.l1, sOps, o0, n, Sf, sR);
  if constexpr (K == 2) level_phase<2>(ft.l2, sOps, o0, n, Sf, sR);
  if constexpr (K == 3) level_phase<3>(ft.l3, sOps, o0, n, Sf, sR);
  if constexpr (K == 4) level_phase<4>(ft.l4, sOps, o0, n, Sf, sR);
  if constexpr (K == 5) level_phase<5>(ft.l5, sOps, o0, n, Sf, sR);
  if constexpr (K == 6) level_phase<6>(ft.l6, sOps, o0, n, Sf, sR);
}

}  // namespace dev
}  // namespace mbc
