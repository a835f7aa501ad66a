// Hadron blocks (Sec. 2) and block-level correlators (Sec. 3) on gfx950.
//
// Block kernel.  For one block type (family, Gamma, momentum) the block is
//
//   f_alpha(A, Y, C) = sum_x e^{-i p.x} sum_c ( S1[4c+alpha][A] B_x[c][C][Y] - S1[4c+alpha][C] B_x[c][A][Y] ),
//   B_x[c][X][Y]     = sum_{a,b} eps_abc sum_{beta,gamma} Gamma_{beta gamma} S1[4a+beta][X] S2[4b+gamma][Y],
//
// (S1 the propagator of the doubly occurring flavour q1, S2 that of q2, both
// at site x): the two pairings of the like quarks, with the baryon's colour
// and spin contracted into B first.  Both terms are entries of one matrix
//
//   G[(alpha, A)][(C, Y)] = sum_{x, c} S1[4c+alpha][A] * (e^{-i p.x} B_x[c][C][Y]),
//
// a 48 x 144 complex product summed over K = 3 x sites, and
// f_alpha(A, Y, C) = G[(alpha, A)][(C, Y)] - G[(alpha, C)][(A, Y)].  One
// workgroup accumulates G over a chunk of sites of one timeslice in
// registers: 256 threads, each a 3 x 9 tile (rows i + 16m, columns j + 16k),
// fed per colour by 3 + 9 LDS loads for 27 complex multiply-adds.  The site's
// two propagators are staged in LDS (the next site's prefetched into
// registers meanwhile) and B is built in LDS with the phase folded in.  A
// second kernel sums the chunks in a fixed order and antisymmetrises.
//
// Contraction kernel.  Each workgroup sums a chunk of one correlator's terms
// (weight times the product of its block factors, gathered from the
// timeslice's blocks) in a fixed per-thread order and a fixed tree; a last
// kernel adds the chunks of each correlator in order.
#include "device_common.hpp"
#include "kernels.hpp"

namespace mbc {

namespace {

using dev::cmac;
using dev::cmul;

constexpr int kBT = 256;          // threads per workgroup of the block kernels
constexpr int kBlockEntries = 6912;  // 4 x 12 x 12 x 12 per block type and timeslice

__device__ __forceinline__ double2 load_c(const double2* p, int64_t i) { return p[i]; }
__device__ __forceinline__ double2 load_c(const float2* p, int64_t i) {
  const float2 v = p[i];
  return make_double2(double(v.x), double(v.y));
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }

struct BlockGArgs {
  const void* S_u;
  const void* S_d;
  const BlockTypeDev* types;
  double2* partial;  // [n_types][T][nch][48][144]
  int64_t V, chunk;
  int T, nch;
  int L1, L2, L3;
};

// e^{-i p.x} at site v: p.x = 2 pi k / (L1 L2 L3) with k reduced exactly in
// integers before the (correctly scaled) sincospi.
__device__ __forceinline__ double2 site_phase(const BlockTypeDev& bt, int64_t v, int L1, int L2, int L3) {
  const int64_t x1 = v % L1, x2 = (v / L1) % L2, x3 = v / (int64_t(L1) * L2);
  const int64_t n1 = ((int64_t(bt.mom[0]) * x1) % L1 + L1) % L1;
  const int64_t n2 = ((int64_t(bt.mom[1]) * x2) % L2 + L2) % L2;
  const int64_t n3 = ((int64_t(bt.mom[2]) * x3) % L3 + L3) % L3;
  const int64_t vt = int64_t(L1) * L2 * L3;
  const int64_t k = (n1 * L2 * L3 + n2 * L1 * L3 + n3 * L1 * L2) % vt;
  double s, c;
  sincospi(2.0 * double(k) / double(vt), &s, &c);
  return make_double2(c, -s);
}

template <typename SIN>
__global__ __launch_bounds__(kBT) void block_g_kernel(BlockGArgs a) {
  __shared__ double2 sS1[144], sS2[144], sB[432];
  const int ch = blockIdx.x, t = blockIdx.y, ty = blockIdx.z;
  const BlockTypeDev& bt = a.types[ty];
  const SIN* S1 = reinterpret_cast<const SIN*>(bt.family == MBC_FAMILY_P ? a.S_u : a.S_d);
  const SIN* S2 = reinterpret_cast<const SIN*>(bt.family == MBC_FAMILY_P ? a.S_d : a.S_u);
  const int tid = threadIdx.x;
  const int i = tid >> 4, j = tid & 15;
  const int64_t v0 = int64_t(ch) * a.chunk;
  const int64_t v1 = v0 + a.chunk < a.V ? v0 + a.chunk : a.V;
  const int64_t site0 = int64_t(t) * a.V;

  double2 acc[3][9];
#pragma unroll
  for (int m = 0; m < 3; ++m)
#pragma unroll
    for (int k = 0; k < 9; ++k) acc[m][k] = make_double2(0.0, 0.0);

  // the 288 entries of a site: thread tid holds entry tid (S1 for tid < 144,
  // else S2) and, for tid < 32, S2 entry tid + 112
  double2 p0 = make_double2(0.0, 0.0), p1 = make_double2(0.0, 0.0);
  auto fetch = [&](int64_t v) {
    const int64_t s = (site0 + v) * 144;
    p0 = tid < 144 ? load_c(S1, s + tid) : load_c(S2, s + tid - 144);
    if (tid < 32) p1 = load_c(S2, s + tid + 112);
  };
  if (v0 < v1) fetch(v0);

  for (int64_t v = v0; v < v1; ++v) {
    if (tid < 144)
      sS1[tid] = p0;
    else
      sS2[tid - 144] = p0;
    if (tid < 32) sS2[tid + 112] = p1;
    __syncthreads();
    if (v + 1 < v1) fetch(v + 1);

    const double2 ph = site_phase(bt, v, a.L1, a.L2, a.L3);
    for (int e = tid; e < 432; e += kBT) {
      const int c = e / 144, X = (e / 12) % 12, Y = e % 12;
      double2 sum = make_double2(0.0, 0.0);
#pragma unroll
      for (int pr = 0; pr < 2; ++pr) {
        // (a, b, c) cyclic: eps = +1; anticyclic: eps = -1
        const int aa = pr == 0 ? (c + 1) % 3 : (c + 2) % 3;
        const int bb = pr == 0 ? (c + 2) % 3 : (c + 1) % 3;
        double2 part = make_double2(0.0, 0.0);
        for (int g = 0; g < bt.n_gamma; ++g) {
          const int be = bt.gidx[g] >> 2, ga = bt.gidx[g] & 3;
          const double2 prod = cmul(sS1[(4 * aa + be) * 12 + X], sS2[(4 * bb + ga) * 12 + Y]);
          part = cmac(make_double2(bt.gval[g][0], bt.gval[g][1]), prod, part);
        }
        sum = pr == 0 ? cadd(sum, part) : csub(sum, part);
      }
      sB[e] = cmul(sum, ph);
    }
    __syncthreads();

#pragma unroll
    for (int c = 0; c < 3; ++c) {
      double2 av[3], bv[9];
#pragma unroll
      for (int m = 0; m < 3; ++m) av[m] = sS1[48 * c + i + 16 * m];
#pragma unroll
      for (int k = 0; k < 9; ++k) bv[k] = sB[144 * c + j + 16 * k];
#pragma unroll
      for (int m = 0; m < 3; ++m)
#pragma unroll
        for (int k = 0; k < 9; ++k) acc[m][k] = cmac(av[m], bv[k], acc[m][k]);
    }
    __syncthreads();
  }

  double2* out = a.partial + ((int64_t(ty) * a.T + t) * a.nch + ch) * kBlockEntries;
#pragma unroll
  for (int m = 0; m < 3; ++m)
#pragma unroll
    for (int k = 0; k < 9; ++k) out[(i + 16 * m) * 144 + j + 16 * k] = acc[m][k];
}

// blocks[t][type][alpha][A][Y][C] = sum over chunks (in order) of
// G[(alpha, A)][(C, Y)] - G[(alpha, C)][(A, Y)]; exactly zero for A == C.
__global__ __launch_bounds__(kBT) void block_reduce_kernel(const double2* __restrict__ partial,
                                                           double2* __restrict__ blocks, int T, int n_types,
                                                           int nch) {
  const int t = blockIdx.x, ty = blockIdx.y;
  const double2* P = partial + (int64_t(ty) * T + t) * nch * kBlockEntries;
  double2* out = blocks + (int64_t(t) * n_types + ty) * kBlockEntries;
  for (int e = threadIdx.x; e < kBlockEntries; e += kBT) {
    const int al = e / 1728, A = (e / 144) % 12, Y = (e / 12) % 12, C = e % 12;
    double2 s = make_double2(0.0, 0.0);
    if (A != C) {
      const int g1 = (al * 12 + A) * 144 + C * 12 + Y;
      const int g2 = (al * 12 + C) * 144 + A * 12 + Y;
      for (int ch = 0; ch < nch; ++ch) s = cadd(s, csub(P[int64_t(ch) * kBlockEntries + g1],
                                                        P[int64_t(ch) * kBlockEntries + g2]));
    }
    out[e] = s;
  }
}

struct ContractArgs {
  const double2* blocks;
  const int32_t* factor;
  const double2* coef;
  const int32_t* chunks;
  double2* partial;  // [n_chunks][T]
  int n_types, T;
};

template <int NS>
__global__ __launch_bounds__(kBT) void block_contract_kernel(ContractArgs a) {
  __shared__ double2 red[kBT];
  const int ch = blockIdx.x, t = blockIdx.y, tid = threadIdx.x;
  const int b = a.chunks[3 * ch + 1], e = a.chunks[3 * ch + 2];
  const double2* bt = a.blocks + int64_t(t) * a.n_types * kBlockEntries;
  double2 sum = make_double2(0.0, 0.0);
  for (int k = b + tid; k < e; k += kBT) {
    double2 p = a.coef[k];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int f = a.factor[int64_t(k) * NS + s];
      if (f >= 0) p = cmul(p, bt[f]);
    }
    sum = cadd(sum, p);
  }
  red[tid] = sum;
  __syncthreads();
  for (int w = kBT / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] = cadd(red[tid], red[tid + w]);
    __syncthreads();
  }
  if (tid == 0) a.partial[int64_t(ch) * a.T + t] = red[0];
}

__global__ __launch_bounds__(kBT) void block_finish_kernel(const double2* __restrict__ partial,
                                                           const int32_t* __restrict__ chunks, int n_chunks, int T,
                                                           int n_corr, double2* __restrict__ C) {
  const int idx = blockIdx.x * kBT + threadIdx.x;
  if (idx >= n_corr * T) return;
  const int c = idx / T, t = idx % T;
  double2 s = make_double2(0.0, 0.0);
  for (int ch = 0; ch < n_chunks; ++ch)
    if (chunks[3 * ch] == c) s = cadd(s, partial[int64_t(ch) * T + t]);
  C[idx] = s;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

BlockLaunch block_launch_shape(const BlockPlanHost& h, int T, int64_t V) {
  BlockLaunch L;
  const int64_t per = int64_t(T) * std::max(h.n_types, 1);
  int64_t nch = (1536 + per - 1) / per;
  if (nch > V) nch = V;
  if (nch < 1) nch = 1;
  L.chunk = (V + nch - 1) / nch;
  L.nch = int((V + L.chunk - 1) / L.chunk);
  return L;
}

size_t block_workspace_bytes(const BlockPlanHost& h, int T, int64_t V) {
  const BlockLaunch L = block_launch_shape(h, T, V);
  const size_t g = align256(size_t(h.n_types) * size_t(T) * size_t(L.nch) * kBlockEntries * 16);
  const size_t c = align256(size_t(h.chunks.size() / 3) * size_t(T) * 16);
  return std::max(g, c);
}

hipError_t launch_blocks(const mbc_block_plan* p, const void* S_u, const void* S_d, int s_c64, int T,
                         const int32_t dims[3], double* blocks, void* workspace, hipStream_t st) {
  const BlockPlanHost& h = p->h;
  if (h.n_types == 0) return hipSuccess;
  const int64_t V = int64_t(dims[0]) * dims[1] * dims[2];
  const BlockLaunch L = block_launch_shape(h, T, V);
  BlockGArgs a;
  a.S_u = S_u;
  a.S_d = S_d;
  a.types = p->types;
  a.partial = static_cast<double2*>(workspace);
  a.V = V;
  a.chunk = L.chunk;
  a.T = T;
  a.nch = L.nch;
  a.L1 = dims[0];
  a.L2 = dims[1];
  a.L3 = dims[2];
  const dim3 grid(static_cast<unsigned>(L.nch), static_cast<unsigned>(T), static_cast<unsigned>(h.n_types));
  if (s_c64)
    hipLaunchKernelGGL(block_g_kernel<float2>, grid, dim3(kBT), 0, st, a);
  else
    hipLaunchKernelGGL(block_g_kernel<double2>, grid, dim3(kBT), 0, st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(block_reduce_kernel, dim3(unsigned(T), unsigned(h.n_types)), dim3(kBT), 0, st,
                     static_cast<const double2*>(workspace), reinterpret_cast<double2*>(blocks), T, h.n_types,
                     L.nch);
  return hipGetLastError();
}

hipError_t launch_block_contract(const mbc_block_plan* p, const double* blocks, int T, double* C, void* workspace,
                                 hipStream_t st) {
  const BlockPlanHost& h = p->h;
  const int n_chunks = int(h.chunks.size() / 3);
  if (n_chunks == 0) return launch_zero(C, size_t(h.n_corr) * size_t(T) * 16, st);
  ContractArgs a;
  a.blocks = reinterpret_cast<const double2*>(blocks);
  a.factor = p->factor;
  a.coef = reinterpret_cast<const double2*>(p->coef);
  a.chunks = p->chunks;
  a.partial = static_cast<double2*>(workspace);
  a.n_types = h.n_types;
  a.T = T;
  const dim3 grid(static_cast<unsigned>(n_chunks), static_cast<unsigned>(T));
  switch (h.n_slots) {
    case 1: hipLaunchKernelGGL(block_contract_kernel<1>, grid, dim3(kBT), 0, st, a); break;
    case 2: hipLaunchKernelGGL(block_contract_kernel<2>, grid, dim3(kBT), 0, st, a); break;
    case 3: hipLaunchKernelGGL(block_contract_kernel<3>, grid, dim3(kBT), 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int n_out = h.n_corr * T;
  hipLaunchKernelGGL(block_finish_kernel, dim3(unsigned((n_out + kBT - 1) / kBT)), dim3(kBT), 0, st,
                     static_cast<const double2*>(workspace), p->chunks, n_chunks, T, h.n_corr,
                     reinterpret_cast<double2*>(C));
  return hipGetLastError();
}

}  // namespace mbc
