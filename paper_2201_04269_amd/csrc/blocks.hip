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
constexpr int kBlockSitesPerRound = 2;  // K = 6 per site: two sites fill three 16x16x4 MFMA steps
constexpr int kTilesPerWave = 7;        // ceil(27 tiles / 4 waves)
typedef double f64x4 __attribute__((ext_vector_type(4)));

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
  const BlockTypeDev* types;  // G types
  double2* partial;           // [n_gtypes][T][nch][48][144]
  int64_t V, chunk;
  int64_t pstride;            // complex entries per source point's propagator set
  int T, nch;
  int L1, L2, L3;
  int g0;                     // first G type of this launch (blockIdx.z counts from it)
};

// e^{-i p.x} at site v of a timeslice: p.x = 2 pi k / (L1 L2 L3) with k
// reduced exactly in integers before the (correctly scaled) sincospi.
__device__ __forceinline__ double2 site_phase(const BlockTypeDev& bt, int v, int L1, int L2, int L3) {
  const int x1 = v % L1, x2 = (v / L1) % L2, x3 = v / (L1 * L2);
  const int64_t n1 = ((int64_t(bt.mom[0]) * x1) % L1 + L1) % L1;
  const int64_t n2 = ((int64_t(bt.mom[1]) * x2) % L2 + L2) % L2;
  const int64_t n3 = ((int64_t(bt.mom[2]) * x3) % L3 + L3) % L3;
  const int64_t vt = int64_t(L1) * L2 * L3;
  const int64_t k = (n1 * L2 * L3 + n2 * L1 * L3 + n3 * L1 * L2) % vt;
  double s, c;
  sincospi(2.0 * double(k) / double(vt), &s, &c);
  return make_double2(c, -s);
}

// NS sites per round: their propagators (staged in LDS, the next round's
// prefetched into registers meanwhile), B matrices and G updates share the
// round's three barriers.  (Building B for the next round while the matrix
// cores work on this one, over two LDS buffers, measured no faster.)
// MIXED: the S1 of B comes from another source point than the S1 of the
// rows (a third propagator matrix per site is staged).
template <typename SIN, int NS, bool MIXED>
__global__ __launch_bounds__(kBT, 2) void block_g_kernel(BlockGArgs a) {
  __shared__ double2 sS1[NS][144], sS2[NS][144], sS1b[MIXED ? NS : 1][144], sB[NS][432], sPh[kBlockMaxChunk];
  const int ch = blockIdx.x, t = blockIdx.y, ty = a.g0 + int(blockIdx.z);
  const BlockTypeDev& bt = a.types[ty];
  // S1 of the rows, S1 and S2 of B, each from its own source point's set
  const SIN* S1q = reinterpret_cast<const SIN*>(bt.family == MBC_FAMILY_P ? a.S_u : a.S_d);
  const SIN* S2q = reinterpret_cast<const SIN*>(bt.family == MBC_FAMILY_P ? a.S_d : a.S_u);
  const SIN* S1 = S1q + bt.pt[0] * a.pstride;
  const SIN* S1B = S1q + bt.pt[1] * a.pstride;
  const SIN* S2 = S2q + bt.pt[2] * a.pstride;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int64_t v0 = int64_t(ch) * a.chunk;
  const int64_t v1 = v0 + a.chunk < a.V ? v0 + a.chunk : a.V;
  const int64_t site0 = int64_t(t) * a.V;

  // G's 27 tiles of 16 x 16 (row block tile / 9, column block tile % 9):
  // wave w accumulates tiles w, w + 4, .., real and imaginary parts apart
  f64x4 accr[kTilesPerWave], acci[kTilesPerWave];
#pragma unroll
  for (int m = 0; m < kTilesPerWave; ++m) {
    accr[m] = f64x4{0.0, 0.0, 0.0, 0.0};
    acci[m] = f64x4{0.0, 0.0, 0.0, 0.0};
  }

  // the entries of a round (S1, S2 and, for mixed source points, the S1 of
  // B, of each site), NL per thread; sites past the chunk's end read as zero
  // (their B vanishes)
  constexpr int PER = MIXED ? 432 : 288;
  constexpr int NE = PER * NS;
  constexpr int NL = (NE + kBT - 1) / kBT;
  double2 pre[NL];
  auto fetch = [&](int64_t v) {
#pragma unroll
    for (int k = 0; k < NL; ++k) {
      const int e = tid + k * kBT;
      pre[k] = make_double2(0.0, 0.0);
      if (e < NE) {
        const int s = e / PER, r = e % PER;
        if (v + s < v1) {
          const int64_t base = (site0 + v + s) * 144;
          pre[k] = r < 144 ? load_c(S1, base + r) : (r < 288 ? load_c(S2, base + r - 144) : load_c(S1B, base + r - 288));
        }
      }
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int k = 0; k < NL; ++k) {
      const int e = tid + k * kBT;
      if (e < NE) {
        const int s = e / PER, r = e % PER;
        if (r < 144)
          sS1[s][r] = pre[k];
        else if (r < 288)
          sS2[s][r - 144] = pre[k];
        else if constexpr (MIXED)
          sS1b[s][r - 288] = pre[k];
      }
    }
  };
  // B of the round starting at site v: one thread per (site, colour c, row
  // X, four columns Y); the eight S1 entries of (c, X) serve the four columns
  auto build_b = [&](int64_t v) {
    for (int e = tid; e < 108 * NS; e += kBT) {
      const int s = e / 108, r = e % 108;
      const int c = r / 36, X = (r / 3) % 12, Y0 = 4 * (r % 3);
      // (a, b, c) cyclic (eps = +1) and anticyclic (eps = -1)
      const int a1 = c == 2 ? 0 : c + 1, b1 = c == 0 ? 2 : c - 1;
      const double2* s1b = MIXED ? sS1b[s] : sS1[s];
      double2 x1[4], x2[4];
#pragma unroll
      for (int be = 0; be < 4; ++be) {
        x1[be] = s1b[(4 * a1 + be) * 12 + X];
        x2[be] = s1b[(4 * b1 + be) * 12 + X];
      }
      const double2 ph = v + s < v1 ? sPh[v + s - v0] : make_double2(0.0, 0.0);
#pragma unroll
      for (int y = 0; y < 4; ++y) {
        double2 sum = make_double2(0.0, 0.0);
#pragma unroll
        for (int be = 0; be < 4; ++be) {
          const int ga = bt.gcol[be];
          if (ga < 0) continue;
          double2 d = cmul(x1[be], sS2[s][(4 * b1 + ga) * 12 + Y0 + y]);
          d = dev::cmsub(x2[be], sS2[s][(4 * a1 + ga) * 12 + Y0 + y], d);
          const double sg = bt.gsign[be];
          sum.x = fma(sg, d.x, sum.x);
          sum.y = fma(sg, d.y, sum.y);
        }
        sB[s][c * 144 + X * 12 + Y0 + y] = cmul(sum, ph);
      }
    }
  };
  // G += sum over the round's (site, colour) of S1 x B on the matrix cores:
  // real K index k = 6 s + 2 c + part (12 per round, three 16x16x4 steps);
  // Re G takes (a.x, -a.y) x (b.x, b.y), Im G (a.x, a.y) x (b.y, b.x).  Lane
  // l holds A[row l % 16][k l / 16] and B[k l / 16][column l % 16].
  auto accumulate_g = [&]() {
#pragma unroll
    for (int st = 0; st < 3 * NS / 2; ++st) {
      const int kk = 4 * st + (lane >> 4);
      const int s = kk / 6, c = (kk % 6) >> 1, part = kk & 1;
      double ar[3], ai[3];
#pragma unroll
      for (int rb = 0; rb < 3; ++rb) {
        const double2 av = sS1[s][48 * c + 16 * rb + (lane & 15)];
        ar[rb] = part ? -av.y : av.x;
        ai[rb] = part ? av.y : av.x;
      }
#pragma unroll
      for (int m = 0; m < kTilesPerWave; ++m) {
        const int tile = wave + 4 * m;
        if (tile < 27) {
          const double2 bv = sB[s][144 * c + 16 * (tile % 9) + (lane & 15)];
          const int rb = tile / 9;
          accr[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[rb], part ? bv.y : bv.x, accr[m], 0, 0, 0);
          acci[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[rb], part ? bv.x : bv.y, acci[m], 0, 0, 0);
        }
      }
    }
  };

  if (v0 < v1) fetch(v0);
  // the chunk's phases, once (visible after the loop's first barrier)
  for (int k = tid; k < int(v1 - v0); k += kBT) sPh[k] = site_phase(bt, int(v0) + k, a.L1, a.L2, a.L3);
  for (int64_t v = v0; v < v1; v += NS) {
    store();
    __syncthreads();
    if (v + NS < v1) fetch(v + NS);
    build_b(v);
    __syncthreads();
    accumulate_g();
    __syncthreads();
  }

  // lane l, register r of a tile's accumulator: G row 16 rb + l / 16 + 4 r,
  // column 16 cb + l % 16
  double2* out = a.partial + ((int64_t(ty) * a.T + t) * a.nch + ch) * kBlockEntries;
#pragma unroll
  for (int m = 0; m < kTilesPerWave; ++m) {
    const int tile = wave + 4 * m;
    if (tile < 27) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * (tile / 9) + (lane >> 4) + 4 * r, col = 16 * (tile % 9) + (lane & 15);
        out[row * 144 + col] = make_double2(accr[m][r], acci[m][r]);
      }
    }
  }
}

// blocks[t][type][alpha][A][Y][C] = sum over chunks (in order) of
// G1[(alpha, A)][(C, Y)] - G2[(alpha, C)][(A, Y)], with (G1, G2) the type's
// two G types (equal when its like antiquarks share a source point: then
// exactly zero for A == C).  One thread per entry: grid (entry blocks of
// kBT, T, n_types).
__global__ __launch_bounds__(kBT) void block_reduce_kernel(const double2* __restrict__ partial,
                                                           const int32_t* __restrict__ block_g,
                                                           double2* __restrict__ blocks, int T, int n_types,
                                                           int nch) {
  const int e = blockIdx.x * kBT + threadIdx.x, t = blockIdx.y, ty = blockIdx.z;
  if (e >= kBlockEntries) return;
  const double2* P1 = partial + (int64_t(block_g[2 * ty]) * T + t) * nch * kBlockEntries;
  const double2* P2 = partial + (int64_t(block_g[2 * ty + 1]) * T + t) * nch * kBlockEntries;
  const int al = e / 1728, A = (e / 144) % 12, Y = (e / 12) % 12, C = e % 12;
  double2 s = make_double2(0.0, 0.0);
  if (A != C || P1 != P2) {
    const int g1 = (al * 12 + A) * 144 + C * 12 + Y;
    const int g2 = (al * 12 + C) * 144 + A * 12 + Y;
    for (int ch = 0; ch < nch; ++ch)
      s = cadd(s, csub(P1[int64_t(ch) * kBlockEntries + g1], P2[int64_t(ch) * kBlockEntries + g2]));
  }
  blocks[(int64_t(t) * n_types + ty) * kBlockEntries + e] = s;
}

struct ContractArgs {
  const double2* blocks;
  const int32_t* factor;
  const double2* coef;
  const int32_t* chunks;
  double2* partial;  // [n_chunks][T]
  int n_types, T;
};

// Each thread reads a term (weight and factor indices) once and applies it to
// kContractT timeslices, whose blocks sit side by side in L2.
constexpr int kContractT = 8;

template <int NS>
__global__ __launch_bounds__(kBT) void block_contract_kernel(ContractArgs a) {
  __shared__ double2 red[kContractT][kBT];
  const int ch = blockIdx.x, t0 = blockIdx.y * kContractT, tid = threadIdx.x;
  const int nt = a.T - t0 < kContractT ? a.T - t0 : kContractT;
  const int b = a.chunks[3 * ch + 1], e = a.chunks[3 * ch + 2];
  const int64_t tstride = int64_t(a.n_types) * kBlockEntries;
  const double2* bt = a.blocks + int64_t(t0) * tstride;
  double2 sum[kContractT];
#pragma unroll
  for (int u = 0; u < kContractT; ++u) sum[u] = make_double2(0.0, 0.0);
  for (int k = b + tid; k < e; k += kBT) {
    const double2 w = a.coef[k];
    int f[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) f[s] = a.factor[int64_t(k) * NS + s];
#pragma unroll
    for (int u = 0; u < kContractT; ++u) {
      if (u < nt) {
        double2 p = w;
#pragma unroll
        for (int s = 0; s < NS; ++s)
          if (f[s] >= 0) p = cmul(p, bt[u * tstride + f[s]]);
        sum[u] = cadd(sum[u], p);
      }
    }
  }
#pragma unroll
  for (int u = 0; u < kContractT; ++u) red[u][tid] = sum[u];
  __syncthreads();
  for (int w = kBT / 2; w > 0; w >>= 1) {
    if (tid < w)
#pragma unroll
      for (int u = 0; u < kContractT; ++u) red[u][tid] = cadd(red[u][tid], red[u][tid + w]);
    __syncthreads();
  }
  if (tid < nt) a.partial[int64_t(ch) * a.T + t0 + tid] = red[tid][0];
}

// Factor-tree contraction (Sec. 4).  A correlator's terms are the root-to-leaf
// paths of its linearised factor tree, and its value the sum over leaf
// parents P of (the factors above P) x f(P) x sum_{leaves l of P} w_l f(l).
// Each thread takes a few runs of sibling leaves (items), forms
// each run's inner sum for the workgroup's kContractT timeslices, and
// multiplies it once by the factors of the parent and grandparent the run
// shares.
struct TreeArgs {
  const double2* blocks;
  const int32_t* factor;    // block factor of each vertex
  const double2* coef;      // leaf weights in term order
  const int32_t* items;     // [n_wg * ipt * kBT][kTreeItemInts]
  double2* partial;         // [n_wg][T]
  int n_types, T, ipt;
};

__global__ __launch_bounds__(kBT) void tree_contract_kernel(TreeArgs a) {
  __shared__ double2 red[kContractT][kBT];
  const int wg = blockIdx.x, t0 = blockIdx.y * kContractT, tid = threadIdx.x;
  const int nt = a.T - t0 < kContractT ? a.T - t0 : kContractT;
  const int64_t tstride = int64_t(a.n_types) * kBlockEntries;
  const double2* bt = a.blocks + int64_t(t0) * tstride;
  double2 tot[kContractT];
#pragma unroll
  for (int u = 0; u < kContractT; ++u) tot[u] = make_double2(0.0, 0.0);
  for (int m = 0; m < a.ipt; ++m) {
    const int32_t* it = a.items + ((int64_t(wg) * a.ipt + m) * kBT + tid) * kTreeItemInts;
    const int grand = it[0], parent = it[1], lv = it[2], nl = it[3], lb = it[4];
    double2 s[kContractT];
#pragma unroll
    for (int u = 0; u < kContractT; ++u) s[u] = make_double2(0.0, 0.0);
    for (int k = 0; k < nl; ++k) {
      const int f = a.factor[lv + k];
      const double2 w = a.coef[lb + k];
#pragma unroll
      for (int u = 0; u < kContractT; ++u)
        if (u < nt) s[u] = cmac(w, bt[u * tstride + f], s[u]);
    }
    for (const int anc : {parent, grand}) {
      if (anc < 0) continue;
      const int f = a.factor[anc];
#pragma unroll
      for (int u = 0; u < kContractT; ++u)
        if (u < nt) s[u] = cmul(bt[u * tstride + f], s[u]);
    }
#pragma unroll
    for (int u = 0; u < kContractT; ++u) tot[u] = cadd(tot[u], s[u]);
  }
#pragma unroll
  for (int u = 0; u < kContractT; ++u) red[u][tid] = tot[u];
  __syncthreads();
  for (int w = kBT / 2; w > 0; w >>= 1) {
    if (tid < w)
#pragma unroll
      for (int u = 0; u < kContractT; ++u) red[u][tid] = cadd(red[u][tid], red[u][tid + w]);
    __syncthreads();
  }
  if (tid < nt) a.partial[int64_t(wg) * a.T + t0 + tid] = red[tid][0];
}

// C[c][t] = the chunks of correlator c (consecutive, from corr_chunk[c] to
// corr_chunk[c + 1]) added in order.
__global__ __launch_bounds__(kBT) void block_finish_kernel(const double2* __restrict__ partial,
                                                           const int32_t* __restrict__ corr_chunk, int T,
                                                           int n_corr, double2* __restrict__ C) {
  const int idx = blockIdx.x * kBT + threadIdx.x;
  if (idx >= n_corr * T) return;
  const int c = idx / T, t = idx % T;
  double2 s = make_double2(0.0, 0.0);
  for (int ch = corr_chunk[c]; ch < corr_chunk[c + 1]; ++ch) s = cadd(s, partial[int64_t(ch) * T + t]);
  C[idx] = s;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

BlockLaunch block_launch_shape(const BlockPlanHost& h, int T, int64_t V) {
  BlockLaunch L;
  const int64_t per = int64_t(T) * std::max<int64_t>(int64_t(h.types.size()), 1);
  int64_t nch = (1536 + per - 1) / per;
  nch = std::max<int64_t>(nch, (V + kBlockMaxChunk - 1) / kBlockMaxChunk);
  if (nch > V) nch = V;
  if (nch < 1) nch = 1;
  L.chunk = (V + nch - 1) / nch;
  L.nch = int((V + L.chunk - 1) / L.chunk);
  return L;
}

size_t block_workspace_bytes(const BlockPlanHost& h, int T, int64_t V) {
  const BlockLaunch L = block_launch_shape(h, T, V);
  const size_t g = align256(h.types.size() * size_t(T) * size_t(L.nch) * kBlockEntries * 16);
  return std::max(g, block_contract_workspace_bytes(h, T));
}

size_t block_contract_workspace_bytes(const BlockPlanHost& h, int T) {
  const size_t c = align256(size_t(h.chunks.size() / 3) * size_t(T) * 16);
  const size_t tr = align256(size_t(h.corr_wg.empty() ? 0 : h.corr_wg.back()) * size_t(T) * 16);
  return std::max(c, tr);
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
  a.pstride = int64_t(T) * V * 144;
  a.chunk = L.chunk;
  a.T = T;
  a.nch = L.nch;
  a.L1 = dims[0];
  a.L2 = dims[1];
  a.L3 = dims[2];
  // G types with one source point first (h.n_single of them), then mixed ones
  constexpr int NS = kBlockSitesPerRound;
  for (int mixed = 0; mixed < 2; ++mixed) {
    a.g0 = mixed ? h.n_single : 0;
    const int n = mixed ? int(h.types.size()) - h.n_single : h.n_single;
    if (n == 0) continue;
    const dim3 grid(static_cast<unsigned>(L.nch), static_cast<unsigned>(T), static_cast<unsigned>(n));
    if (s_c64 && mixed)
      hipLaunchKernelGGL((block_g_kernel<float2, NS, true>), grid, dim3(kBT), 0, st, a);
    else if (s_c64)
      hipLaunchKernelGGL((block_g_kernel<float2, NS, false>), grid, dim3(kBT), 0, st, a);
    else if (mixed)
      hipLaunchKernelGGL((block_g_kernel<double2, NS, true>), grid, dim3(kBT), 0, st, a);
    else
      hipLaunchKernelGGL((block_g_kernel<double2, NS, false>), grid, dim3(kBT), 0, st, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const dim3 rgrid(static_cast<unsigned>((kBlockEntries + kBT - 1) / kBT), static_cast<unsigned>(T),
                   static_cast<unsigned>(h.n_types));
  hipLaunchKernelGGL(block_reduce_kernel, rgrid, dim3(kBT), 0, st, static_cast<const double2*>(workspace),
                     p->block_g, reinterpret_cast<double2*>(blocks), T, h.n_types, L.nch);
  return hipGetLastError();
}

hipError_t launch_block_contract(const mbc_block_plan* p, const double* blocks, int T, int method, double* C,
                                 void* workspace, hipStream_t st) {
  const BlockPlanHost& h = p->h;
  const int n_chunks = int(h.chunks.size() / 3);
  if (n_chunks == 0) return launch_zero(C, size_t(h.n_corr) * size_t(T) * 16, st);
  const int n_out = h.n_corr * T;
  if (method == MBC_BLOCK_TREE) {
    TreeArgs a;
    a.blocks = reinterpret_cast<const double2*>(blocks);
    a.factor = p->tree_factor;
    a.coef = reinterpret_cast<const double2*>(p->coef);
    a.items = p->items;
    a.partial = static_cast<double2*>(workspace);
    a.n_types = h.n_types;
    a.T = T;
    a.ipt = h.tree_ipt;
    const dim3 grid(static_cast<unsigned>(h.corr_wg.back()), static_cast<unsigned>((T + kContractT - 1) / kContractT));
    hipLaunchKernelGGL(tree_contract_kernel, grid, dim3(kBT), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(block_finish_kernel, dim3(unsigned((n_out + kBT - 1) / kBT)), dim3(kBT), 0, st,
                       static_cast<const double2*>(workspace), p->corr_wg, T, h.n_corr, reinterpret_cast<double2*>(C));
    return hipGetLastError();
  }
  ContractArgs a;
  a.blocks = reinterpret_cast<const double2*>(blocks);
  a.factor = p->factor;
  a.coef = reinterpret_cast<const double2*>(p->coef);
  a.chunks = p->chunks;
  a.partial = static_cast<double2*>(workspace);
  a.n_types = h.n_types;
  a.T = T;
  const dim3 grid(static_cast<unsigned>(n_chunks), static_cast<unsigned>((T + kContractT - 1) / kContractT));
  switch (h.n_slots) {
    case 1: hipLaunchKernelGGL(block_contract_kernel<1>, grid, dim3(kBT), 0, st, a); break;
    case 2: hipLaunchKernelGGL(block_contract_kernel<2>, grid, dim3(kBT), 0, st, a); break;
    case 3: hipLaunchKernelGGL(block_contract_kernel<3>, grid, dim3(kBT), 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(block_finish_kernel, dim3(unsigned((n_out + kBT - 1) / kBT)), dim3(kBT), 0, st,
                     static_cast<const double2*>(workspace), p->corr_chunk, T, h.n_corr,
                     reinterpret_cast<double2*>(C));
  return hipGetLastError();
}

}  // namespace mbc
