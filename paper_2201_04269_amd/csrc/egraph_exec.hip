// Device evaluation of an extracted tensor e-graph plan (Sec. 5).
//
// Every step is a batched pairwise contraction
//   out[b][o] = coef x sum_s A[b][a(o, s)] B[b][b(o, s)]
// over the step's summed labels s, with operands addressed through one
// stride per label (a label may address several slots of an operand: a
// trace).  Steps run in plan order on one stream; each output element is
// written by one thread (or one workgroup), and the sum over the terms is
// added root by root, so results do not depend on scheduling.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <stdexcept>

#include "egraph.hpp"

namespace mbc {

namespace {

constexpr int kMaxL = 16;   // labels per side (open, summed) of one step
constexpr int kCT = 256;    // threads per workgroup

struct ContractArgs {
  const double2* A;
  const double2* B;  // nullptr: a single operand
  double2* C;
  int64_t a_bs, b_bs, c_bs;  // batch strides (complex elements)
  int64_t n_out, n_sum, total;
  int n_o, n_s;
  int ext_o[kMaxL], ext_s[kMaxL];
  int64_t sa_o[kMaxL], sb_o[kMaxL], sa_s[kMaxL], sb_s[kMaxL];
  double cre, cim;
  int accumulate;
};

__device__ __forceinline__ void operand_base(const ContractArgs& a, int64_t b, int64_t o, int64_t* ia, int64_t* ib) {
  *ia = b * a.a_bs;
  *ib = b * a.b_bs;
  for (int k = a.n_o - 1; k >= 0; --k) {
    const int64_t v = o % a.ext_o[k];
    o /= a.ext_o[k];
    *ia += v * a.sa_o[k];
    *ib += v * a.sb_o[k];
  }
}

__device__ __forceinline__ void mac(const ContractArgs& a, int64_t ia, int64_t ib, double2* acc) {
  const double2 x = a.A[ia];
  if (a.B) {
    const double2 y = a.B[ib];
    acc->x = fma(x.x, y.x, fma(-x.y, y.y, acc->x));
    acc->y = fma(x.x, y.y, fma(x.y, y.x, acc->y));
  } else {
    acc->x += x.x;
    acc->y += x.y;
  }
}

__device__ __forceinline__ void store(const ContractArgs& a, int64_t b, int64_t o, double2 acc) {
  const double vr = a.cre * acc.x - a.cim * acc.y, vi = a.cre * acc.y + a.cim * acc.x;
  double2* c = a.C + b * a.c_bs + o;
  if (a.accumulate) {
    const double2 old = *c;
    *c = make_double2(old.x + vr, old.y + vi);
  } else {
    *c = make_double2(vr, vi);
  }
}

// one thread per output element; the summed labels walked as an odometer
__global__ __launch_bounds__(kCT) void egraph_contract_kernel(ContractArgs a) {
  const int64_t idx = int64_t(blockIdx.x) * kCT + threadIdx.x;
  if (idx >= a.total) return;
  const int64_t b = idx / a.n_out, o = idx - b * a.n_out;
  double2 acc = make_double2(0, 0);
  if (a.A) {
    int64_t ia, ib;
    operand_base(a, b, o, &ia, &ib);
    int cnt[kMaxL];
    for (int k = 0; k < a.n_s; ++k) cnt[k] = 0;
    for (int64_t s = 0; s < a.n_sum; ++s) {
      mac(a, ia, ib, &acc);
      for (int k = a.n_s - 1; k >= 0; --k) {
        ia += a.sa_s[k];
        ib += a.sb_s[k];
        if (++cnt[k] < a.ext_s[k]) break;
        cnt[k] = 0;
        ia -= a.sa_s[k] * a.ext_s[k];
        ib -= a.sb_s[k] * a.ext_s[k];
      }
    }
  }
  store(a, b, o, acc);
}

// one workgroup per output element (few outputs, long sums): strided partial
// sums, then a fixed-order tree in LDS
__global__ __launch_bounds__(kCT) void egraph_contract_reduce_kernel(ContractArgs a) {
  __shared__ double2 part[kCT];
  const int64_t idx = blockIdx.x;
  const int64_t b = idx / a.n_out, o = idx - b * a.n_out;
  int64_t ia0, ib0;
  operand_base(a, b, o, &ia0, &ib0);
  double2 acc = make_double2(0, 0);
  for (int64_t s = threadIdx.x; s < a.n_sum; s += kCT) {
    int64_t ia = ia0, ib = ib0, r = s;
    for (int k = a.n_s - 1; k >= 0; --k) {
      const int64_t v = r % a.ext_s[k];
      r /= a.ext_s[k];
      ia += v * a.sa_s[k];
      ib += v * a.sb_s[k];
    }
    mac(a, ia, ib, &acc);
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kCT / 2; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) {
      part[threadIdx.x].x += part[threadIdx.x + w].x;
      part[threadIdx.x].y += part[threadIdx.x + w].y;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) store(a, b, o, part[0]);
}

// Labels of one step: the out labels (in output slot order), then the summed ones.
struct StepLabels {
  std::vector<int> out_lab, out_ext, sum_lab, sum_ext;
  int index(int lab) const {
    for (size_t k = 0; k < out_lab.size(); ++k)
      if (out_lab[k] == lab) return int(k);
    for (size_t k = 0; k < sum_lab.size(); ++k)
      if (sum_lab[k] == lab) return int(out_lab.size() + k);
    return -1;
  }
};

struct Operand {
  const double2* base = nullptr;
  int64_t bs = 0;       // batch stride
  int64_t elems = 0;    // elements of one batch entry
  std::vector<std::pair<int, int64_t>> slots;  // (step label, stride)
};

// Operand for child class c whose open slot j carries the label map[j]
// (labels of the consuming step); trace labels of a leaf get fresh ids from
// *next_label and are summed.
Operand child_operand(const EGraphHost& g, int c, const std::vector<int>& map, const double* const* inputs,
                      const int64_t* batch_stride, int64_t batch, const double2* ws, std::vector<int>* traces,
                      int* next_label) {
  Operand op;
  const EClass& k = g.cls[c];
  if (k.factors.size() >= 2) {
    const Step& s = g.steps[g.step_of[c]];
    op.base = ws + batch * s.ws_off;
    op.bs = s.elems;
    op.elems = s.elems;
    int64_t st = 1;
    for (int j = k.n_open - 1; j >= 0; --j) {
      op.slots.push_back({map[j], st});
      st *= k.open_ext[j];
    }
    return op;
  }
  const Fac& f = k.factors[0];
  const TensorInfo& ti = g.tensors[f.t];
  op.base = reinterpret_cast<const double2*>(inputs[f.t]);
  op.bs = batch_stride[f.t];
  int tr[MBC_EGRAPH_MAX_LABEL];
  std::fill(tr, tr + MBC_EGRAPH_MAX_LABEL, -1);
  int64_t st = 1;
  op.elems = 1;
  for (int s = ti.rank - 1; s >= 0; --s) {
    const int code = f.lab[s];
    int lab;
    if (code & 1) {
      lab = map[code >> 1];
    } else {
      if (tr[code] < 0) {
        tr[code] = (*next_label)++;
        traces->push_back(tr[code]);
      }
      lab = tr[code];
    }
    op.slots.push_back({lab, st});
    st *= ti.ext[s];
    op.elems *= ti.ext[s];
  }
  return op;
}

hipError_t launch_contract(const StepLabels& L, const Operand& A, const Operand* B, double2* C, int64_t c_bs,
                           int64_t batch, double cre, double cim, bool accumulate, hipStream_t st) {
  ContractArgs a{};
  if (L.out_lab.size() > size_t(kMaxL) || L.sum_lab.size() > size_t(kMaxL))
    throw std::domain_error("an e-graph step has more than 16 open or summed labels");
  a.A = A.base;
  a.B = B ? B->base : nullptr;
  a.C = C;
  a.a_bs = A.bs;
  a.b_bs = B ? B->bs : 0;
  a.c_bs = c_bs;
  a.n_o = int(L.out_lab.size());
  a.n_s = int(L.sum_lab.size());
  a.n_out = 1;
  a.n_sum = 1;
  for (int k = 0; k < a.n_o; ++k) {
    a.ext_o[k] = L.out_ext[k];
    a.n_out *= L.out_ext[k];
  }
  for (int k = 0; k < a.n_s; ++k) {
    a.ext_s[k] = L.sum_ext[k];
    a.n_sum *= L.sum_ext[k];
  }
  auto fill = [&](const Operand& op, int64_t* so, int64_t* ss) {
    int64_t hi = 0;
    for (const auto& sl : op.slots) {
      const int i = L.index(sl.first);
      if (i < 0) throw std::logic_error("operand slot without a step label");
      if (i < a.n_o)
        so[i] += sl.second;
      else
        ss[i - a.n_o] += sl.second;
    }
    for (int k = 0; k < a.n_o; ++k) hi += (a.ext_o[k] - 1) * so[k];
    for (int k = 0; k < a.n_s; ++k) hi += (a.ext_s[k] - 1) * ss[k];
    if (hi >= op.elems) throw std::logic_error("e-graph operand addressed out of bounds");
  };
  if (A.base) fill(A, a.sa_o, a.sa_s);
  if (B) fill(*B, a.sb_o, a.sb_s);
  a.cre = cre;
  a.cim = cim;
  a.accumulate = accumulate ? 1 : 0;
  a.total = a.n_out * batch;
  if (a.total == 0) return hipSuccess;
  if (a.n_sum >= 4096 && a.total < 16384) {
    hipLaunchKernelGGL(egraph_contract_reduce_kernel, dim3(static_cast<unsigned>(a.total)), dim3(kCT), 0, st, a);
  } else {
    const unsigned nb = static_cast<unsigned>((a.total + kCT - 1) / kCT);
    hipLaunchKernelGGL(egraph_contract_kernel, dim3(nb), dim3(kCT), 0, st, a);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t egraph_launch(const EGraphHost& g, const double* const* inputs, const int64_t* batch_stride,
                         int64_t batch, double* out, void* workspace, hipStream_t st) {
  const double2* ws = reinterpret_cast<const double2*>(workspace);
  for (const Step& s : g.steps) {
    const EClass& k = g.cls[s.cls];
    const ENode& nd = k.nodes[s.node];
    StepLabels L;
    for (int j = 0; j < k.n_open; ++j) {
      L.out_lab.push_back(2 * j + 1);
      L.out_ext.push_back(k.open_ext[j]);
    }
    for (uint8_t x : nd.o1)
      for (uint8_t y : nd.o2)
        if (x == y) {
          L.sum_lab.push_back(x);
          L.sum_ext.push_back(k.label_ext[x]);
        }
    int next_label = MBC_EGRAPH_MAX_LABEL;
    std::vector<int> traces;
    const std::vector<int> m1(nd.o1.begin(), nd.o1.end()), m2(nd.o2.begin(), nd.o2.end());
    Operand A = child_operand(g, g.rep(nd.c1), m1, inputs, batch_stride, batch, ws, &traces, &next_label);
    Operand B = child_operand(g, g.rep(nd.c2), m2, inputs, batch_stride, batch, ws, &traces, &next_label);
    for (int t : traces) {
      L.sum_lab.push_back(t);
      // the trace's extent: the extent of any slot it addresses
      int e = 0;
      for (const Operand* op : {&A, &B}) {
        const Fac* f = nullptr;
        const int c = g.rep(op == &A ? nd.c1 : nd.c2);
        if (g.cls[c].factors.size() == 1) f = &g.cls[c].factors[0];
        if (!f) continue;
        for (size_t q = 0; q < op->slots.size(); ++q)
          if (op->slots[q].first == t) e = g.tensors[f->t].ext[g.tensors[f->t].rank - 1 - int(q)];
      }
      L.sum_ext.push_back(e);
    }
    double2* C = const_cast<double2*>(ws) + batch * s.ws_off;
    const hipError_t e = launch_contract(L, A, &B, C, s.elems, batch, double(nd.sign), 0.0, false, st);
    if (e != hipSuccess) return e;
  }
  // the sum over the terms, root by root
  double2* C = reinterpret_cast<double2*>(out);
  StepLabels R;
  for (size_t j = 0; j < g.out_labels.size(); ++j) {
    R.out_lab.push_back(g.out_labels[j]);
    R.out_ext.push_back(g.out_ext[j]);
  }
  if (g.roots.empty()) {
    Operand none;
    return launch_contract(R, none, nullptr, C, g.out_elems, batch, 0.0, 0.0, false, st);
  }
  for (size_t r = 0; r < g.roots.size(); ++r) {
    const TermRoot& q = g.roots[r];
    StepLabels L = R;
    int next_label = MBC_EGRAPH_MAX_LABEL;
    std::vector<int> traces;
    const std::vector<int> map(q.opens.begin(), q.opens.end());
    Operand A = child_operand(g, q.cls, map, inputs, batch_stride, batch, ws, &traces, &next_label);
    for (int t : traces) {
      L.sum_lab.push_back(t);
      const Fac& f = g.cls[q.cls].factors[0];
      int e = 0;
      for (size_t qq = 0; qq < A.slots.size(); ++qq)
        if (A.slots[qq].first == t) e = g.tensors[f.t].ext[g.tensors[f.t].rank - 1 - int(qq)];
      L.sum_ext.push_back(e);
    }
    const hipError_t e = launch_contract(L, A, nullptr, C, g.out_elems, batch, q.re, q.im, r > 0, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace mbc
