// Device evaluation of an extracted tensor e-graph plan (Sec. 5).
//
// Every step is a batched pairwise contraction
//   out[b][o] = sign x sum_s A[b][a(o, s)] B[b][b(o, s)]
// over the step's summed labels s, with operands addressed through one
// stride per label (a label may address several slots of an operand: a
// trace).  Steps are grouped by dependency level: one launch per level runs
// all of its steps, each workgroup reading its step from a per-level map of
// workgroups to steps.  G lanes share an output element (G = 1, 4, 16, 64 or 256,
// chosen per step so that small steps still fill the chip) and add their
// partial sums in a fixed tree order; the sum over the terms is one more
// launch, again a fixed-order reduction.  Results do not depend on
// scheduling.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <stdexcept>

#include "egraph.hpp"

namespace mbc {

namespace {

constexpr int kMaxL = 16;  // labels per side (open, summed) of one step
constexpr int kCT = 256;   // threads per workgroup

// One contraction step.  src >= 0: input tensor id; -1: a workspace buffer
// (ws + batch * off, batch stride bs).
struct DevStep {
  int32_t a_src, b_src, n_o, n_s, G, pad;
  int64_t a_off, a_bs, b_off, b_bs, c_off, c_bs;
  int64_t n_out, n_sum, total;
  int64_t blk0;  // first workgroup of the step within its level
  int32_t ext_o[kMaxL], ext_s[kMaxL];
  int32_t sa_o[kMaxL], sb_o[kMaxL], sa_s[kMaxL], sb_s[kMaxL];
  double sign;
};

// One term of the final sum: coef x value of its class, open slots mapped to
// the result's labels (so), traces summed (ext_s, sa_s).
struct DevRoot {
  int32_t src, n_s;
  int64_t off, bs;
  int32_t so[kMaxL], ext_s[kMaxL], sa_s[kMaxL];
  double re, im;
};

struct Inputs {
  const double2* p[kEgraphMaxInputs];
  int64_t bs[kEgraphMaxInputs];
};

struct LevelArgs {
  const DevStep* steps;
  const uint32_t* blk_step;  // step of each workgroup of the level
  int n_steps;
  Inputs in;
  double2* ws;
  int64_t batch;
};

struct RootArgs {
  const DevRoot* roots;
  int n_roots, G, n_o;
  int ext_o[kMaxL];
  Inputs in;
  const double2* ws;
  double2* out;
  int64_t batch, out_elems, total;
};

__device__ __forceinline__ double2 cmad(double2 x, double2 y, double2 acc) {
  acc.x = fma(x.x, y.x, fma(-x.y, y.y, acc.x));
  acc.y = fma(x.x, y.y, fma(x.y, y.x, acc.y));
  return acc;
}

// fixed-order tree over the G lanes of each group (every thread takes part)
__device__ __forceinline__ double2 group_sum(double2 acc, int G, int lane, double2* part) {
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int w = G / 2; w > 0; w >>= 1) {
    if (lane < w) {
      part[threadIdx.x].x += part[threadIdx.x + w].x;
      part[threadIdx.x].y += part[threadIdx.x + w].y;
    }
    __syncthreads();
  }
  return part[threadIdx.x];
}

__global__ __launch_bounds__(kCT) void egraph_level_kernel(LevelArgs a) {
  __shared__ double2 part[kCT];
  const DevStep& s = a.steps[a.blk_step[blockIdx.x]];
  const int G = s.G;
  const int64_t gid = ((int64_t(blockIdx.x) - s.blk0) * kCT + threadIdx.x) / G;
  const int lane = int(threadIdx.x) % G;
  const bool live = gid < s.total;
  int64_t b = 0, o = 0;
  double2 acc = make_double2(0, 0);
  if (live) {
    b = gid / s.n_out;
    o = gid - b * s.n_out;
    const double2* A = s.a_src >= 0 ? a.in.p[s.a_src] : a.ws + a.batch * s.a_off;
    const double2* B = s.b_src >= 0 ? a.in.p[s.b_src] : a.ws + a.batch * s.b_off;
    int64_t ia = b * (s.a_src >= 0 ? a.in.bs[s.a_src] : s.a_bs);
    int64_t ib = b * (s.b_src >= 0 ? a.in.bs[s.b_src] : s.b_bs);
    int64_t r = o;
    for (int k = s.n_o - 1; k >= 0; --k) {
      const int64_t v = r % s.ext_o[k];
      r /= s.ext_o[k];
      ia += v * s.sa_o[k];
      ib += v * s.sb_o[k];
    }
    const int last = s.n_s - 1;
    const int E = last >= 0 ? s.ext_s[last] : 1;
    const int64_t sa = last >= 0 ? s.sa_s[last] : 0, sb = last >= 0 ? s.sb_s[last] : 0;
    const int64_t runs = s.n_sum / E;
    for (int64_t q = lane; q < runs; q += G) {
      int64_t ja = ia, jb = ib, rq = q;
      for (int k = last - 1; k >= 0; --k) {
        const int64_t v = rq % s.ext_s[k];
        rq /= s.ext_s[k];
        ja += v * s.sa_s[k];
        jb += v * s.sb_s[k];
      }
      for (int e = 0; e < E; ++e) {
        acc = cmad(A[ja], B[jb], acc);
        ja += sa;
        jb += sb;
      }
    }
  }
  if (G > 1) acc = group_sum(acc, G, lane, part);
  if (live && lane == 0) {
    double2* C = a.ws + a.batch * s.c_off + b * s.c_bs + o;
    *C = make_double2(s.sign * acc.x, s.sign * acc.y);
  }
}

__global__ __launch_bounds__(kCT) void egraph_root_kernel(RootArgs a) {
  __shared__ double2 part[kCT];
  const int G = a.G;
  const int64_t gid = (int64_t(blockIdx.x) * kCT + threadIdx.x) / G;
  const int lane = int(threadIdx.x) % G;
  const bool live = gid < a.total;
  int64_t b = 0, o = 0;
  double2 acc = make_double2(0, 0);
  if (live) {
    b = gid / a.out_elems;
    o = gid - b * a.out_elems;
    for (int r = lane; r < a.n_roots; r += G) {
      const DevRoot& q = a.roots[r];
      const double2* A = q.src >= 0 ? a.in.p[q.src] : a.ws + a.batch * q.off;
      int64_t ia = b * (q.src >= 0 ? a.in.bs[q.src] : q.bs);
      int64_t rr = o;
      for (int k = a.n_o - 1; k >= 0; --k) {
        const int64_t v = rr % a.ext_o[k];
        rr /= a.ext_o[k];
        ia += v * q.so[k];
      }
      int64_t n_tr = 1;
      for (int k = 0; k < q.n_s; ++k) n_tr *= q.ext_s[k];
      double2 v = make_double2(0, 0);
      for (int64_t t = 0; t < n_tr; ++t) {
        int64_t ja = ia, rt = t;
        for (int k = q.n_s - 1; k >= 0; --k) {
          const int64_t d = rt % q.ext_s[k];
          rt /= q.ext_s[k];
          ja += d * q.sa_s[k];
        }
        v.x += A[ja].x;
        v.y += A[ja].y;
      }
      acc = cmad(make_double2(q.re, q.im), v, acc);
    }
  }
  if (G > 1) acc = group_sum(acc, G, lane, part);
  if (live && lane == 0) a.out[b * a.out_elems + o] = acc;
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
  int src = -1;  // input tensor id, or -1: a workspace buffer
  int64_t off = 0, bs = 0, elems = 0;
  std::vector<std::pair<int, int64_t>> slots;  // (step label, stride)
  std::vector<int> trace_ext;                  // extents of the trace labels it introduced
};

// Operand for child class c whose open slot j carries the label map[j] (labels
// of the consuming step); the trace labels of a leaf get fresh ids from
// *next_label.
Operand child_operand(const EGraphHost& g, int c, const std::vector<int>& map, std::vector<int>* traces,
                      int* next_label) {
  Operand op;
  const EClass& k = g.cls[c];
  if (k.factors.size() >= 2) {
    const Step& s = g.steps[g.step_of[c]];
    op.src = -1;
    op.off = s.ws_off;
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
  op.src = f.t;
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
        op.trace_ext.push_back(ti.ext[s]);
      }
      lab = tr[code];
    }
    op.slots.push_back({lab, st});
    st *= ti.ext[s];
    op.elems *= ti.ext[s];
  }
  return op;
}

// per-label strides of an operand over the step's labels; checks that every
// address stays inside one batch entry of the operand
void strides_of(const StepLabels& L, const Operand& op, int32_t* so, int32_t* ss) {
  const int n_o = int(L.out_lab.size()), n_s = int(L.sum_lab.size());
  int64_t o64[kMaxL] = {}, s64[kMaxL] = {};
  for (const auto& sl : op.slots) {
    const int i = L.index(sl.first);
    if (i < 0) throw std::logic_error("operand slot without a step label");
    if (i < n_o)
      o64[i] += sl.second;
    else
      s64[i - n_o] += sl.second;
  }
  int64_t hi = 0;
  for (int k = 0; k < n_o; ++k) hi += (L.out_ext[k] - 1) * o64[k];
  for (int k = 0; k < n_s; ++k) hi += (L.sum_ext[k] - 1) * s64[k];
  if (hi >= op.elems || op.elems > (int64_t(1) << 31))
    throw std::logic_error("e-graph operand addressed out of bounds");
  for (int k = 0; k < n_o; ++k) so[k] = int32_t(o64[k]);
  for (int k = 0; k < n_s; ++k) ss[k] = int32_t(s64[k]);
}

// lanes per output: grow while the launch stays under 2^19 threads and every
// lane still gets a run
int lanes_for(int64_t total, int64_t runs) {
  int G = 1;
  while (G < 256 && total * G * 4 <= (int64_t(1) << 19) && int64_t(G) * 4 <= runs) G *= 4;
  return G;
}

void build_tables(const EGraphHost& g, int64_t batch, EGraphExec* x) {
  const int ns = int(g.steps.size());
  // dependency levels (children come before parents in g.steps)
  std::vector<int> level(ns, 0);
  for (int i = 0; i < ns; ++i) {
    const ENode& nd = g.cls[g.steps[i].cls].nodes[g.steps[i].node];
    for (int c : {nd.c1, nd.c2}) {
      const int k = g.step_of[g.rep(c)];
      if (k >= 0) level[i] = std::max(level[i], level[k] + 1);
    }
  }
  std::vector<int> order(ns);
  for (int i = 0; i < ns; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int p, int q) { return level[p] < level[q]; });
  std::vector<DevStep> steps(ns);
  std::vector<int> lb(1, 0);
  std::vector<unsigned> lblocks;
  std::vector<uint32_t> blk_step;  // per level, concatenated: the step (within its level) of each workgroup
  int64_t blocks = 0;
  for (int j = 0; j < ns; ++j) {
    const int i = order[j];
    if (j > 0 && level[i] != level[order[j - 1]]) {
      lb.push_back(j);
      lblocks.push_back(unsigned(blocks));
      blocks = 0;
    }
    const Step& st = g.steps[i];
    const EClass& k = g.cls[st.cls];
    const ENode& nd = k.nodes[st.node];
    StepLabels L;
    for (int o = 0; o < k.n_open; ++o) {
      L.out_lab.push_back(2 * o + 1);
      L.out_ext.push_back(k.open_ext[o]);
    }
    for (uint8_t p : nd.o1)
      for (uint8_t q : nd.o2)
        if (p == q) {
          L.sum_lab.push_back(p);
          L.sum_ext.push_back(k.label_ext[p]);
        }
    int next_label = MBC_EGRAPH_MAX_LABEL;
    std::vector<int> traces;
    const std::vector<int> m1(nd.o1.begin(), nd.o1.end()), m2(nd.o2.begin(), nd.o2.end());
    const Operand A = child_operand(g, g.rep(nd.c1), m1, &traces, &next_label);
    const Operand B = child_operand(g, g.rep(nd.c2), m2, &traces, &next_label);
    for (size_t t = 0; t < traces.size(); ++t) {
      L.sum_lab.push_back(traces[t]);
      L.sum_ext.push_back(t < A.trace_ext.size() ? A.trace_ext[t] : B.trace_ext[t - A.trace_ext.size()]);
    }
    if (L.out_lab.size() > size_t(kMaxL) || L.sum_lab.size() > size_t(kMaxL))
      throw std::domain_error("an e-graph step has more than 16 open or summed labels");
    DevStep& d = steps[j];
    d = DevStep{};
    d.a_src = A.src;
    d.b_src = B.src;
    d.a_off = A.off;
    d.a_bs = A.bs;
    d.b_off = B.off;
    d.b_bs = B.bs;
    d.c_off = st.ws_off;
    d.c_bs = st.elems;
    d.n_o = int(L.out_lab.size());
    d.n_s = int(L.sum_lab.size());
    d.n_out = 1;
    d.n_sum = 1;
    for (int q = 0; q < d.n_o; ++q) {
      d.ext_o[q] = L.out_ext[q];
      d.n_out *= L.out_ext[q];
    }
    for (int q = 0; q < d.n_s; ++q) {
      d.ext_s[q] = L.sum_ext[q];
      d.n_sum *= L.sum_ext[q];
    }
    strides_of(L, A, d.sa_o, d.sa_s);
    strides_of(L, B, d.sb_o, d.sb_s);
    d.sign = double(nd.sign);
    d.total = d.n_out * batch;
    d.G = lanes_for(d.total, d.n_s > 0 ? d.n_sum / d.ext_s[d.n_s - 1] : 1);
    d.blk0 = blocks;
    const int64_t nb = (d.total * d.G + kCT - 1) / kCT;
    blocks += nb;
    if (blocks >= (int64_t(1) << 31)) throw std::domain_error("an e-graph level needs too many workgroups");
    const uint32_t local = uint32_t(j - lb.back());
    blk_step.insert(blk_step.end(), size_t(nb), local);
  }
  if (ns > 0) {
    lb.push_back(ns);
    lblocks.push_back(unsigned(blocks));
  }
  // the terms
  std::vector<DevRoot> roots;
  StepLabels R;
  for (size_t j = 0; j < g.out_labels.size(); ++j) {
    R.out_lab.push_back(g.out_labels[j]);
    R.out_ext.push_back(g.out_ext[j]);
  }
  if (R.out_lab.size() > size_t(kMaxL)) throw std::domain_error("the result has more than 16 open labels");
  for (const TermRoot& q : g.roots) {
    StepLabels L = R;
    int next_label = MBC_EGRAPH_MAX_LABEL;
    std::vector<int> traces;
    const std::vector<int> map(q.opens.begin(), q.opens.end());
    const Operand A = child_operand(g, q.cls, map, &traces, &next_label);
    for (size_t t = 0; t < traces.size(); ++t) {
      L.sum_lab.push_back(traces[t]);
      L.sum_ext.push_back(A.trace_ext[t]);
    }
    if (L.sum_lab.size() > size_t(kMaxL)) throw std::domain_error("a term has more than 16 traces");
    DevRoot d{};
    d.src = A.src;
    d.off = A.off;
    d.bs = A.bs;
    d.n_s = int(L.sum_lab.size());
    for (int k = 0; k < d.n_s; ++k) d.ext_s[k] = L.sum_ext[k];
    strides_of(L, A, d.so, d.sa_s);
    d.re = q.re;
    d.im = q.im;
    roots.push_back(d);
  }
  const int64_t total = g.out_elems * batch;
  if (total * 256 >= (int64_t(1) << 40)) throw std::domain_error("e-graph result too large");
  egraph_exec_free(x);
  if (!steps.empty()) {
    if (hipMalloc(&x->steps, steps.size() * sizeof(DevStep)) != hipSuccess) throw std::bad_alloc();
    if (hipMemcpy(x->steps, steps.data(), steps.size() * sizeof(DevStep), hipMemcpyHostToDevice) != hipSuccess)
      throw std::runtime_error("e-graph step table upload failed");
    if (hipMalloc(&x->blk_step, blk_step.size() * sizeof(uint32_t)) != hipSuccess) throw std::bad_alloc();
    if (hipMemcpy(x->blk_step, blk_step.data(), blk_step.size() * sizeof(uint32_t), hipMemcpyHostToDevice) !=
        hipSuccess)
      throw std::runtime_error("e-graph workgroup map upload failed");
  }
  if (!roots.empty()) {
    if (hipMalloc(&x->roots, roots.size() * sizeof(DevRoot)) != hipSuccess) throw std::bad_alloc();
    if (hipMemcpy(x->roots, roots.data(), roots.size() * sizeof(DevRoot), hipMemcpyHostToDevice) != hipSuccess)
      throw std::runtime_error("e-graph root table upload failed");
  }
  x->level_begin = lb;
  x->level_blocks = lblocks;
  x->root_g = lanes_for(total, int64_t(roots.size()));
  x->root_blocks = unsigned((total * x->root_g + kCT - 1) / kCT);
  x->batch = batch;
}

}  // namespace

void egraph_exec_free(EGraphExec* x) {
  if (x->steps || x->roots || x->blk_step) (void)hipDeviceSynchronize();
  if (x->steps) (void)hipFree(x->steps);
  if (x->roots) (void)hipFree(x->roots);
  if (x->blk_step) (void)hipFree(x->blk_step);
  x->steps = x->roots = x->blk_step = nullptr;
  x->batch = -1;
}

hipError_t egraph_launch(const EGraphHost& g, EGraphExec* x, const double* const* inputs,
                         const int64_t* batch_stride, int64_t batch, double* out, void* workspace, hipStream_t st) {
  const int nt = int(g.tensors.size());
  if (nt > kEgraphMaxInputs) throw std::domain_error("the executor takes at most 64 tensors");
  if (x->batch != batch) build_tables(g, batch, x);
  Inputs in{};
  for (int t = 0; t < nt; ++t) {
    in.p[t] = reinterpret_cast<const double2*>(inputs[t]);
    in.bs[t] = batch_stride[t];
  }
  double2* ws = reinterpret_cast<double2*>(workspace);
  const DevStep* steps = reinterpret_cast<const DevStep*>(x->steps);
  const uint32_t* blk_step = reinterpret_cast<const uint32_t*>(x->blk_step);
  for (size_t l = 0; l + 1 < x->level_begin.size(); ++l) {
    LevelArgs a{};
    a.steps = steps + x->level_begin[l];
    a.blk_step = blk_step;
    blk_step += x->level_blocks[l];
    a.n_steps = x->level_begin[l + 1] - x->level_begin[l];
    a.in = in;
    a.ws = ws;
    a.batch = batch;
    hipLaunchKernelGGL(egraph_level_kernel, dim3(x->level_blocks[l]), dim3(kCT), 0, st, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  RootArgs r{};
  r.roots = reinterpret_cast<const DevRoot*>(x->roots);
  r.n_roots = int(g.roots.size());
  r.G = x->root_g;
  r.n_o = int(g.out_labels.size());
  for (int k = 0; k < r.n_o; ++k) r.ext_o[k] = g.out_ext[k];
  r.in = in;
  r.ws = ws;
  r.out = reinterpret_cast<double2*>(out);
  r.batch = batch;
  r.out_elems = g.out_elems;
  r.total = g.out_elems * batch;
  hipLaunchKernelGGL(egraph_root_kernel, dim3(x->root_blocks), dim3(kCT), 0, st, r);
  return hipGetLastError();
}

}  // namespace mbc
