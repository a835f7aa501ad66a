// C ABI of libmbc (see include/mbc.h): argument validation, error reporting,
// plan upload and the orchestration of the device kernels.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <new>
#include <stdexcept>
#include <string>

#include "../../include/mbc_debug.h"
#include "../../include/mbc_tree.h"
#include "kernels.hpp"
#include "egraph.hpp"
#include "factor_tree.hpp"
#include "mbc_internal.hpp"

namespace mbc {

mbc_status debug_eval(const mbc_index_set* s, int precision, const double* S_u, const double* S_d, int T,
                      int64_t V, const double* W, double* C, mbc_plan_stats* stats);
mbc_status debug_backward(const mbc_index_set* s, int precision, const double* S_u, const double* S_d, int T,
                          int64_t V, const double* W, const double* grad_C, double* grad_W, double* grad_Su,
                          double* grad_Sd);

namespace {
thread_local std::string g_err;

mbc_status fail(mbc_status s, const std::string& m) {
  g_err = m;
  return s;
}

// MBC_LOG set (and not "0"): one stderr line per handle built, with its sizes
bool log_on() {
  static const bool on = [] {
    const char* v = std::getenv("MBC_LOG");
    return v && *v && std::string(v) != "0";
  }();
  return on;
}
#define MBC_LOGF(...)                                  \
  do {                                                 \
    if (log_on()) {                                    \
      std::fprintf(stderr, "[mbc] " __VA_ARGS__);      \
      std::fputc('\n', stderr);                       \
    }                                                  \
  } while (0)

mbc_status hip_fail(hipError_t e, const char* where) {
  g_err = std::string(where) + ": " + hipGetErrorString(e);
  return MBC_ERR_HIP;
}

#define MBC_HIP(call)                                 \
  do {                                                \
    hipError_t e_ = (call);                           \
    if (e_ != hipSuccess) return hip_fail(e_, #call); \
  } while (0)

template <typename F>
mbc_status guarded(F&& f) {
  try {
    return f();
  } catch (const std::bad_alloc&) {
    return fail(MBC_ERR_NOMEM, "host allocation failed");
  } catch (const std::domain_error& e) {
    return fail(MBC_ERR_UNSUPPORTED, e.what());
  } catch (const std::invalid_argument& e) {
    return fail(MBC_ERR_INVALID, e.what());
  } catch (const std::exception& e) {
    return fail(MBC_ERR_INTERNAL, e.what());
  } catch (...) {
    return fail(MBC_ERR_INTERNAL, "unknown exception");
  }
}

// True if p is device memory (or managed) accessible from the current device.
bool is_device_ptr(const void* p) {
  if (p == nullptr) return false;
  hipPointerAttribute_t attr;
  std::memset(&attr, 0, sizeof(attr));
  if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

template <typename T>
mbc_status upload(const std::vector<T>& v, T** out, hipStream_t st) {
  *out = nullptr;
  if (v.empty()) return MBC_OK;
  MBC_HIP(hipMalloc(reinterpret_cast<void**>(out), v.size() * sizeof(T)));
  MBC_HIP(hipMemcpyAsync(*out, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
  return MBC_OK;
}

void free_device(PlanDevice& d) {
  void* ptrs[] = {d.corr,    d.tiles,   d.ops,   d.meta,    d.src_cu, d.src_cd,  d.tabs,   d.perm,
                  d.w_exact, d.b_tiles, d.b_ops, d.b_meta, d.b_extra, d.btab, d.w_tiles, d.w_ops, d.w_meta,
                  d.f_tiles, d.f_ops, d.f_meta, d.f_extra, d.wu, d.wv};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  d = PlanDevice();
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct FwdWorkspace {
  size_t w_plan = 0, partial = 0, total = 0;
};

// The forward of the exact weights runs factored when the plan allows it.
bool fwd_factored(const PlanHost& h, bool user_w) { return !user_w && h.fwd_fact; }

FwdWorkspace fwd_workspace(const PlanHost& h, const Launch& L, bool user_w) {
  FwdWorkspace w;
  const size_t csz = h.precision == MBC_F64 ? 16 : 8;
  w.w_plan = user_w ? align256(size_t(h.nnz) * csz) : 0;
  const int n_tiles = fwd_factored(h, user_w) ? h.f_n_tiles : h.n_tiles;
  w.partial = align256(size_t(n_tiles) * size_t(L.T) * size_t(L.nc) * 16);
  w.total = w.w_plan + w.partial;
  return w;
}

struct BwdWorkspace {
  size_t w_plan = 0, partial = 0, total = 0;
};

BwdWorkspace bwd_workspace(const PlanHost& h, const Launch& L, bool user_w) {
  BwdWorkspace w;
  const size_t csz = h.precision == MBC_F64 ? 16 : 8;
  w.w_plan = user_w ? align256(size_t(h.nnz) * csz) : 0;
  w.partial = align256(size_t(L.T) * size_t(L.nc) * size_t(h.nnz) * 16);
  w.total = w.w_plan + w.partial;
  return w;
}

mbc_status check_inputs(const void* S_u, const void* S_d, int32_t s_dtype, int32_t T, int64_t V) {
  if (T <= 0) return fail(MBC_ERR_INVALID, "T must be positive");
  if (V <= 0) return fail(MBC_ERR_INVALID, "sites_per_t must be positive");
  if (s_dtype != MBC_C128 && s_dtype != MBC_C64) return fail(MBC_ERR_INVALID, "unknown s_dtype");
  if (!is_device_ptr(S_u) || !is_device_ptr(S_d))
    return fail(MBC_ERR_INVALID, "S_u and S_d must be device pointers");
  if (!aligned16(S_u) || !aligned16(S_d)) return fail(MBC_ERR_INVALID, "S_u/S_d must be 16-byte aligned");
  return MBC_OK;
}

mbc_status check_common(const mbc_plan* p, const void* S_u, const void* S_d, int32_t s_dtype,
                        int32_t T, int64_t V) {
  if (!p) return fail(MBC_ERR_INVALID, "plan is NULL");
  return check_inputs(S_u, S_d, s_dtype, T, V);
}

}  // namespace

void set_error(const std::string& msg) { g_err = msg; }

}  // namespace mbc

using namespace mbc;

extern "C" {

const char* mbc_last_error(void) { return g_err.c_str(); }

const char* mbc_version(void) { return "mbc 0.1 (gfx950)"; }

mbc_status mbc_build_index_set(const mbc_op_desc* ops, int32_t n_corr, mbc_index_set** out) {
  if (!ops || !out) return fail(MBC_ERR_INVALID, "NULL argument");
  if (n_corr < 1) return fail(MBC_ERR_INVALID, "n_corr must be >= 1");
  *out = nullptr;
  return guarded([&]() {
    auto* s = new mbc_index_set();
    try {
      build_index_set(ops, n_corr, &s->s);
    } catch (...) {
      delete s;
      throw;
    }
    MBC_LOGF("index set: %d correlators, n_u %d, n_d %d, %lld entries", s->s.n_corr, s->s.n_u, s->s.n_d,
             (long long)s->s.entries.size());
    *out = s;
    return MBC_OK;
  });
}

mbc_status mbc_index_set_dims(const mbc_index_set* s, int32_t* n_u, int32_t* n_d, int64_t* nnz,
                              int32_t* n_corr) {
  if (!s) return fail(MBC_ERR_INVALID, "index set is NULL");
  if (n_u) *n_u = s->s.n_u;
  if (n_d) *n_d = s->s.n_d;
  if (nnz) *nnz = int64_t(s->s.entries.size());
  if (n_corr) *n_corr = s->s.n_corr;
  return MBC_OK;
}

mbc_status mbc_index_set_export(const mbc_index_set* s, int32_t* snk_u, int32_t* src_u, int32_t* snk_d,
                                int32_t* src_d, int32_t* corr_id, int64_t* w_num_re, int64_t* w_num_im,
                                int64_t* w_den) {
  if (!s) return fail(MBC_ERR_INVALID, "index set is NULL");
  const int nu = s->s.n_u, nd = s->s.n_d;
  int64_t k = 0;
  for (const Entry& e : s->s.entries) {
    for (int i = 0; i < nu; ++i) {
      if (snk_u) snk_u[k * nu + i] = e.ru.v[i];
      if (src_u) src_u[k * nu + i] = e.cu.v[i];
    }
    for (int i = 0; i < nd; ++i) {
      if (snk_d) snk_d[k * nd + i] = e.rd.v[i];
      if (src_d) src_d[k * nd + i] = e.cd.v[i];
    }
    if (corr_id) corr_id[k] = e.corr;
    if (w_num_re) w_num_re[k] = e.w_re;
    if (w_num_im) w_num_im[k] = e.w_im;
    ++k;
  }
  if (w_den)
    for (int c = 0; c < s->s.n_corr; ++c) w_den[c] = s->s.w_den[c];
  return MBC_OK;
}

void mbc_index_set_free(mbc_index_set* s) { delete s; }

mbc_status mbc_plan_create(const mbc_index_set* s, int32_t precision, void* stream, mbc_plan** out) {
  if (!s || !out) return fail(MBC_ERR_INVALID, "NULL argument");
  if (precision != MBC_F64 && precision != MBC_F32C) return fail(MBC_ERR_INVALID, "unknown precision");
  *out = nullptr;
  return guarded([&]() -> mbc_status {
    auto* p = new mbc_plan();
    mbc_status st = MBC_OK;
    try {
      compile_plan(s->s, precision, &p->h);
    } catch (...) {
      delete p;
      throw;
    }
    std::string why;
    if (!forward_supports(p->h, &why) || !backward_supports(p->h, &why)) {
      delete p;
      return fail(MBC_ERR_UNSUPPORTED, why);
    }
    hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
    if (hipGetDevice(&p->device) != hipSuccess) {
      delete p;
      return hip_fail(hipGetLastError(), "hipGetDevice");
    }
    const PlanHost& h = p->h;
    std::vector<float> wf;
    if ((st = upload(h.corr, &p->d.corr, hs)) != MBC_OK ||
        (st = upload(h.tiles, &p->d.tiles, hs)) != MBC_OK ||
        (st = upload(h.ops, &p->d.ops, hs)) != MBC_OK || (st = upload(h.meta, &p->d.meta, hs)) != MBC_OK ||
        (st = upload(h.src_cu, &p->d.src_cu, hs)) != MBC_OK ||
        (st = upload(h.src_cd, &p->d.src_cd, hs)) != MBC_OK ||
        (st = upload(h.tabs, &p->d.tabs, hs)) != MBC_OK || (st = upload(h.perm, &p->d.perm, hs)) != MBC_OK ||
        (st = upload(h.b_tiles, &p->d.b_tiles, hs)) != MBC_OK ||
        (st = upload(h.b_ops, &p->d.b_ops, hs)) != MBC_OK || (st = upload(h.b_meta, &p->d.b_meta, hs)) != MBC_OK ||
        (st = upload(h.b_extra, &p->d.b_extra, hs)) != MBC_OK || (st = upload(h.btab, &p->d.btab, hs)) != MBC_OK ||
        (st = upload(h.w_tiles, &p->d.w_tiles, hs)) != MBC_OK || (st = upload(h.w_ops, &p->d.w_ops, hs)) != MBC_OK ||
        (st = upload(h.w_meta, &p->d.w_meta, hs)) != MBC_OK ||
        (st = upload(h.f_tiles, &p->d.f_tiles, hs)) != MBC_OK || (st = upload(h.f_ops, &p->d.f_ops, hs)) != MBC_OK ||
        (st = upload(h.f_meta, &p->d.f_meta, hs)) != MBC_OK || (st = upload(h.f_extra, &p->d.f_extra, hs)) != MBC_OK) {
      free_device(p->d);
      delete p;
      return st;
    }
    // exact weights and their sink and source factors, in the plan's precision
    std::vector<float> wuf, wvf;
    if (h.precision == MBC_F64) {
      double *w = nullptr, *u = nullptr, *v = nullptr;
      if ((st = upload(h.w_exact, &w, hs)) == MBC_OK && (st = upload(h.wu, &u, hs)) == MBC_OK)
        st = upload(h.wv, &v, hs);
      p->d.w_exact = w;
      p->d.wu = u;
      p->d.wv = v;
    } else {
      wf.assign(h.w_exact.begin(), h.w_exact.end());
      wuf.assign(h.wu.begin(), h.wu.end());
      wvf.assign(h.wv.begin(), h.wv.end());
      float *w = nullptr, *u = nullptr, *v = nullptr;
      if ((st = upload(wf, &w, hs)) == MBC_OK && (st = upload(wuf, &u, hs)) == MBC_OK) st = upload(wvf, &v, hs);
      p->d.w_exact = w;
      p->d.wu = u;
      p->d.wv = v;
    }
    hipError_t e = hipStreamSynchronize(hs);
    if (st == MBC_OK && e != hipSuccess) st = hip_fail(e, "hipStreamSynchronize");
    if (st != MBC_OK) {
      free_device(p->d);
      delete p;
      return st;
    }
    MBC_LOGF("plan: %s, %lld entries, %d/%d/%d tiles (forward/dS/dW), %d threads, %lld LDS bytes, "
             "%.3e algorithmic flops per site forward",
             p->h.precision == MBC_F64 ? "f64" : "f32c", (long long)p->h.nnz, p->h.n_tiles, p->h.b_n_tiles,
             p->h.w_n_tiles, p->h.threads, (long long)p->h.lds_bytes, p->h.alg_flops_per_site);
    *out = p;
    return MBC_OK;
  });
}

mbc_status mbc_plan_get_stats(const mbc_plan* p, mbc_plan_stats* out) {
  if (!p || !out) return fail(MBC_ERR_INVALID, "NULL argument");
  out->nnz = p->h.nnz;
  out->n_corr = p->h.n_corr;
  out->n_u = p->h.n_u;
  out->n_d = p->h.n_d;
  out->precision = p->h.precision;
  out->n_tiles = p->h.n_tiles;
  out->threads = p->h.threads;
  out->lds_bytes = p->h.lds_bytes;
  out->alg_flops_per_site = p->h.alg_flops_per_site;
  out->exec_flops_per_site = p->h.exec_flops_per_site;
  out->in_bytes_per_site = 2.0 * 144.0 * 16.0;
  out->b_n_tiles = p->h.b_n_tiles;
  out->b_lds_bytes_ds = p->h.b_lds_ds;
  out->b_lds_bytes_dw = p->h.b_lds_dw;
  out->ds_alg_flops_per_site = p->h.ds_alg_flops_per_site;
  out->dw_alg_flops_per_site = p->h.dw_alg_flops_per_site;
  out->w_n_tiles = p->h.w_n_tiles;
  out->rank1 = p->h.rank1 ? 1 : 0;
  out->f_n_tiles = p->h.f_n_tiles;
  out->f_lds_bytes_ds = p->h.f_lds_ds;
  out->fwd_factored = p->h.fwd_fact ? 1 : 0;
  out->ds_factored = (p->h.rank1 && ds_factored(p->h.n_u, p->h.n_d, p->h.precision)) ? 1 : 0;
  out->f_lds_bytes_fwd = p->h.f_lds_fwd;
  out->fact_alg_flops_per_site = p->h.fact_alg_flops_per_site;
  out->fact_ds_alg_flops_per_site = p->h.fact_ds_alg_flops_per_site;
  return MBC_OK;
}

mbc_status mbc_plan_workspace_bytes(const mbc_plan* p, int32_t T, int64_t sites_per_t, int32_t backward,
                                    size_t* bytes) {
  if (!p || !bytes) return fail(MBC_ERR_INVALID, "NULL argument");
  if (T <= 0 || sites_per_t <= 0) return fail(MBC_ERR_INVALID, "T and sites_per_t must be positive");
  if (backward) {
    const Launch L = backward_dw_launch_shape(p->h, T, sites_per_t);
    *bytes = bwd_workspace(p->h, L, true).total;
  } else {
    // enough for either weights: user W, or the plan's exact ones (factored or not)
    const Launch L = forward_launch_shape(p->h, T, sites_per_t, false);
    const Launch Lf = forward_launch_shape(p->h, T, sites_per_t, fwd_factored(p->h, false));
    *bytes = std::max(fwd_workspace(p->h, L, true).total, fwd_workspace(p->h, Lf, false).total);
  }
  return MBC_OK;
}

void mbc_plan_destroy(mbc_plan* p) {
  if (!p) return;
  (void)hipDeviceSynchronize();
  free_device(p->d);
  delete p;
}

mbc_status mbc_contract(const mbc_plan* p, const void* S_u, const void* S_d, int32_t s_dtype, int32_t T,
                        int64_t sites_per_t, const double* W, double* C, void* workspace, size_t ws_bytes,
                        void* stream) {
  mbc_status st = check_common(p, S_u, S_d, s_dtype, T, sites_per_t);
  if (st != MBC_OK) return st;
  if (!is_device_ptr(C)) return fail(MBC_ERR_INVALID, "C must be a device pointer");
  if (W && !is_device_ptr(W)) return fail(MBC_ERR_INVALID, "W must be a device pointer or NULL");
  if (W && !aligned16(W)) return fail(MBC_ERR_INVALID, "W must be 16-byte aligned");
  const bool fact = fwd_factored(p->h, W != nullptr);
  const Launch L = forward_launch_shape(p->h, T, sites_per_t, fact);
  const FwdWorkspace ws = fwd_workspace(p->h, L, W != nullptr);
  if (ws.total > 0 && (!workspace || !is_device_ptr(workspace)))
    return fail(MBC_ERR_INVALID, "workspace must be a device pointer");
  if (ws_bytes < ws.total) return fail(MBC_ERR_INVALID, "workspace too small");
  if (!aligned16(workspace)) return fail(MBC_ERR_INVALID, "workspace must be 16-byte aligned");
  hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
  int dev = -1;
  MBC_HIP(hipGetDevice(&dev));
  if (dev != p->device) return fail(MBC_ERR_INVALID, "plan was created on another device");
  char* wsb = static_cast<char*>(workspace);
  const void* W_plan = p->d.w_exact;
  if (W) {
    MBC_HIP(launch_gather_w(p, W, wsb, hs));
    W_plan = wsb;
  }
  double* partial = reinterpret_cast<double*>(wsb + ws.w_plan);
  MBC_HIP(launch_forward(p, S_u, S_d, s_dtype == MBC_C64, L, W_plan, partial, fact, hs));
  MBC_HIP(launch_reduce(p, L, partial, C, fact, hs));
  return MBC_OK;
}

mbc_status mbc_contract_noalloc(const mbc_plan* p, const void* S_u, const void* S_d, int32_t s_dtype, int32_t T,
                                int64_t sites_per_t, const double* W, double* C, void* stream) {
  mbc_status st = check_common(p, S_u, S_d, s_dtype, T, sites_per_t);
  if (st != MBC_OK) return st;
  if (!is_device_ptr(C)) return fail(MBC_ERR_INVALID, "C must be a device pointer");
  if (W && !is_device_ptr(W)) return fail(MBC_ERR_INVALID, "W must be a device pointer or NULL");
  if (W && !aligned16(W)) return fail(MBC_ERR_INVALID, "W must be 16-byte aligned");
  const bool fact = fwd_factored(p->h, W != nullptr);
  const Launch L = forward_launch_shape(p->h, T, sites_per_t, fact);
  const FwdWorkspace ws = fwd_workspace(p->h, L, W != nullptr);
  if (ws.total > kScratchBytes)
    return fail(MBC_ERR_UNSUPPORTED, "mbc_contract_noalloc needs " + std::to_string(ws.total) +
                                         " bytes of scratch, more than its fixed " + std::to_string(kScratchBytes) +
                                         " (use mbc_contract with a workspace)");
  int dev = -1;
  MBC_HIP(hipGetDevice(&dev));
  if (dev != p->device) return fail(MBC_ERR_INVALID, "plan was created on another device");
  void* scr = nullptr;
  MBC_HIP(scratch_device_ptr(&scr));
  hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
  // the scratch needs no clearing: the weight gather and the forward kernel
  // write every element they later read
  char* wsb = static_cast<char*>(scr);
  const void* W_plan = p->d.w_exact;
  if (W) {
    MBC_HIP(launch_gather_w(p, W, wsb, hs));
    W_plan = wsb;
  }
  double* partial = reinterpret_cast<double*>(wsb + ws.w_plan);
  MBC_HIP(launch_forward(p, S_u, S_d, s_dtype == MBC_C64, L, W_plan, partial, fact, hs));
  MBC_HIP(launch_reduce(p, L, partial, C, fact, hs));
  return MBC_OK;
}

mbc_status mbc_contract_backward(const mbc_plan* p, const void* S_u, const void* S_d, int32_t s_dtype,
                                 int32_t T, int64_t sites_per_t, const double* W, const double* grad_C,
                                 double* grad_W, void* grad_S_u, void* grad_S_d, void* workspace,
                                 size_t ws_bytes, void* stream) {
  mbc_status st = check_common(p, S_u, S_d, s_dtype, T, sites_per_t);
  if (st != MBC_OK) return st;
  if (!is_device_ptr(grad_C) || !aligned16(grad_C)) return fail(MBC_ERR_INVALID, "grad_C must be an aligned device pointer");
  if (W && (!is_device_ptr(W) || !aligned16(W))) return fail(MBC_ERR_INVALID, "W must be an aligned device pointer or NULL");
  if (grad_W && (!is_device_ptr(grad_W) || !aligned16(grad_W)))
    return fail(MBC_ERR_INVALID, "grad_W must be an aligned device pointer or NULL");
  for (void* g : {grad_S_u, grad_S_d})
    if (g && (!is_device_ptr(g) || !aligned16(g)))
      return fail(MBC_ERR_INVALID, "grad_S_u/grad_S_d must be aligned device pointers or NULL");
  const Launch L = backward_dw_launch_shape(p->h, T, sites_per_t);
  const BwdWorkspace ws = bwd_workspace(p->h, L, W != nullptr);
  const size_t need = (grad_W ? ws.total : ws.w_plan);
  if (need > 0 && (!workspace || !is_device_ptr(workspace)))
    return fail(MBC_ERR_INVALID, "workspace must be a device pointer");
  if (ws_bytes < need) return fail(MBC_ERR_INVALID, "workspace too small");
  if (workspace && !aligned16(workspace)) return fail(MBC_ERR_INVALID, "workspace must be 16-byte aligned");
  hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
  int dev = -1;
  MBC_HIP(hipGetDevice(&dev));
  if (dev != p->device) return fail(MBC_ERR_INVALID, "plan was created on another device");
  char* wsb = static_cast<char*>(workspace);
  const void* W_plan = p->d.w_exact;
  if (W) {
    MBC_HIP(launch_gather_w(p, W, wsb, hs));
    W_plan = wsb;
  }
  const int s_c64 = s_dtype == MBC_C64;
  if (grad_W) {
    if (p->h.nnz == 0) {
      // nothing to write
    } else {
      double* partial = reinterpret_cast<double*>(wsb + ws.w_plan);
      MBC_HIP(launch_backward_dw(p, S_u, S_d, s_c64, L, W_plan, grad_C, partial, grad_W, hs));
    }
  }
  if (grad_S_u || grad_S_d) {
    const size_t bytes = size_t(T) * size_t(sites_per_t) * 144 * (s_c64 ? 8 : 16);
    if (p->h.b_n_tiles == 0) {
      if (grad_S_u) MBC_HIP(launch_zero(grad_S_u, bytes, hs));
      if (grad_S_d) MBC_HIP(launch_zero(grad_S_d, bytes, hs));
    } else {
      // the plan's exact weights as a product of factors: the factored tiling
      const bool factored = (W == nullptr) && p->h.rank1 && ds_factored(p->h.n_u, p->h.n_d, p->h.precision);
      MBC_HIP(launch_backward_ds(p, S_u, S_d, s_c64, T, sites_per_t, W_plan, grad_C, grad_S_u, grad_S_d, factored,
                                 hs));
    }
  }
  return MBC_OK;
}

mbc_status mbc_debug_eval_host(const mbc_index_set* s, int32_t precision, const double* S_u,
                               const double* S_d, int32_t T, int64_t sites_per_t, const double* W,
                               double* C, mbc_plan_stats* stats) {
  if (!s || !S_u || !S_d || !C) return fail(MBC_ERR_INVALID, "NULL argument");
  if (T <= 0 || sites_per_t <= 0) return fail(MBC_ERR_INVALID, "T and sites_per_t must be positive");
  if (precision != MBC_F64 && precision != MBC_F32C) return fail(MBC_ERR_INVALID, "unknown precision");
  return guarded([&]() { return debug_eval(s, precision, S_u, S_d, T, sites_per_t, W, C, stats); });
}

mbc_status mbc_debug_backward_host(const mbc_index_set* s, int32_t precision, const double* S_u,
                                   const double* S_d, int32_t T, int64_t sites_per_t, const double* W,
                                   const double* grad_C, double* grad_W, double* grad_S_u,
                                   double* grad_S_d) {
  if (!s || !S_u || !S_d || !grad_C) return fail(MBC_ERR_INVALID, "NULL argument");
  if (T <= 0 || sites_per_t <= 0) return fail(MBC_ERR_INVALID, "T and sites_per_t must be positive");
  if (precision != MBC_F64 && precision != MBC_F32C) return fail(MBC_ERR_INVALID, "unknown precision");
  return guarded([&]() {
    return debug_backward(s, precision, S_u, S_d, T, sites_per_t, W, grad_C, grad_W, grad_S_u, grad_S_d);
  });
}

// ---- hadron blocks and block-level correlators (include/mbc_blocks.h) ----

mbc_status mbc_block_set_build(const mbc_block_corr_desc* corrs, int32_t n_corr, mbc_block_set** out) {
  if (!corrs || !out) return fail(MBC_ERR_INVALID, "NULL argument");
  if (n_corr < 1) return fail(MBC_ERR_INVALID, "n_corr must be >= 1");
  *out = nullptr;
  return guarded([&]() {
    auto* s = new mbc_block_set();
    try {
      build_block_set(corrs, n_corr, &s->s);
    } catch (...) {
      delete s;
      throw;
    }
    MBC_LOGF("block set: %d correlators, %d block types, %lld terms, %d source points", s->s.n_corr,
             int(s->s.types.size()), (long long)s->s.corr.size(), s->s.n_points);
    *out = s;
    return MBC_OK;
  });
}

mbc_status mbc_block_set_dims(const mbc_block_set* s, int32_t* n_corr, int32_t* n_slots, int32_t* n_types,
                              int64_t* n_terms, int32_t* n_points) {
  if (!s) return fail(MBC_ERR_INVALID, "block set is NULL");
  if (n_corr) *n_corr = s->s.n_corr;
  if (n_slots) *n_slots = s->s.n_slots;
  if (n_types) *n_types = int32_t(s->s.types.size());
  if (n_terms) *n_terms = int64_t(s->s.corr.size());
  if (n_points) *n_points = s->s.n_points;
  return MBC_OK;
}

mbc_status mbc_block_set_types(const mbc_block_set* s, int32_t* family, int32_t* projector, int32_t* mom,
                               int32_t* src) {
  if (!s) return fail(MBC_ERR_INVALID, "block set is NULL");
  for (size_t k = 0; k < s->s.types.size(); ++k) {
    const BlockType& t = s->s.types[k];
    if (family) family[k] = t.family;
    if (projector) projector[k] = t.proj;
    for (int d = 0; d < 3; ++d) {
      if (mom) mom[3 * k + d] = t.mom[d];
      if (src) src[3 * k + d] = t.src[d];
    }
  }
  return MBC_OK;
}

mbc_status mbc_block_set_export(const mbc_block_set* s, int32_t* factor, int32_t* corr_id, int64_t* num_re,
                                int64_t* num_im, int64_t* den) {
  if (!s) return fail(MBC_ERR_INVALID, "block set is NULL");
  const BlockSet& b = s->s;
  if (factor) std::copy(b.factor.begin(), b.factor.end(), factor);
  if (corr_id) std::copy(b.corr.begin(), b.corr.end(), corr_id);
  if (num_re) std::copy(b.num_re.begin(), b.num_re.end(), num_re);
  if (num_im) std::copy(b.num_im.begin(), b.num_im.end(), num_im);
  if (den) std::copy(b.den.begin(), b.den.end(), den);
  return MBC_OK;
}

mbc_status mbc_block_set_factor_tree(const mbc_block_set* s, int32_t corr, int64_t* n_vertices, int32_t* factors,
                                     int32_t* children) {
  if (!s) return fail(MBC_ERR_INVALID, "block set is NULL");
  if (corr < 0 || corr >= s->s.n_corr) return fail(MBC_ERR_INVALID, "correlator index out of range");
  const int64_t b = s->s.tree_vertex[corr], e = s->s.tree_vertex[corr + 1];
  if (n_vertices) *n_vertices = e - b;
  if (factors) std::copy(s->s.tree_factor.begin() + b, s->s.tree_factor.begin() + e, factors);
  if (children) std::copy(s->s.tree_children.begin() + b, s->s.tree_children.begin() + e, children);
  return MBC_OK;
}

void mbc_block_set_free(mbc_block_set* s) { delete s; }

mbc_status mbc_block_multiplicities(const mbc_block_corr_desc* corr, int64_t max_terms, int64_t* n_terms,
                                    int64_t* n_distinct, int64_t* max_mult, int64_t* hist, int32_t hist_len) {
  if (!corr) return fail(MBC_ERR_INVALID, "NULL argument");
  if (hist && hist_len < 1) return fail(MBC_ERR_INVALID, "hist_len must be >= 1");
  return guarded([&]() {
    int64_t nt = 0, nd = 0;
    std::vector<int64_t> hh;
    const bool done = block_multiplicities(*corr, max_terms, &nt, &nd, &hh);
    if (n_terms) *n_terms = nt;
    if (!done) return fail(MBC_ERR_UNSUPPORTED, "expansion has more than max_terms terms");
    if (n_distinct) *n_distinct = nd;
    if (max_mult) *max_mult = int64_t(hh.size()) - 1;
    if (hist)
      for (int32_t m = 0; m < hist_len; ++m) hist[m] = size_t(m) < hh.size() ? hh[m] : 0;
    return MBC_OK;
  });
}

mbc_status mbc_block_plan_create(const mbc_block_set* s, void* stream, mbc_block_plan** out) {
  if (!s || !out) return fail(MBC_ERR_INVALID, "NULL argument");
  *out = nullptr;
  return guarded([&]() -> mbc_status {
    auto* p = new mbc_block_plan();
    try {
      compile_block_plan(s->s, &p->h);
    } catch (...) {
      delete p;
      throw;
    }
    auto release = [](mbc_block_plan* q) {
      for (void* ptr : {static_cast<void*>(q->types), static_cast<void*>(q->factor), static_cast<void*>(q->coef),
                        static_cast<void*>(q->chunks), static_cast<void*>(q->corr_chunk),
                        static_cast<void*>(q->block_g),
                        static_cast<void*>(q->tree_factor), static_cast<void*>(q->items),
                        static_cast<void*>(q->corr_wg)})
        if (ptr) (void)hipFree(ptr);
      delete q;
    };
    if (hipGetDevice(&p->device) != hipSuccess) {
      delete p;
      return hip_fail(hipGetLastError(), "hipGetDevice");
    }
    hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
    mbc_status st = MBC_OK;
    if ((st = upload(p->h.types, &p->types, hs)) != MBC_OK || (st = upload(p->h.factor, &p->factor, hs)) != MBC_OK ||
        (st = upload(p->h.coef, &p->coef, hs)) != MBC_OK || (st = upload(p->h.chunks, &p->chunks, hs)) != MBC_OK ||
        (st = upload(p->h.corr_chunk, &p->corr_chunk, hs)) != MBC_OK ||
        (st = upload(p->h.block_g, &p->block_g, hs)) != MBC_OK ||
        (st = upload(p->h.tree_factor, &p->tree_factor, hs)) != MBC_OK ||
        (st = upload(p->h.items, &p->items, hs)) != MBC_OK || (st = upload(p->h.corr_wg, &p->corr_wg, hs)) != MBC_OK) {
      release(p);
      return st;
    }
    hipError_t e = hipStreamSynchronize(hs);
    if (e != hipSuccess) {
      release(p);
      return hip_fail(e, "hipStreamSynchronize");
    }
    MBC_LOGF("block plan: %d types from %d G matrices, %lld terms, %.3e flops per site", p->h.n_types,
             int(p->h.types.size()), (long long)p->h.n_terms, p->h.block_flops_per_site);
    *out = p;
    return MBC_OK;
  });
}

mbc_status mbc_block_plan_get_stats(const mbc_block_plan* p, mbc_block_plan_stats* out) {
  if (!p || !out) return fail(MBC_ERR_INVALID, "NULL argument");
  out->n_types = p->h.n_types;
  out->n_slots = p->h.n_slots;
  out->n_corr = p->h.n_corr;
  out->n_points = p->h.n_points;
  out->n_terms = p->h.n_terms;
  out->n_gmats = int32_t(p->h.types.size());
  out->block_flops_per_site = p->h.block_flops_per_site;
  out->contract_flops_per_t = p->h.contract_flops_per_t;
  out->tree_vertices = p->h.tree_vertices;
  out->tree_flops_per_t = p->h.tree_flops_per_t;
  return MBC_OK;
}

mbc_status mbc_block_workspace_bytes(const mbc_block_plan* p, int32_t T, const int32_t dims[3], size_t* bytes) {
  if (!p || !dims || !bytes) return fail(MBC_ERR_INVALID, "NULL argument");
  if (T <= 0 || dims[0] <= 0 || dims[1] <= 0 || dims[2] <= 0)
    return fail(MBC_ERR_INVALID, "T and dims must be positive");
  *bytes = block_workspace_bytes(p->h, T, int64_t(dims[0]) * dims[1] * dims[2]);
  return MBC_OK;
}

void mbc_block_plan_destroy(mbc_block_plan* p) {
  if (!p) return;
  (void)hipDeviceSynchronize();
  for (void* ptr : {static_cast<void*>(p->types), static_cast<void*>(p->factor), static_cast<void*>(p->coef),
                    static_cast<void*>(p->chunks), static_cast<void*>(p->corr_chunk),
                    static_cast<void*>(p->block_g),
                    static_cast<void*>(p->tree_factor), static_cast<void*>(p->items),
                    static_cast<void*>(p->corr_wg)})
    if (ptr) (void)hipFree(ptr);
  delete p;
}

mbc_status mbc_blocks_compute(const mbc_block_plan* p, const void* S_u, const void* S_d, int32_t s_dtype, int32_t T,
                              const int32_t dims[3], double* blocks, void* workspace, size_t ws_bytes,
                              void* stream) {
  if (!p || !dims) return fail(MBC_ERR_INVALID, "NULL argument");
  if (T <= 0 || dims[0] <= 0 || dims[1] <= 0 || dims[2] <= 0)
    return fail(MBC_ERR_INVALID, "T and dims must be positive");
  const int64_t V = int64_t(dims[0]) * dims[1] * dims[2];
  mbc_status st = check_inputs(S_u, S_d, s_dtype, T, V);
  if (st != MBC_OK) return st;
  if (p->h.n_types == 0) return MBC_OK;
  if (!is_device_ptr(blocks) || !aligned16(blocks)) return fail(MBC_ERR_INVALID, "blocks must be an aligned device pointer");
  const size_t need = block_workspace_bytes(p->h, T, V);
  if (!workspace || !is_device_ptr(workspace) || !aligned16(workspace))
    return fail(MBC_ERR_INVALID, "workspace must be an aligned device pointer");
  if (ws_bytes < need) return fail(MBC_ERR_INVALID, "workspace too small");
  int dev = -1;
  MBC_HIP(hipGetDevice(&dev));
  if (dev != p->device) return fail(MBC_ERR_INVALID, "plan was created on another device");
  MBC_HIP(launch_blocks(p, S_u, S_d, s_dtype == MBC_C64, T, dims, blocks, workspace,
                        reinterpret_cast<hipStream_t>(stream)));
  return MBC_OK;
}

mbc_status mbc_block_contract(const mbc_block_plan* p, const double* blocks, int32_t T, int32_t method, double* C,
                              void* workspace, size_t ws_bytes, void* stream) {
  if (!p) return fail(MBC_ERR_INVALID, "plan is NULL");
  if (T <= 0) return fail(MBC_ERR_INVALID, "T must be positive");
  if (method != MBC_BLOCK_TERMS && method != MBC_BLOCK_TREE) return fail(MBC_ERR_INVALID, "unknown method");
  if (!is_device_ptr(C) || !aligned16(C)) return fail(MBC_ERR_INVALID, "C must be an aligned device pointer");
  const size_t need = block_contract_workspace_bytes(p->h, T);
  if (p->h.n_terms > 0) {
    if (!is_device_ptr(blocks) || !aligned16(blocks))
      return fail(MBC_ERR_INVALID, "blocks must be an aligned device pointer");
    if (!workspace || !is_device_ptr(workspace) || !aligned16(workspace))
      return fail(MBC_ERR_INVALID, "workspace must be an aligned device pointer");
    if (ws_bytes < need) return fail(MBC_ERR_INVALID, "workspace too small");
  }
  int dev = -1;
  MBC_HIP(hipGetDevice(&dev));
  if (dev != p->device) return fail(MBC_ERR_INVALID, "plan was created on another device");
  MBC_HIP(launch_block_contract(p, blocks, T, method, C, workspace, reinterpret_cast<hipStream_t>(stream)));
  return MBC_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Tensor e-graphs (mbc_egraph.h)
// ---------------------------------------------------------------------------
struct mbc_egraph {
  mbc::EGraphHost g;
  mbc::EGraphExec x;            // device step tables of the last batch size
  std::vector<double*> dconst;  // device copies of the library-defined constants
  int device = -1;
};

namespace {

mbc_status finish_egraph(const mbc::TensorProblem& prob, int64_t node_limit, int32_t objective, mbc_egraph** out) {
  auto* e = new mbc_egraph();
  try {
    mbc::egraph_build(prob, node_limit, objective, &e->g);
  } catch (...) {
    delete e;
    throw;
  }
  const mbc::EGraphHost& g = e->g;
  MBC_LOGF("e-graph: %d terms, %d classes, %lld e-nodes (%s), %d roots, %d steps, plan %.3e flops (direct %.3e), "
           "workspace %lld elements per batch entry",
           g.n_input_terms, int(g.cls.size()), (long long)g.n_nodes, g.saturated ? "saturated" : "node limit reached",
           int(g.roots.size()), int(g.steps.size()), g.flops_plan, g.flops_direct, (long long)g.ws_elems);
  *out = e;
  return MBC_OK;
}

}  // namespace

extern "C" {

mbc_status mbc_egraph_build(const mbc_tensor_decl* tensors, int32_t n_tensors, const mbc_tensor_factor* factors,
                            const int32_t* term_begin, const double* coef, int32_t n_terms, int64_t node_limit,
                            int32_t objective, mbc_egraph** out) {
  if (!tensors || !factors || !term_begin || !coef || !out) return fail(MBC_ERR_INVALID, "NULL argument");
  if (n_tensors < 1 || n_terms < 1) return fail(MBC_ERR_INVALID, "n_tensors and n_terms must be >= 1");
  *out = nullptr;
  return guarded([&]() {
    mbc::TensorProblem prob;
    prob.decls.assign(tensors, tensors + n_tensors);
    prob.constant.resize(n_tensors);
    if (term_begin[0] != 0) throw std::invalid_argument("term_begin[0] must be 0");
    for (int k = 0; k < n_terms; ++k)
      if (term_begin[k + 1] <= term_begin[k]) throw std::invalid_argument("every term needs a factor");
    prob.term_begin.assign(term_begin, term_begin + n_terms + 1);
    prob.factors.assign(factors, factors + term_begin[n_terms]);
    prob.coef.assign(coef, coef + 2 * size_t(n_terms));
    return finish_egraph(prob, node_limit, objective, out);
  });
}

mbc_status mbc_egraph_build_blocks(const mbc_block_set* s, int32_t corr, int64_t node_limit, int32_t objective,
                                   mbc_egraph** out) {
  if (!s || !out) return fail(MBC_ERR_INVALID, "NULL argument");
  *out = nullptr;
  return guarded([&]() {
    mbc::TensorProblem prob;
    mbc::block_expressions(s->s, corr, &prob);
    return finish_egraph(prob, node_limit, objective, out);
  });
}

mbc_status mbc_egraph_get_stats(const mbc_egraph* e, mbc_egraph_stats* out) {
  if (!e || !out) return fail(MBC_ERR_INVALID, "NULL argument");
  const mbc::EGraphHost& g = e->g;
  std::memset(out, 0, sizeof(*out));
  out->n_tensors = int32_t(g.tensors.size());
  out->n_terms = g.n_input_terms;
  for (size_t c = 0; c < g.cls.size(); ++c) out->n_classes += g.parent[c] == int(c);
  out->n_nodes = int32_t(g.n_nodes);
  out->saturated = g.saturated ? 1 : 0;
  out->n_roots = int32_t(g.roots.size());
  out->n_steps = int32_t(g.steps.size());
  out->n_open = int32_t(g.out_labels.size());
  for (size_t j = 0; j < g.out_ext.size(); ++j) out->out_ext[j] = g.out_ext[j];
  out->out_elems = g.out_elems;
  out->ws_elems = g.ws_elems;
  out->flops_direct = g.flops_direct;
  out->flops_plan = g.flops_plan;
  return MBC_OK;
}

mbc_status mbc_egraph_export(const mbc_egraph* e, int32_t* buf, int64_t cap, int64_t* len) {
  if (!e || !len) return fail(MBC_ERR_INVALID, "NULL argument");
  return guarded([&]() {
    const mbc::EGraphHost& g = e->g;
    std::vector<int32_t> v;
    v.push_back(int32_t(g.cls.size()));
    for (size_t c = 0; c < g.cls.size(); ++c) {
      const mbc::EClass& k = g.cls[c];
      v.push_back(g.parent[c]);
      v.push_back(int32_t(k.factors.size()));
      v.push_back(k.n_open);
      v.push_back(int32_t(k.code.size()));
      v.insert(v.end(), k.code.begin(), k.code.end());
      v.push_back(int32_t(k.nodes.size()));
      for (const mbc::ENode& n : k.nodes) {
        v.push_back(n.c1);
        v.push_back(n.c2);
        v.push_back(n.sign);
        v.push_back(int32_t(n.o1.size()));
        v.insert(v.end(), n.o1.begin(), n.o1.end());
        v.push_back(int32_t(n.o2.size()));
        v.insert(v.end(), n.o2.begin(), n.o2.end());
      }
    }
    v.push_back(int32_t(g.terms.size()));
    for (const mbc::TermRoot& r : g.terms) {
      v.push_back(r.cls);
      v.push_back(int32_t(r.opens.size()));
      v.insert(v.end(), r.opens.begin(), r.opens.end());
    }
    v.push_back(int32_t(g.steps.size()));
    for (const mbc::Step& s : g.steps) {
      v.push_back(s.cls);
      v.push_back(s.node);
    }
    *len = int64_t(v.size());
    if (buf) {
      if (cap < *len) return fail(MBC_ERR_INVALID, "buffer too small");
      std::copy(v.begin(), v.end(), buf);
    }
    return MBC_OK;
  });
}

mbc_status mbc_egraph_term_coefs(const mbc_egraph* e, double* coef) {
  if (!e || !coef) return fail(MBC_ERR_INVALID, "NULL argument");
  for (size_t k = 0; k < e->g.terms.size(); ++k) {
    coef[2 * k] = e->g.terms[k].re;
    coef[2 * k + 1] = e->g.terms[k].im;
  }
  return MBC_OK;
}

mbc_status mbc_egraph_workspace_bytes(const mbc_egraph* e, int64_t batch, size_t* bytes) {
  if (!e || !bytes) return fail(MBC_ERR_INVALID, "NULL argument");
  if (batch < 1) return fail(MBC_ERR_INVALID, "batch must be >= 1");
  *bytes = size_t(e->g.ws_elems) * size_t(batch) * 16;
  return MBC_OK;
}

mbc_status mbc_egraph_execute(mbc_egraph* e, const double* const* inputs, const int64_t* batch_stride, int64_t batch,
                              double* out, void* workspace, size_t ws_bytes, void* stream) {
  if (!e || !inputs || !batch_stride) return fail(MBC_ERR_INVALID, "NULL argument");
  if (batch < 1) return fail(MBC_ERR_INVALID, "batch must be >= 1");
  if (!is_device_ptr(out) || !aligned16(out)) return fail(MBC_ERR_INVALID, "out must be an aligned device pointer");
  const size_t need = size_t(e->g.ws_elems) * size_t(batch) * 16;
  if (need > 0) {
    if (!workspace || !is_device_ptr(workspace) || !aligned16(workspace))
      return fail(MBC_ERR_INVALID, "workspace must be an aligned device pointer");
    if (ws_bytes < need) return fail(MBC_ERR_INVALID, "workspace too small");
  }
  const hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  int dev = -1;
  MBC_HIP(hipGetDevice(&dev));
  const int nt = int(e->g.tensors.size());
  if (e->dconst.empty()) {
    e->dconst.assign(nt, nullptr);
    e->device = dev;
    for (int t = 0; t < nt; ++t) {
      const std::vector<double>& v = e->g.constant[t];
      if (v.empty()) continue;
      MBC_HIP(hipMalloc(reinterpret_cast<void**>(&e->dconst[t]), v.size() * sizeof(double)));
      MBC_HIP(hipMemcpyAsync(e->dconst[t], v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice, st));
    }
    MBC_HIP(hipStreamSynchronize(st));
  }
  if (dev != e->device) return fail(MBC_ERR_INVALID, "graph's constants live on another device");
  std::vector<const double*> in(nt);
  std::vector<int64_t> bs(nt);
  for (int t = 0; t < nt; ++t) {
    in[t] = inputs[t];
    bs[t] = batch_stride[t];
    if (!in[t] && e->dconst[t]) {
      in[t] = e->dconst[t];
      bs[t] = 0;
    }
    if (!is_device_ptr(in[t]) || !aligned16(in[t]))
      return fail(MBC_ERR_INVALID, "input " + std::to_string(t) + " must be an aligned device pointer");
    if (bs[t] < 0) return fail(MBC_ERR_INVALID, "batch strides must be >= 0");
  }
  return guarded([&]() {
    MBC_HIP(mbc::egraph_launch(e->g, &e->x, in.data(), bs.data(), batch, out, workspace, st));
    return MBC_OK;
  });
}

void mbc_egraph_free(mbc_egraph* e) {
  if (!e) return;
  mbc::egraph_exec_free(&e->x);
  bool any = false;
  for (double* p : e->dconst) any = any || p;
  if (any) {
    (void)hipDeviceSynchronize();
    for (double* p : e->dconst)
      if (p) (void)hipFree(p);
  }
  delete e;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Linearised factor trees over arbitrary factor sets (mbc_tree.h)
// ---------------------------------------------------------------------------
struct mbc_factor_tree {
  mbc::TreeHost h;
  mbc::TreeDev d;
  int device = -1;
};

namespace {

void free_tree(mbc_factor_tree* t) {
  for (void* p : {static_cast<void*>(t->d.factor), static_cast<void*>(t->d.child_begin),
                  static_cast<void*>(t->d.child_list), static_cast<void*>(t->d.leaf),
                  static_cast<void*>(t->d.level_vertices), static_cast<void*>(t->d.coef)})
    if (p) (void)hipFree(p);
  delete t;
}

}  // namespace

extern "C" {

mbc_status mbc_factor_tree_create(const int32_t* factors, const int32_t* children, int64_t n_vertices,
                                  const double* coefficients, int64_t n_leaves, int32_t n_values, void* stream,
                                  mbc_factor_tree** out) {
  if (!factors || !children || !out || (n_leaves > 0 && !coefficients)) return fail(MBC_ERR_INVALID, "NULL argument");
  *out = nullptr;
  return guarded([&]() -> mbc_status {
    auto* t = new mbc_factor_tree();
    try {
      mbc::build_tree_host(factors, children, n_vertices, coefficients, n_leaves, n_values, &t->h);
    } catch (...) {
      delete t;
      throw;
    }
    if (hipGetDevice(&t->device) != hipSuccess) {
      delete t;
      return hip_fail(hipGetLastError(), "hipGetDevice");
    }
    const hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
    mbc_status st = MBC_OK;
    if ((st = upload(t->h.factor, &t->d.factor, hs)) != MBC_OK ||
        (st = upload(t->h.child_begin, &t->d.child_begin, hs)) != MBC_OK ||
        (st = upload(t->h.child_list, &t->d.child_list, hs)) != MBC_OK ||
        (st = upload(t->h.leaf, &t->d.leaf, hs)) != MBC_OK ||
        (st = upload(t->h.level_vertices, &t->d.level_vertices, hs)) != MBC_OK ||
        (st = upload(t->h.coef, &t->d.coef, hs)) != MBC_OK) {
      free_tree(t);
      return st;
    }
    const hipError_t e = hipStreamSynchronize(hs);
    if (e != hipSuccess) {
      free_tree(t);
      return hip_fail(e, "hipStreamSynchronize");
    }
    MBC_LOGF("factor tree: %lld vertices, depth %d, %lld leaves", (long long)t->h.n_vertices, t->h.depth,
             (long long)(t->h.coef.size() / 2));
    *out = t;
    return MBC_OK;
  });
}

mbc_status mbc_factor_tree_stats(const mbc_factor_tree* t, int32_t* depth, double* flops) {
  if (!t) return fail(MBC_ERR_INVALID, "tree is NULL");
  if (depth) *depth = t->h.depth;
  if (flops) *flops = t->h.flops;
  return MBC_OK;
}

mbc_status mbc_factor_tree_workspace_bytes(const mbc_factor_tree* t, int64_t batch, size_t* bytes) {
  if (!t || !bytes) return fail(MBC_ERR_INVALID, "NULL argument");
  if (batch < 1) return fail(MBC_ERR_INVALID, "batch must be >= 1");
  *bytes = size_t(batch) * size_t(t->h.n_vertices) * 16;
  return MBC_OK;
}

mbc_status mbc_factor_tree_evaluate(const mbc_factor_tree* t, const double* values, int64_t batch, double* out,
                                    void* workspace, size_t ws_bytes, void* stream) {
  if (!t) return fail(MBC_ERR_INVALID, "tree is NULL");
  if (batch < 1) return fail(MBC_ERR_INVALID, "batch must be >= 1");
  if (!is_device_ptr(out) || !aligned16(out)) return fail(MBC_ERR_INVALID, "out must be an aligned device pointer");
  if (t->h.n_values > 0 && (!is_device_ptr(values) || !aligned16(values)))
    return fail(MBC_ERR_INVALID, "values must be an aligned device pointer");
  if (!workspace || !is_device_ptr(workspace) || !aligned16(workspace))
    return fail(MBC_ERR_INVALID, "workspace must be an aligned device pointer");
  if (ws_bytes < size_t(batch) * size_t(t->h.n_vertices) * 16) return fail(MBC_ERR_INVALID, "workspace too small");
  int dev = -1;
  MBC_HIP(hipGetDevice(&dev));
  if (dev != t->device) return fail(MBC_ERR_INVALID, "tree was created on another device");
  MBC_HIP(mbc::launch_tree_eval(t->h, t->d, values, batch, out, workspace, reinterpret_cast<hipStream_t>(stream)));
  return MBC_OK;
}

void mbc_factor_tree_destroy(mbc_factor_tree* t) {
  if (!t) return;
  (void)hipDeviceSynchronize();
  free_tree(t);
}

}  // extern "C"
