// Host-side launchers of the HIP kernels (defined in kernels.hip).
#pragma once

#include <hip/hip_runtime_api.h>

#include <string>

#include "mbc_internal.hpp"

namespace mbc {

struct Launch {
  int T = 0;
  int64_t V = 0;     // sites per timeslice
  int chunk = 1;     // sites per workgroup (one timeslice)
  int nc = 1;        // chunks per timeslice
};

// fact: the factored forward on the f_* tiles (the exact weights, h.fwd_fact).
Launch forward_launch_shape(const PlanHost& h, int T, int64_t V, bool fact);

// Whether the kernels are instantiated for a compiled plan's family and
// sizes (source keys per thread, columns per level, dW keys per tile, dS
// bins and source-key lists); false with the reason in *why otherwise.
// mbc_plan_create rejects such a plan with MBC_ERR_UNSUPPORTED.
bool forward_supports(const PlanHost& h, std::string* why);
bool backward_supports(const PlanHost& h, std::string* why);

// W_plan[i] = W_user[perm[i]] in the plan's precision.
hipError_t launch_gather_w(const mbc_plan* p, const double* W_user, void* W_plan, hipStream_t st);

// Per-tile, per-chunk partial sums of the correlator: partial[tile][T][nc]
// complex128.  fact: the exact weights through their sink and source factors
// on the f_* tiles (requires h.fwd_fact; W_plan unused); otherwise W_plan on
// the forward tiles.
hipError_t launch_forward(const mbc_plan* p, const void* S_u, const void* S_d, int s_c64,
                          const Launch& L, const void* W_plan, double* partial, bool fact, hipStream_t st);

// C[corr][t] = fixed-order FP64 sum of the partials of the correlator's tiles
// (of the tiling launch_forward ran on).
hipError_t launch_reduce(const mbc_plan* p, const Launch& L, const double* partial, double* C, bool fact,
                         hipStream_t st);

// Size of the fixed per-device scratch array behind mbc_contract_noalloc,
// and its device address on the current device (looked up once per device).
constexpr size_t kScratchBytes = size_t(32) << 20;
hipError_t scratch_device_ptr(void** out);

// Zero-fills bytes (a multiple of 8) of device memory with a kernel (no
// memset node when the caller captures the stream).
hipError_t launch_zero(void* p, size_t bytes, hipStream_t st);

// Backward: dW (tile-major over timeslice chunks, then a fixed-order sum over
// chunks into grad_W in index-set order) and dS (one workgroup per site).
Launch backward_dw_launch_shape(const PlanHost& h, int T, int64_t V);
hipError_t launch_backward_dw(const mbc_plan* p, const void* S_u, const void* S_d, int s_c64, const Launch& L,
                              const void* W_plan, const double* grad_C, double* partial, double* grad_W,
                              hipStream_t st);
// factored: the plan's exact weights through their sink and source factors
// (requires h.rank1), on the factored dS tiling; otherwise W_plan.
hipError_t launch_backward_ds(const mbc_plan* p, const void* S_u, const void* S_d, int s_c64, int T, int64_t V,
                              const void* W_plan, const double* grad_C, void* grad_S_u, void* grad_S_d,
                              bool factored, hipStream_t st);

// Hadron blocks: per timeslice and block type, chunks of nch sites; the
// partial G matrices of the chunks live in the workspace.
struct BlockLaunch {
  int nch = 1;        // site chunks per timeslice
  int64_t chunk = 1;  // sites per chunk
};
BlockLaunch block_launch_shape(const BlockPlanHost& h, int T, int64_t V);
size_t block_workspace_bytes(const BlockPlanHost& h, int T, int64_t V);
size_t block_contract_workspace_bytes(const BlockPlanHost& h, int T);
hipError_t launch_blocks(const mbc_block_plan* p, const void* S_u, const void* S_d, int s_c64, int T,
                         const int32_t dims[3], double* blocks, void* workspace, hipStream_t st);
// method: MBC_BLOCK_TERMS (one product per term) or MBC_BLOCK_TREE (factor trees)
hipError_t launch_block_contract(const mbc_block_plan* p, const double* blocks, int T, int method, double* C,
                                 void* workspace, hipStream_t st);

}  // namespace mbc
