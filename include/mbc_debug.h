/*
 * mbc_debug.h -- host-side checking aid for the plan compiler.
 *
 * Not part of the compute path: mbc_contract never calls it and it runs no
 * device code.  It walks a compiled schedule (tiles, Laplace row operations,
 * factor-tree leaves) exactly as the device kernel interprets it, in FP64 on
 * the host, so the plan compiler can be checked against an independent
 * reference on machines without a GPU.
 */
#ifndef MBC_DEBUG_H
#define MBC_DEBUG_H

#include "mbc.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Compiles the plan of index set `s` on the host only (no device arrays) and
 * evaluates eq. 1 with it:
 *   S_u, S_d  host [T][sites_per_t][12][12] complex128 (re/im interleaved)
 *   W         host [nnz] complex128 in index-set order, or NULL (exact W)
 *   C         host [n_corr][T] complex128 output
 *   stats     optional: the plan's statistics (lds_bytes etc.)
 * Errors as in mbc_plan_create (MBC_ERR_INVALID, MBC_ERR_UNSUPPORTED). */
mbc_status mbc_debug_eval_host(const mbc_index_set* s, int32_t precision, const double* S_u,
                               const double* S_d, int32_t T, int64_t sites_per_t, const double* W,
                               double* C, mbc_plan_stats* stats);

/* Gradients of eq. 1 (PyTorch's complex convention, as mbc_contract_backward)
 * computed on the host by walking the backward schedule: the leaf adjoints of
 * the determinant rows and the reverse sweep of the Laplace recursion for
 * grad_S, the per-entry sums over sites for grad_W.  All arrays are host
 * complex128; grad_W [nnz], grad_S_u/grad_S_d like S; any output may be NULL. */
mbc_status mbc_debug_backward_host(const mbc_index_set* s, int32_t precision, const double* S_u,
                                   const double* S_d, int32_t T, int64_t sites_per_t, const double* W,
                                   const double* grad_C, double* grad_W, double* grad_S_u,
                                   double* grad_S_d);

#ifdef __cplusplus
}
#endif

#endif /* MBC_DEBUG_H */
