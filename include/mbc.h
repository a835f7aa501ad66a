/*
 * mbc.h -- C ABI of the multi-baryon correlator contraction library (gfx950).
 *
 * The library evaluates two-point correlators of multi-baryon interpolating
 * operators in the determinant form of eq. 1 of Humphrey, Detmold, Young and
 * Zanotti, "Novel Algorithms for Computing Correlation Functions of Nuclei"
 * (arXiv:2201.04269):
 *
 *   C_c[t] = sum_{x in t} sum_{k in I_c} W_k det(S_u(x)[snk_u_k; src_u_k]) det(S_d(x)[snk_d_k; src_d_k])
 *
 * per correlator c and timeslice t (zero-momentum sink sum, Sec. 2), with the
 * index set I of non-zero weights (Sec. 1, "index set"), the canonical
 * ordering of terms with merged multiplicities (Sec. 3), and the factor-tree
 * evaluation of Sec. 4 (one u-determinant times the weighted sum of its
 * d-determinant children), over minors shared through the Laplace recursion.
 *
 * Conventions shared by every entry point
 *   quark index   a = 4*colour + spin, 0 <= a < 12 (rows: sink, columns: source)
 *   propagators   S[T][V][12][12] complex, V = sites per timeslice, row-major,
 *                 re/im interleaved; complex128 (MBC_C128) or complex64 (MBC_C64)
 *   correlators   C[n_corr][T] complex128 (re/im interleaved doubles)
 *   weights       W[nnz] complex128 in the index set's entry order
 *   pointers      "device" arguments must be device memory of the current HIP
 *                 device (checked with hipPointerGetAttributes); host arrays
 *                 are caller-owned and read or written before return
 *   streams       `stream` is a hipStream_t (NULL = default stream); all device
 *                 work is asynchronous on it; outputs are complete when the
 *                 stream reaches that point
 *   ownership     index sets and plans are library-owned handles; every other
 *                 buffer is caller-owned and never retained past the call
 *   errors        every function returns a status and never throws or aborts;
 *                 mbc_last_error() describes the last failure of the calling
 *                 thread (HIP errors carry hipGetErrorString); outputs are
 *                 unspecified after an error
 *   logging       with the environment variable MBC_LOG set (and not "0"),
 *                 every index set, plan, block set, block plan and e-graph
 *                 built writes one "[mbc] ..." line with its sizes to stderr
 */
#ifndef MBC_H
#define MBC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MBC_OK = 0,
  MBC_ERR_INVALID = 1,     /* bad argument: null, range, alignment, non-device pointer */
  MBC_ERR_UNSUPPORTED = 2, /* valid request the library does not implement */
  MBC_ERR_NOMEM = 3,       /* host or device allocation failed */
  MBC_ERR_HIP = 4,         /* a HIP runtime call failed */
  MBC_ERR_INTERNAL = 5
} mbc_status;

/* operators of eq. "ops" and the single baryons of Sec. 1 */
enum { MBC_OP_PROTON = 0, MBC_OP_NEUTRON = 1, MBC_OP_DI = 2, MBC_OP_DII = 3,
       MBC_OP_HE3_I = 4, MBC_OP_HE3_II = 5 };
/* relative signs of the written terms of D_II and 3He_II:
 * EXACT keeps them (both operators then vanish at a local sink and their
 * canonical index sets are empty); R2 sets every written relative sign to +1,
 * a non-physical stand-in with a non-empty index set */
enum { MBC_SIGNS_EXACT = 0, MBC_SIGNS_R2 = 1 };
/* arithmetic of a plan: FP64 throughout, or complex-FP32 minors and products
 * with compensated (TwoSum) FP32 accumulation and an FP64 final reduction */
enum { MBC_F64 = 0, MBC_F32C = 1 };
/* element type of propagator buffers */
enum { MBC_C128 = 0, MBC_C64 = 1 };

typedef struct {
  int32_t op;         /* MBC_OP_* */
  int32_t snk_spin;   /* open spin index at the sink: alpha (proton/neutron), j (3He); 0..3 */
  int32_t src_spin;   /* the same at the source (alpha', j') */
  int32_t sign_mode;  /* MBC_SIGNS_EXACT or MBC_SIGNS_R2 */
  int32_t symmetrise; /* 1: canonical sorted/merged keys; 0: raw written terms */
} mbc_op_desc;

typedef struct mbc_index_set mbc_index_set; /* opaque, host, library-owned */
typedef struct mbc_plan mbc_plan;           /* opaque, owns its device arrays */

/* Description of the last error on the calling thread ("" if none). */
const char* mbc_last_error(void);
/* Library version string. */
const char* mbc_version(void);

/* ---- index sets (host only; eq. 1 "index set", Sec. 3 canonical order) ----
 * Builds the index set of n_corr >= 1 correlators that share (n_u, n_d).
 * Correlator c gets W_{r,c'} = sigma s^2 w_r conj(w_c') on the Cartesian
 * product of its sink keys r and source keys c' (s^2 = 1, 1/2, 1/6 for the
 * I, D_II, 3He_II operators; sigma the Grassmann sign of the flavour-separated
 * determinant form).  Canonical entries are ordered by correlator, then
 * lexicographically by (snk_u, src_u, snk_d, src_d).  Integer arithmetic only;
 * a correlator may have an empty set.  Errors: MBC_ERR_INVALID for a null
 * pointer, n_corr < 1, an unknown operator, a spin outside 0..3, or mixed
 * (n_u, n_d). */
mbc_status mbc_build_index_set(const mbc_op_desc* ops, int32_t n_corr, mbc_index_set** out);
/* Sizes of an index set; any output pointer may be NULL. */
mbc_status mbc_index_set_dims(const mbc_index_set* s, int32_t* n_u, int32_t* n_d,
                              int64_t* nnz, int32_t* n_corr);
/* Copies the index set into caller-allocated host arrays (any may be NULL):
 * snk_u/src_u [nnz][n_u], snk_d/src_d [nnz][n_d] (sorted tuples), corr_id [nnz],
 * w_num_re/w_num_im [nnz] exact numerators (sigma included), w_den [n_corr];
 * W_k = (w_num_re[k] + i w_num_im[k]) / w_den[corr_id[k]]. */
mbc_status mbc_index_set_export(const mbc_index_set* s, int32_t* snk_u, int32_t* src_u,
                                int32_t* snk_d, int32_t* src_d, int32_t* corr_id,
                                int64_t* w_num_re, int64_t* w_num_im, int64_t* w_den);
/* Frees an index set (NULL-safe). */
void mbc_index_set_free(mbc_index_set* s);

/* ---- plans (host compiles once per index set; device arrays uploaded) ----
 * Compiles the factor-tree evaluation schedule of a canonical index set:
 * per correlator, the sink keys are ordered so that equal u-rows are
 * adjacent, cut into tiles, and each tile gets the Laplace-recursion row
 * operations (shared minors) that produce its u- and d-determinant rows.
 * Every correlator's entries must form the Cartesian product of its sink and
 * source keys (always true for mbc_build_index_set with symmetrise = 1);
 * otherwise MBC_ERR_UNSUPPORTED.  n_u, n_d must lie in 1..6.  `precision` is
 * MBC_F64 or MBC_F32C.  The plan's device arrays are uploaded on `stream`;
 * the call synchronises that stream before returning. */
mbc_status mbc_plan_create(const mbc_index_set* s, int32_t precision, void* stream, mbc_plan** out);

typedef struct {
  int64_t nnz;              /* index entries (all correlators) */
  int32_t n_corr, n_u, n_d, precision;
  int32_t n_tiles;          /* tiles over all correlators */
  int32_t threads;          /* threads per workgroup */
  int64_t lds_bytes;        /* dynamic LDS per workgroup of the forward kernel */
  double alg_flops_per_site;  /* sum_k #minors_k (8k-2) + 8 (#leaves + #groups), global minor DAG */
  double exec_flops_per_site; /* the same count over what the kernel executes (with recomputation) */
  double in_bytes_per_site;   /* propagator bytes read per site (both flavours) */
  int32_t b_n_tiles;          /* tiles of the backward schedule */
  int64_t b_lds_bytes_ds;     /* dynamic LDS per workgroup, dS kernel */
  int64_t b_lds_bytes_dw;     /* dynamic LDS per workgroup, dW kernel */
  double ds_alg_flops_per_site; /* dS: minors + reverse sweep (16k per level-k minor) + 16 per entry */
  double dw_alg_flops_per_site; /* dW: minors + 8 per entry */
  int32_t w_n_tiles;            /* tiles of the dW schedule */
  int32_t rank1;                /* 1: every correlator's exact weights are a sink vector times a
                                   source vector (the factored schedules below apply) */
  int32_t f_n_tiles;            /* tiles of the factored schedule */
  int64_t f_lds_bytes_ds;       /* dynamic LDS per workgroup of the factored dS kernel */
  int32_t fwd_factored;         /* 1: mbc_contract with W = NULL evaluates the exact weights through
                                   their factors on the factored schedule (per run of equal
                                   u-tuples: sum over d columns of (sum_b u[b] Dd)(sum_s v[s] Du)) */
  int32_t ds_factored;          /* 1: mbc_contract_backward with W = NULL runs the factored dS
                                   schedule (rank1, and not the (3,3) family in FP32-comp) */
  int64_t f_lds_bytes_fwd;      /* dynamic LDS per workgroup of that factored forward */
  double fact_alg_flops_per_site;    /* forward flops of the factored evaluation (global minor DAG) */
  double fact_ds_alg_flops_per_site; /* dS flops with the factored leaf adjoints */
} mbc_plan_stats;
mbc_status mbc_plan_get_stats(const mbc_plan* p, mbc_plan_stats* out);

/* Device workspace needed by mbc_contract (backward = 0) or
 * mbc_contract_backward (backward = 1) for T timeslices of sites_per_t sites. */
mbc_status mbc_plan_workspace_bytes(const mbc_plan* p, int32_t T, int64_t sites_per_t,
                                    int32_t backward, size_t* bytes);
/* Destroys a plan (NULL-safe); synchronises the device first. */
void mbc_plan_destroy(mbc_plan* p);

/* ---- forward: eq. 1 per site, zero-momentum sum per timeslice ----
 * S_u, S_d  device [T][sites_per_t][12][12] complex (s_dtype), 16-byte aligned
 * W         device [nnz] complex128 in index-set order, or NULL for the
 *           plan's exact weights (num/den of the index set)
 * C         device [n_corr][T] complex128 output
 * workspace device, >= mbc_plan_workspace_bytes(p, T, sites_per_t, 0)
 * The per-site sums are combined over sites in a fixed order in FP64, so the
 * result is run-to-run reproducible.  An empty index set gives C = 0. */
mbc_status mbc_contract(const mbc_plan* p, const void* S_u, const void* S_d, int32_t s_dtype,
                        int32_t T, int64_t sites_per_t, const double* W, double* C,
                        void* workspace, size_t ws_bytes, void* stream);

/* ---- forward without allocation or workspace ----
 * For callers that cannot allocate device memory or pass a workspace (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation).  Same arguments, result and errors as mbc_contract without
 * the workspace: the intermediate buffers (plan-ordered weights when W is
 * given, per-tile partial sums) live in a fixed scratch array of
 * 32 MiB = 33554432 bytes per GPU, held by the library until the process
 * ends.  A call whose intermediates would exceed it returns
 * MBC_ERR_UNSUPPORTED (for example the 3He batch with a caller W: 8.35M
 * weights); use mbc_contract with a workspace there.  The call allocates
 * nothing.  Every call on one GPU shares that GPU's scratch: calls that
 * overlap on one GPU (other streams, other threads) race and must be
 * serialised by the caller. */
mbc_status mbc_contract_noalloc(const mbc_plan* p, const void* S_u, const void* S_d, int32_t s_dtype,
                                int32_t T, int64_t sites_per_t, const double* W, double* C, void* stream);

/* ---- backward (adjoint of mbc_contract), PyTorch's complex convention ----
 * grad_C    device [n_corr][T] complex128: dL/dC* of a real loss L
 * grad_W    device [nnz] complex128 or NULL:
 *           grad_W[k] = sum_t grad_C[c_k][t] conj(dC_{c_k}[t]/dW_k)
 *                     = sum_{x} grad_C[c_k][t(x)] conj(det_u det_d)  (C is linear in W, eq. 1)
 * grad_S_u, grad_S_d device, same layout and dtype as S, or NULL:
 *           grad_S(x)[a,b] = sum_c grad_C[c][t(x)] conj(dC_c[t(x)]/dS(x)[a,b]),
 *           by Jacobi's formula through the Laplace recursion (reverse sweep),
 *           with every minor recomputed, none stored.
 * workspace device, >= mbc_plan_workspace_bytes(p, T, sites_per_t, 1) */
mbc_status mbc_contract_backward(const mbc_plan* p, const void* S_u, const void* S_d,
                                 int32_t s_dtype, int32_t T, int64_t sites_per_t,
                                 const double* W, const double* grad_C, double* grad_W,
                                 void* grad_S_u, void* grad_S_d, void* workspace,
                                 size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* MBC_H */
