/*
 * mbc_blocks.h -- hadron blocks and block-level correlators (C ABI, gfx950).
 *
 * Sec. 2 of Humphrey, Detmold, Young and Zanotti (arXiv:2201.04269) defines
 * a baryon block: the three-quark expectation of one sink baryon, projected
 * to a sink momentum, with its source colour/spin indices left open.  Here
 *
 *   f^h_p[t][alpha][A][Y][C] = sum_{x in t} e^{-i p.x} < h_alpha(x) q1bar(A) q2bar(Y) q1bar(C) >
 *
 * for the baryon families h = p (q1 = u, q2 = d) and n (q1 = d, q2 = u) with
 * Gamma = C gamma5 or C gamma5 P+- (Sec. 1), alpha the sink spin and
 * A, Y, C = 4*colour + spin the source indices, antiquarks in the order of
 * the paper's proton block.  Blocks are antisymmetric in A <-> C.
 *
 * Sec. 3 writes a multi-baryon correlator as a sum of products of blocks.  A
 * block-level correlator here places baryon i of every written product of
 * the sink operator of eq. "ops" at its own sink point, projected to its own
 * momentum p_i, with source baryon i at source point z_i (a local source
 * when all z_i coincide; the general block form of Sec. 3 lets the blocks'
 * source points differ):
 *
 *   C[t] = sum_{x_1..x_A in t} e^{-i sum_i p_i.x_i} < O_snk(x_1, .., x_A) Obar_src(z_1, .., z_A) >
 *        = sum_k w_k prod_i f^{h_i}_{p_i}[t][eta_{i,k}]
 *
 * A block's three antiquarks may then come from different source points:
 * f^h_p[t][alpha][A][Y][C] for source points (z_A, z_Y, z_C), its quarks
 * propagating from those points.
 *
 * The host expands the Wick contraction by the set partitions of the source
 * antiquarks among the baryons (D_I: N_w = 9 partitions, Sec. 3), over the
 * canonical source keys of eq. 1's index set, orders each product's factors
 * and merges equal products exactly (the canonical ordering with
 * multiplicities of Sec. 3).  With one site per timeslice the block-level
 * correlator equals the local correlator of mbc_contract.
 *
 * Conventions beyond mbc.h
 *   sites         V = L1 L2 L3 sites per timeslice, site v at coordinates
 *                 (x1, x2, x3) with v = x1 + L1 (x2 + L2 x3)
 *   momenta       integer triples n: p.x = 2 pi (n1 x1/L1 + n2 x2/L2 + n3 x3/L3)
 *   propagators   S[n_points][T][V][12][12]: one set per source point
 *   blocks        device [T][n_types][4][12][12][12] complex128 (re/im
 *                 interleaved doubles); type order as mbc_block_set_types
 *   arithmetic    FP64 throughout; block sums over sites and term sums are
 *                 combined in a fixed order (run-to-run reproducible)
 * Errors, streams and ownership are as in mbc.h.
 */
#ifndef MBC_BLOCKS_H
#define MBC_BLOCKS_H

#include "mbc.h"

#ifdef __cplusplus
extern "C" {
#endif

/* baryon families of a block type */
enum { MBC_FAMILY_P = 0, MBC_FAMILY_N = 1 };
/* evaluation of the block-level terms: one product per term, or the
 * correlator's linearised factor tree (Sec. 4: terms sharing their leading
 * factors share those multiplications) */
enum { MBC_BLOCK_TERMS = 0, MBC_BLOCK_TREE = 1 };

typedef struct {
  int32_t op;         /* MBC_OP_* */
  int32_t snk_spin;   /* alpha (proton/neutron), j (3He); 0..3 */
  int32_t src_spin;   /* alpha', j' */
  int32_t sign_mode;  /* MBC_SIGNS_EXACT or MBC_SIGNS_R2 */
  int32_t mom[3][3];  /* sink momentum of baryon slot i (written order); slots
                         beyond the operator's baryon count are ignored */
  int32_t src_pt[3];  /* source point (0..2) of source baryon slot i (written
                         order): all 0 is a local source; distinct points
                         displace the source baryons, each point with its own
                         propagator set (see mbc_blocks_compute) */
} mbc_block_corr_desc;

typedef struct mbc_block_set mbc_block_set;   /* opaque, host, library-owned */
typedef struct mbc_block_plan mbc_block_plan; /* opaque, owns its device arrays */

/* ---- block sets (host only; Sec. 3 expanded form) ----
 * Builds the block types (distinct (family, projector, momentum, source
 * points of A, Y, C) over the expansion of every correlator, in order of
 * first use) and the merged
 * product terms of n_corr >= 1 correlators.  Term k of correlator c is
 * w_k prod_i blocks[t][factor[k][i]] with factor = (type*4 + alpha)*1728 +
 * (A*12 + Y)*12 + C and (z_A, A) < (z_C, C); the weights are exact: w_k = (num_re[k] +
 * i num_im[k]) / den[c] (den = 1, 2, 6 for the I, D_II, 3He_II operators).
 * A term of a correlator with fewer baryons than n_slots has factor -1 in
 * the unused slots.  Terms are ordered by correlator, then by factors.
 * Errors: MBC_ERR_INVALID for a NULL pointer, n_corr < 1, an unknown
 * operator or sign mode, a spin outside 0..3, a source point outside 0..2. */
mbc_status mbc_block_set_build(const mbc_block_corr_desc* corrs, int32_t n_corr, mbc_block_set** out);
/* Sizes (any output may be NULL): correlators, slots per term (the largest
 * baryon count), block types, terms, source points (1 + the largest src_pt). */
mbc_status mbc_block_set_dims(const mbc_block_set* s, int32_t* n_corr, int32_t* n_slots, int32_t* n_types,
                              int64_t* n_terms, int32_t* n_points);
/* Block types into caller-allocated host arrays (any may be NULL):
 * family [n_types] (MBC_FAMILY_*), projector [n_types] (0, +1, -1),
 * mom [n_types][3], src [n_types][3] (source points of A, Y, C). */
mbc_status mbc_block_set_types(const mbc_block_set* s, int32_t* family, int32_t* projector, int32_t* mom,
                               int32_t* src);
/* Terms into caller-allocated host arrays (any may be NULL):
 * factor [n_terms][n_slots], corr_id [n_terms], num_re/num_im [n_terms],
 * den [n_corr]. */
mbc_status mbc_block_set_export(const mbc_block_set* s, int32_t* factor, int32_t* corr_id, int64_t* num_re,
                                int64_t* num_im, int64_t* den);
/* Linearised factor tree (Sec. 4) of correlator `corr` of a block set: the
 * prefix tree of its terms' factor strings in depth-first order, as the
 * paper's three arrays.  factors[v] is the block factor of vertex v (-1 for
 * the root, vertex 0), children[v] its number of children; the leaves, in
 * depth-first order, are the correlator's terms in export order, so the
 * coefficients array is that correlator's num_re/num_im over den.  The
 * correlator's value is the sum over root-to-leaf paths of the leaf
 * coefficient times the product of the factors on the path.  *n_vertices
 * receives the vertex count; factors and children (caller-allocated host
 * arrays of that length) may be NULL.  MBC_ERR_INVALID for a bad corr. */
mbc_status mbc_block_set_factor_tree(const mbc_block_set* s, int32_t corr, int64_t* n_vertices, int32_t* factors,
                                     int32_t* children);
/* Frees a block set (NULL-safe). */
void mbc_block_set_free(mbc_block_set* s);

/* ---- multiplicity analytics (host only; Sec. 3, Fig. 2) ----
 * Expands one correlator in the paper's way: every written source term x
 * every sink product x every partition is a string of block factors
 * (hadron, momentum, source points, index bundle (A, Y, C, alpha)), with no
 * merging of the source and no use of block antisymmetry.  Each string's
 * factors are put in lexicographic order and identical strings are counted.
 * On return *n_terms is the length of the expansion, *n_distinct the number
 * of distinct strings, *max_mult the largest multiplicity, and hist[m]
 * (0 < m < hist_len) the number of distinct strings that occur m times
 * (hist[0] = 0; hist may be NULL).  MBC_ERR_UNSUPPORTED if the expansion
 * has more than max_terms terms (checked before any is formed; *n_terms is
 * still set). */
mbc_status mbc_block_multiplicities(const mbc_block_corr_desc* corr, int64_t max_terms, int64_t* n_terms,
                                    int64_t* n_distinct, int64_t* max_mult, int64_t* hist, int32_t hist_len);

/* ---- plans and kernels ----
 * Uploads a block set's types and terms to the current device on `stream`
 * (synchronised before return). */
mbc_status mbc_block_plan_create(const mbc_block_set* s, void* stream, mbc_block_plan** out);

typedef struct {
  int32_t n_types, n_slots, n_corr, n_points;
  int64_t n_terms;
  int32_t n_gmats;             /* G matrices the block kernel forms per site (one per block
                                  type, two for a type whose like antiquarks come from
                                  different source points) */
  double block_flops_per_site; /* per site, all G matrices: 432 entries x (2 x nnz(Gamma)
                                  products + phase) + 6912 x 3 complex multiply-adds each */
  double contract_flops_per_t; /* per timeslice: 8 per complex multiply or add of the terms */
  int64_t tree_vertices;       /* factor-tree vertices over all correlators (roots included) */
  double tree_flops_per_t;     /* per timeslice, factor trees: 8 per non-root vertex (its
                                  factor times its children's sum, added into its parent) */
} mbc_block_plan_stats;
mbc_status mbc_block_plan_get_stats(const mbc_block_plan* p, mbc_block_plan_stats* out);

/* Device workspace of mbc_blocks_compute (T timeslices, lattice dims) and of
 * mbc_block_contract (T timeslices); *bytes is the larger of the two. */
mbc_status mbc_block_workspace_bytes(const mbc_block_plan* p, int32_t T, const int32_t dims[3], size_t* bytes);
/* Destroys a block plan (NULL-safe); synchronises the device first. */
void mbc_block_plan_destroy(mbc_block_plan* p);

/* Blocks of every type (Sec. 2, momentum projected).
 * S_u, S_d   device [n_points][T][V][12][12] complex (s_dtype), 16-byte
 *            aligned, set p the propagators from source point p;
 *            V = dims[0] dims[1] dims[2] (dims: host array, each >= 1)
 * blocks     device output [T][n_types][4][1728] complex128, both halves of
 *            the A <-> C antisymmetry written (zero where A == C)
 * workspace  device, >= mbc_block_workspace_bytes(p, T, dims) */
mbc_status mbc_blocks_compute(const mbc_block_plan* p, const void* S_u, const void* S_d, int32_t s_dtype,
                              int32_t T, const int32_t dims[3], double* blocks, void* workspace,
                              size_t ws_bytes, void* stream);
/* Block-level correlators from blocks (Sec. 3 expanded form).
 * blocks     device [T][n_types][4][1728] complex128 (mbc_blocks_compute)
 * method     MBC_BLOCK_TERMS or MBC_BLOCK_TREE (same value up to rounding)
 * C          device output [n_corr][T] complex128
 * workspace  device, >= mbc_block_workspace_bytes(p, T, dims) */
mbc_status mbc_block_contract(const mbc_block_plan* p, const double* blocks, int32_t T, int32_t method, double* C,
                              void* workspace, size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* MBC_BLOCKS_H */
