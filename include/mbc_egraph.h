/*
 * mbc_egraph.h -- tensor e-graphs (C ABI; host planner, gfx950 executor).
 *
 * Sec. 5 of Humphrey, Detmold, Young and Zanotti (arXiv:2201.04269) finds
 * common sub-expressions of a sum of tensor products with a tensor e-graph:
 * e-classes of equal expressions, e-nodes E = E1 E2 produced by a re-write
 * rule that permutes E's index slots by a signed permutation and splits it
 * into two canonicalised sub-expressions, a union-find over class ids and a
 * hash-cons from e-nodes to classes.  A plan is extracted by choosing one
 * e-node per class with an objective that rewards re-used, costly
 * sub-expressions.  Here:
 *
 *   expressions  sum_k coef_k prod_i T_{t_ki}[labels]: a label that occurs
 *                twice in a term is summed, once is open; every term has the
 *                same open labels, and the result is indexed by them in
 *                increasing label order
 *   symmetries   (p, s) is a symmetry of T when T[x_p0, x_p1, ..] = s T[x_0, x_1, ..]
 *   canonical    factors listed by increasing tensor id, each rewritten by any
 *     form       symmetry of its tensor; labels renamed by first appearance
 *                (the k-th summed label to code 2k, the k-th open one to
 *                2k + 1); the code (per factor: tensor id, slot codes) is the
 *                lexicographically smallest over all arrangements, and among
 *                arrangements reaching it the smallest tuple of open labels
 *                fixes the open-slot map and the sign (an expression reaching
 *                it with both signs vanishes identically)
 *   re-writes    E = E1 E2 over every split of a class's canonical factors
 *                (E1 holds its first factor; splits in increasing subset
 *                mask), admitted when (1) both parts hold a label that is
 *                summed in E and (2) one of them holds a factor with no open
 *                label of E (the paper's two conditions); classes are
 *                expanded first in, first out until node_limit e-nodes exist;
 *                a class left without an e-node is split at the root of a
 *                greedy pairwise contraction order of its factors (join the
 *                two operands that remove the most intermediate elements,
 *                then the pair carrying the fewest label combinations, then
 *                the first pair)
 *   roots        terms with the same class and open map are one root, their
 *                coefficients (times the canonical signs) summed; a root
 *                whose sum is exactly zero is dropped (those terms cancel)
 *   extraction   from the roots, in order of first appearance.
 *                MBC_EXTRACT_REUSE (the paper's objective): per class the
 *                e-node with the largest sum over its distinct children c
 *                with two or more factors of (parent classes of c - 1) x the
 *                direct cost of c, then the fewest flops of its own
 *                contraction, then the first.  MBC_EXTRACT_FLOPS: the
 *                smallest tree cost (own contraction + children's).
 *                MBC_EXTRACT_SHARED: the MBC_EXTRACT_FLOPS choice refined in
 *                rounds (at most 10): with P the classes of the current plan,
 *                each class of P (by id) takes the e-node minimising its own
 *                flops plus the tree cost of its distinct children with two
 *                or more factors that are not in P (a class of the plan is
 *                computed once), if strictly cheaper; new children take
 *                their tree-cost e-node.
 *   flops        a contraction E1 E2 -> E costs 8 x the product of the
 *                extents of the labels of E1 and E2 (one complex
 *                multiply-add per point); the direct cost of an n-factor
 *                expression is 8 (n - 1) x the product of all its extents
 *
 * Errors, streams and ownership are as in mbc.h.  Handles are host objects;
 * a graph with library-defined constant tensors (mbc_egraph_build_blocks)
 * keeps device copies of them, made on first execution on `stream`.
 */
#ifndef MBC_EGRAPH_H
#define MBC_EGRAPH_H

#include "mbc.h"
#include "mbc_blocks.h"

#ifdef __cplusplus
extern "C" {
#endif

enum { MBC_EGRAPH_MAX_RANK = 8, MBC_EGRAPH_MAX_SYM = 4, MBC_EGRAPH_MAX_LABEL = 64, MBC_EGRAPH_MAX_FACTORS = 16 };
enum { MBC_EXTRACT_REUSE = 0, MBC_EXTRACT_FLOPS = 1, MBC_EXTRACT_SHARED = 2 };

typedef struct {
  int32_t rank;                                       /* 1..MBC_EGRAPH_MAX_RANK */
  int32_t ext[MBC_EGRAPH_MAX_RANK];                   /* extent of each slot, 1..4096 */
  int32_t n_sym;                                      /* symmetry generators, 0..MBC_EGRAPH_MAX_SYM */
  int32_t perm[MBC_EGRAPH_MAX_SYM][MBC_EGRAPH_MAX_RANK]; /* generator g: slot permutation */
  int32_t sign[MBC_EGRAPH_MAX_SYM];                   /* generator g: +1 or -1 */
} mbc_tensor_decl;

typedef struct {
  int32_t tensor;                                     /* index into the tensor declarations */
  int32_t label[MBC_EGRAPH_MAX_RANK];                 /* 0..MBC_EGRAPH_MAX_LABEL-1, first `rank` used */
} mbc_tensor_factor;

typedef struct mbc_egraph mbc_egraph; /* opaque, library-owned */

/* Builds the e-graph of sum_k coef_k prod (factors[term_begin[k] .. term_begin[k+1]))
 * and extracts a plan.  coef: host [n_terms][2] (re, im).  Every term has
 * 1..MBC_EGRAPH_MAX_FACTORS factors.  node_limit >= 0 bounds the e-nodes made
 * by re-writes.  MBC_ERR_INVALID for a bad declaration (rank, extent,
 * permutation, sign), a label out of range or used more than twice or with
 * two extents, terms with different open labels, n_terms < 1;
 * MBC_ERR_UNSUPPORTED if a symmetry group makes a tensor vanish, a
 * sub-expression vanishes identically, or a canonical form needs more than
 * 2^20 partial arrangements. */
mbc_status mbc_egraph_build(const mbc_tensor_decl* tensors, int32_t n_tensors, const mbc_tensor_factor* factors,
                            const int32_t* term_begin, const double* coef, int32_t n_terms, int64_t node_limit,
                            int32_t objective, mbc_egraph** out);

/* The block-level correlator `corr` of a block set (mbc_blocks.h) as tensor
 * expressions, and their e-graph.  Each pair (written sink product, written
 * source product) of eq. "ops" and each set partition of the written
 * source's antiquarks among the sink baryons is one term:
 *   sign(P) (-1)^{A(A-1)/2} x relative signs / den
 *   x [C gamma5 tying the sink spins; unit vector e_j for a fixed spin]
 *   x prod_i f^{h_i}(sigma_i; colour, spin of its antiquarks A, Y, C)
 *   x prod_{source baryons} eps(colours) Gamma(spins of the first two antiquarks)
 *   x [C gamma5 tying the source spins; e_j for a fixed one].
 * Tensor ids: 0..n_types-1 are the set's block types, [4][3][4][3][4][3][4]
 * (the layout of mbc_blocks_compute's [4][1728] per type), with the A <-> C
 * antisymmetry when z_A = z_C; then the library-defined constants eps
 * [3][3][3], C gamma5, C gamma5 P+, C gamma5 P- [4][4] and e_0..e_3 [4].
 * The result is a scalar per timeslice.  MBC_ERR_INVALID if a block type
 * the expressions need is not in the set (a correlator whose canonical
 * expansion is empty, such as exact-sign D_II with a local source, adds no
 * types of its own). */
mbc_status mbc_egraph_build_blocks(const mbc_block_set* s, int32_t corr, int64_t node_limit, int32_t objective,
                                   mbc_egraph** out);

typedef struct {
  int32_t n_tensors, n_terms;
  int32_t n_classes;     /* e-classes (union-find roots) */
  int32_t n_nodes;       /* e-nodes */
  int32_t saturated;     /* 1: no admitted re-write was cut by node_limit */
  int32_t n_roots;       /* distinct (class, open map) pairs of the terms whose
                            summed coefficients are not exactly zero */
  int32_t n_steps;       /* contractions of the extracted plan */
  int32_t n_open;        /* rank of the result */
  int32_t out_ext[MBC_EGRAPH_MAX_LABEL];
  int64_t out_elems;     /* elements of the result */
  int64_t ws_elems;      /* complex elements of all intermediates, per batch entry */
  double flops_direct;   /* every term as one loop nest */
  double flops_plan;     /* the extracted plan: its contractions + the sum over roots */
} mbc_egraph_stats;
mbc_status mbc_egraph_get_stats(const mbc_egraph* g, mbc_egraph_stats* out);

/* Flat int32 description (for inspection and tests):
 *   n_classes, then per class id: representative, n_factors, n_open,
 *     code length L, code[L], n_nodes, per e-node: child1, child2, sign,
 *     n1, labels of child1's open slots[n1], n2, labels[n2]
 *   n, then per term whose product does not vanish identically (n of them,
 *     in input order): class, n_open, the caller's labels of the class's
 *     open slots
 *   n_steps, then per step: class, chosen e-node index
 * Labels are the class's canonical codes.  *len receives the length; buf
 * (capacity cap) may be NULL. */
mbc_status mbc_egraph_export(const mbc_egraph* g, int32_t* buf, int64_t cap, int64_t* len);
/* For the terms listed by mbc_egraph_export: coef_k x the sign of its
 * canonical form, host [n][2]. */
mbc_status mbc_egraph_term_coefs(const mbc_egraph* g, double* coef);

/* Device workspace of mbc_egraph_execute for `batch` entries. */
mbc_status mbc_egraph_workspace_bytes(const mbc_egraph* g, int64_t batch, size_t* bytes);
/* Evaluates the extracted plan for `batch` independent sets of inputs.
 * inputs       host array [n_tensors] of device pointers to complex128
 *              tensors (row-major over the slots); entry b of tensor t
 *              starts at inputs[t] + 2 * b * batch_stride[t] doubles
 *              (stride 0: shared).  For mbc_egraph_build_blocks graphs,
 *              entries for the constant tensors may be NULL (library values).
 * batch_stride host [n_tensors], complex elements
 * out          device [batch][out_elems] complex128
 * workspace    device, >= mbc_egraph_workspace_bytes(g, batch)
 * At most 64 tensors.  The steps run level by level (one launch per
 * dependency level, one for the sum over the terms); the device tables of a
 * batch size are built on its first use (a synchronous upload).  Sums are
 * taken in a fixed order (run-to-run reproducible). */
mbc_status mbc_egraph_execute(mbc_egraph* g, const double* const* inputs, const int64_t* batch_stride, int64_t batch,
                              double* out, void* workspace, size_t ws_bytes, void* stream);
/* Frees a graph and its device constants (NULL-safe; synchronises the device). */
void mbc_egraph_free(mbc_egraph* g);

#ifdef __cplusplus
}
#endif

#endif /* MBC_EGRAPH_H */
