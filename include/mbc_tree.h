/*
 * mbc_tree.h -- linearised factor trees over arbitrary factor sets (C ABI, gfx950).
 *
 * Sec. 4 of Humphrey, Detmold, Young and Zanotti (arXiv:2201.04269) writes a
 * sum of products sum_k w_k prod_i F_{k,i} as a tree: every term is a
 * root-to-leaf path whose vertices carry its factors, and terms that begin
 * with the same factors share those vertices.  The linearised form is three
 * arrays in depth-first order of the vertices:
 *
 *   factors[v]       the factor of vertex v: an index into a table of factor
 *                    values (-1 for the root, vertex 0, and only there)
 *   children[v]      the number of children of vertex v
 *   coefficients[l]  the coefficient of the l-th leaf in depth-first order
 *
 * The value of the tree is the sum over root-to-leaf paths of the leaf's
 * coefficient times the product of the factor values on the path; bottom
 * up, a vertex's value is its factor's value times the sum of its children's
 * values (a leaf: times its coefficient).  Any factor set fits: blocks,
 * minors, matrix entries; the factor values are a caller table, evaluated for
 * a batch of independent tables at once.  (mbc_blocks.h evaluates the trees
 * of block-level correlators with a kernel specialised to block products.)
 *
 * Errors, streams and ownership are as in mbc.h.
 */
#ifndef MBC_TREE_H
#define MBC_TREE_H

#include "mbc.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mbc_factor_tree mbc_factor_tree; /* opaque, owns its device arrays */

/* Validates the linearised arrays and uploads them to the current device on
 * `stream` (synchronised before return).
 * factors, children  host [n_vertices]; coefficients host [n_leaves][2]
 *                    (re, im); n_values: size of the factor-value table.
 * MBC_ERR_INVALID unless the arrays describe exactly one tree in depth-first
 * order (the root's children and their subtrees consume all n_vertices
 * vertices), the root alone has factor -1, every other factor is in
 * [0, n_values), and the number of leaves (non-root vertices without
 * children) is n_leaves. */
mbc_status mbc_factor_tree_create(const int32_t* factors, const int32_t* children, int64_t n_vertices,
                                  const double* coefficients, int64_t n_leaves, int32_t n_values, void* stream,
                                  mbc_factor_tree** out);
/* Tree statistics (any output may be NULL): depth (the root has depth 0) and
 * the flops of one evaluation (8 per non-root vertex: its factor times its
 * children's sum, added into its parent). */
mbc_status mbc_factor_tree_stats(const mbc_factor_tree* t, int32_t* depth, double* flops);
/* Device workspace of mbc_factor_tree_evaluate for `batch` tables. */
mbc_status mbc_factor_tree_workspace_bytes(const mbc_factor_tree* t, int64_t batch, size_t* bytes);
/* The tree's value for each of `batch` factor tables.
 * values     device [batch][n_values] complex128 (re/im interleaved)
 * out        device [batch] complex128
 * workspace  device, >= mbc_factor_tree_workspace_bytes(t, batch)
 * Launches per depth level, deepest first; a vertex with many children is
 * summed by a wavefront in a fixed order, the others by one thread in
 * depth-first order (run-to-run reproducible). */
mbc_status mbc_factor_tree_evaluate(const mbc_factor_tree* t, const double* values, int64_t batch, double* out,
                                    void* workspace, size_t ws_bytes, void* stream);
/* Destroys a tree (NULL-safe); synchronises the device first. */
void mbc_factor_tree_destroy(mbc_factor_tree* t);

#ifdef __cplusplus
}
#endif

#endif /* MBC_TREE_H */
