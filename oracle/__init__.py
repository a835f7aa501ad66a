"""Plain FP64 CPU oracle for multi-baryon two-point correlators.

TEST INFRASTRUCTURE ONLY.  Nothing in the library imports, links or calls this
package; only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py`` may use it.  It shares no code with the GPU path: its
operator algebra, index-set construction, determinants, permanents and
gradients are written here from the paper (Humphrey, Detmold, Young, Zanotti,
"Novel Algorithms for Computing Correlation Functions of Nuclei",
arXiv:2201.04269), with NumPy/LAPACK as the only numerical library.

Modules
-------
gamma        Euclidean Dirac-basis gamma matrices, C, C*gamma5, P+- (Sec. 1).
operators    Baryon and multi-baryon sink tensors (Sec. 1, eq. "ops"), flavour
             separation, canonical (symmetrised) and raw index sets (eq. 1).
wick         Brute-force Grassmann Wick contraction of one (sink term, source
             term) pair, straight from the definition of the expectation in
             eq. 1; used to pin the determinant form.
correlator   Determinant-form correlator C[t], sum of |Wick terms| A[t], and
             the gradients dC/dW, dC/dS (Jacobi's formula with explicit
             cofactors).
blocks       Hadron blocks with sink momentum projection (Sec. 2), the
             block-level correlator by the partition sum of Wick's theorem
             (Sec. 3), a site-labelled determinant brute force that pins it,
             and the multiplicity count of the expanded form (Sec. 3, Fig. 2).
factor_tree  Linearised factor trees (Sec. 4): prefix-tree construction of a
             sum of products and its depth-first evaluation.
egraph       Tensor e-graphs (Sec. 5): canonical forms of tensor products under
             signed slot symmetries (brute force), the e-graph (union-find,
             class map, hash-cons) with the paper's two re-write conditions,
             extraction and plan evaluation, and block-level correlators
             written as sums of tensor expressions.

Every function documents the passage it follows.  Where the paper is silent the
reading used is stated in the docstring.
"""
