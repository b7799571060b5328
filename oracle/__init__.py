"""CPU FP64 oracle for Nystrom kernel filtering.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package:
it is used by ``tests/``, by ``__graft_entry__.smoke()`` and by the
``cpu_baseline`` leg of ``bench.py``, and nowhere else.  It shares no code,
constants or helpers with the HIP library.

Contents (each function cites the passage of Nair & Chaudhury, "Fast
High-Dimensional Kernel Filtering", that it follows):

* ``exact``    -- the kernel filter of Eq. (num) by brute force, the spatial
                  and range kernels (Section II, Section IV), the NLM patch guide.
* ``seeding``  -- SplitMix64 and a partial Fisher-Yates draw of distinct pixel
                  indices (k-means initialisation, which the paper leaves open).
* ``kmeans``   -- Lloyd's k-means on the range list (Section III).
* ``nystrom``  -- the landmark Gram matrix, its eigendecomposition and
                  Algorithm 1 in the paper's own alpha_k / v_k form, plus a
                  per-pixel evaluation of the same approximation before the sum
                  switch, and small dense K / K-hat matrices.
* ``recursive``-- Young and van Vliet's recursive Gaussian (Section IV's O(1)
                  Gaussian filter) with zero extension at the borders.
* ``grad``     -- an independent float64 autograd formulation (symmetric
                  A^{-1/2} form) used as the gradient reference, and central
                  finite differences.

All floating point is float64.
"""
