"""Plain, slow FP64 CPU oracle for GoDec by bilateral random projection.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) imports, calls or links anything in this package; only
the tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use it.  It shares no code with the GPU path: the only thing the
two sides have in common is the seeded input generator module
(``paper_1309_0302_amd.workloads``), which holds none of the method's
arithmetic.

Modules
-------
godec_ref
    Algorithm 1 of Zhou & Tao, "Unmixing Incoherent Structures of Big Data by
    Randomized or Greedy Decomposition" (arXiv 1309.0302), step by step in
    FP64: the power-scheme BRP low-rank update (Eq. 5-9 and the projection
    update of Sec. 3.1.1), the cardinality-constrained hard threshold
    (Eq. 4), and the naive SVD GoDec of Eq. 4 used as an independent pin.
rng_ref
    An independent implementation, from their published definitions, of the
    counter-based SplitMix64 generator and the Box-Muller transform that the
    library uses to draw the random projection matrix A1 from a seed.

Pinning status (each function's docstring repeats it):
    godec_ref.brp_power        pinned (exact rank-r reproduction; LAPACK
                               truncated SVD on large-gap inputs; Thm. 3
                               bound at q = 0; invariance under A1 -> A1 T)
    godec_ref.hard_threshold   pinned (brute-force sort on tiny, tie-heavy
                               inputs; Eq. 4 optimality condition)
    godec_ref.godec_brp        pinned (trajectory equals naive SVD GoDec on
                               the 500x500 workload; Thm. 1 S-step
                               monotonicity; nnz and rank invariants)
    godec_ref.godec_naive      pinned (LAPACK SVD is the definition; exact
                               recovery of a noiseless low-rank + sparse X)
    rng_ref.a1_gaussian        pinned (SplitMix64 published test vectors;
                               moments of the Gaussian draw)
    mse_ref.mse_train          pinned (MSE training, Sec. 4.2.1 / Algorithm 4:
                               initialisation invariant; label update against
                               the printed lines, the truncated SVD and the
                               Thm. 3 bound; one-sweep recovery with disjoint
                               labels; signed brute-force top-K; label order;
                               one label = GoDec at q = 0)
"""
