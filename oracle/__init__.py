"""FP64 CPU oracle for the wavelet-domain l1-l2 deblurring hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
Python binding) imports, links or calls anything in this package; only the
test-suite, the smoke check and the benchmark's CPU-baseline leg do.  It is a
plain, slow, obviously-correct restatement of the method of Escande & Weiss,
"Real-time l1-l2 deblurring using wavelet expansions of operators":

* ``filters``   Haar and Daubechies (4 vanishing moments) filters, Sec. 2.
* ``dwt``       periodic separable 2D orthogonal wavelet transform, Sec. 2.
* ``blur``      the spatially varying blur H as an integral operator, Sec. 3.1.
* ``theta``     Theta = Psi^* H Psi (Sec. 3.4, eq. for Theta) and the naive
                K-largest thresholding (Sec. 3.7).
* ``lipschitz`` power iteration for ||Theta_K||_2^2 (step size of Alg. 1).
* ``fista``     Alg. 1 and its preconditioned form Alg. 2, the objective of
                the approximate problem (Sec. 1.3), a Lasso duality gap and the
                l1 optimality conditions.
* ``precond``   Jacobi (Sec. 4.2) and SPAI (Sec. 4.3, lemma) diagonals, plus
                the per-scale grouping of the SPAI objective.
* ``lasso``     brute-force exact Lasso for tiny problems (a pin, not a method).

Every routine works in float64 with numpy/scipy and shares no code, table or
constant with the GPU library.
"""
