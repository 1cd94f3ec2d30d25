"""CPU oracle for the condensed-KKT solves -- TEST INFRASTRUCTURE ONLY.

This package is the slow, plain FP64 reference that the HIP library is
checked against.  Only the test-suite, the entry module's ``smoke()`` check
and the benchmark's ``cpu_baseline`` leg may import it.  The product path
(the C-ABI library and its Python binding) never imports, links or runs
anything in here, and this package never imports the product path.

Modules
-------
``dense``   dense numpy forms of every matrix in the paper's Sec. 2.2 / Sec. 3
            (K2, K1, K, K_gamma, K_tau), brute-force solves, inertia,
            the HyKKT algorithm step by step (Cholesky + CG, Sec. 3.1).
``sparse``  scipy.sparse forms for the large workloads: the unassembled
            FP64 operator, residual certificates, direct solves (SuperLU as
            the library primitive) with FP64 Richardson refinement.
``exact``   rational (``fractions.Fraction``) Gaussian elimination used to
            write the golden fixtures under ``tests/golden``.

Every function cites the passage of the paper it follows.  Pins (tests
that tie this code to something other than itself) live in
``tests/test_oracle_pins.py``; no function here is "parity unpinned".
"""
