"""CPU oracle for the nonuniform discrete Hankel transform.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, FP64 reference the
GPU library is checked against.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import it; the GPU library never does, and the
two share no code.

Layers (Beckman & O'Neil, "A Nonuniform Fast Hankel Transform"):

* :mod:`oracle.direct`    -- O1, the direct O(nm) sum g_j = sum_k c_k J_nu(w_j r_k)
                             (Sec. 1, eq. DHT) with its own J_nu evaluator.
* :mod:`oracle.params`    -- the expansion parameters M, z, L (Sec. 3.3, Lemma 3.1,
                             eq. asy-error, eq. num-asy-terms).
* :mod:`oracle.partition` -- the staircase and Alg. 1 (Subdivide) of Sec. 4.1.
* :mod:`oracle.method`    -- O2, the method-exact reference: Alg. 2 with every
                             block applied by its expansion summed directly (no NUFFT).
"""
