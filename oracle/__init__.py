"""CPU oracle for DROT (Douglas-Rachford splitting for optimal transport).

TEST INFRASTRUCTURE ONLY: only the tests, the package's smoke check and the
benchmark's CPU-baseline leg may import anything from here.  The oracle shares
no code with the GPU implementation and neither imports the other.

Modules
-------
ref      ctypes wrapper of drot_ref.c: plain FP64 Algorithm 1 + stopping test.
dr3      the literal three-matrix DR iteration (X, Z, Y) with the closed-form
         projection of Lemma 2, for tiny sizes.
exact    exact optima by definition: brute force over permutations, the 1-D
         monotone coupling, m = 1 / n = 1, separable costs, LP (HiGHS) and
         linear_sum_assignment.
certify  certified bracket LB <= OPT <= UB from a dual vector (c-transform)
         and a primal plan (rounding onto the transport polytope).
"""
