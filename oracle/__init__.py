"""Plain, slow FP64 CPU oracle for the overlap topological charge density.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
Python binding) imports, calls or links anything here; only the tests, the
smoke check and the CPU-baseline leg of the benchmark use it.  It shares no code
with the GPU path: the two meet only in the seeded input generators of
``smpq_inputs``, which hold none of the method's arithmetic.

Everything is numpy/scipy in complex128/float64, written for a reader checking
it against the paper (Xiong, Zhang, Zou, "Evaluating topological charge density
with symmetric multi-probing method", arXiv:1901.02211):

  lattice   site indexing and periodic neighbours                 (section 2.1)
  dirac     gamma basis, Wilson kernel D_W, H_W = gamma5 D_W        (section 1, Eq. 3)
  zolotarev 14-pole Zolotarev coefficients c_0, c_i, q_i          (section 1, Eq. 4)
  lanczos   spectral bounds of |H_W| for the Zolotarev interval   (Eq. 4, bounds implied)
  mscg      multi-shift CG for (D_W^dag D_W + q_i) x_i = b          (section 2.1, Eqs. 6-8)
  probing   symmetric multi-probing colourings, modes 0/1/2       (section 2.2, Eqs. 15-19)
  charge    q(x) from point sources, SMP sources and dense eps    (Eqs. 5, 16)
  trinv     probing estimate of Tr D_W^-1, the proposed application (Conclusion)
  locality  mean block entries of D_ov against distance            (Eq. 12, Fig. 1)
  deflation exact sign on the lowest modes of H_W^2, Zolotarev on the rest

Every function names the passage it follows.  No function here is "parity
unpinned": each is checked in tests/test_oracle_*.py against closed forms,
library routines, invariants or the paper's printed integers.
"""
