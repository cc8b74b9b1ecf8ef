"""Plain FP64 CPU oracle for the THC-oo-K exchange build.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or
link this package: only the test suite, the smoke check and the CPU-baseline
leg of the benchmark use it. It shares no code with the HIP path; the two
meet only in the seeded input generator ``synth``.

Contents (Rettig, Lee, Head-Gordon, "Even Faster Exact Exchange for Solids
via Tensor Hypercontraction"):

* ``coulomb``  -- the periodic Coulomb kernel 4 pi/|G+q|^2 on the FFT box and
  the pair Coulomb integral evaluated by FFT (GPW, Sec. 2.1 after Eq. 9 and
  Sec. 3).
* ``direct``   -- O1: exact k-point exchange (Eq. 2) by one FFT-Poisson
  solve per occupied pair density; energy and AO-basis K^k.
* ``thc``      -- O2: THC-oo-K (Sec. 2.3, Eqs. 16-18, Algorithm 2) with one
  occupied-pair ISDF fit per momentum transfer q, written step by step with
  direct O(N_k^2) k-sums.
* ``select``   -- interpolation-point selection by pivoted Cholesky of the
  pair Gram matrix (QR with column pivoting, Sec. 2.1 after Eq. 5).

Parity status: every function is pinned by the CPU tests in
``tests/test_oracle_*.py`` except the absolute ISDF error at a given N_ISDF,
which the paper only shows in figures ("parity unpinned": reported, never
gated).
"""
