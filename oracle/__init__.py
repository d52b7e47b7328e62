"""FP64 CPU oracle for sketching-based recompression of Tucker-tensor sums.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously correct
statement of what the hot path computes, used to check the GPU library.  Only
the test suite, the smoke check and the benchmark's CPU-baseline leg may import
it.  It shares no code with the GPU path, and the GPU path never calls it.

Contents (each function cites the passage of the paper it follows):
  philox      Philox4x32-10 counter generator (Salmon et al., SC'11)
  omega       seeded Gaussian test matrices Omega_k (Box-Muller, BF16-exact)
  tensor      unfolding, fold, TTM, Kronecker and Khatri-Rao products,
              Tucker-to-dense (Section 2.1, Section 2.2, Proposition 1)
  sketch      dense and structured sketches Y_n (Section 3.1, Algorithms 4/5)
  recompress  thin QR with sign fix, core projection, reconstruction,
              sketch sizes (Section 3.2-3.3, Algorithms 3/4/5)
  adjoint     loss and hand adjoint of the recompression (derived)
"""

