"""Plain FP64 CPU oracle for randomized proximal TT-ALS with TensorSketch.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package may import, call or
execute this package; only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code, tables or
constants with the HIP path: it re-derives every quantity from the paper
(Chen, Jiang, Yu, Qi, "Low-rank Tensor Train Decomposition Using TensorSketch",
arXiv 2309.08093).

Conventions (0-based throughout; the paper is 1-based):
  * A d-way tensor X with mode sizes n[0..d-1] is a flat array in the paper's
    linear order (Sec. 2.2, the bijection before the TensorSketch definition):
    index i_0 varies fastest, i.e. numpy ``order='F'``.
  * TT ranks R[0..d] with R[0] = R[d] = 1; core k has shape
    (R[k], n[k], R[k+1]) (Sec. 2.1).
  * Per sweep t and mode s a hash table h_s in [0, J) and a sign table v_s in
    {-1, +1}, both of length n[s] (Sec. 2.2, Definitions of CountSketch and
    TensorSketch; Algorithm 1 draws them once per outer iteration).

Modules:
  tables  -- seeded hash/sign tables (SplitMix64, counter based)
  sketch  -- explicit TensorSketch matrix, data sketch, interface sketch
  solve   -- proximal update, QR with sign normalisation, orthogonalisation
  als     -- one sweep of Algorithm 1, TT reconstruction, residual, metrics
  bound   -- the sketch-size bound of Corollary 3
"""
