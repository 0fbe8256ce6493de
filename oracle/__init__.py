"""The oracle: plain CPU implementations of what the tree-LQR hot path computes.

TEST INFRASTRUCTURE ONLY.  Only `tests/`, `__graft_entry__.smoke()` and the
CPU-baseline leg of `bench.py` may import anything in this package.  Nothing
here is shared with the GPU solver (no common kernels, headers, helpers or
tables); the two meet only through the seeded input generators.

Contents
  riccati     ctypes front end of tree_riccati.c, the sequential FP64 tree
              Riccati recursion (Sec. XI-A baseline; Lemma 5, eqs. (FW),
              (factor-local), (local-affine-solve), (xroot), (recover)).
  dense_kkt   the KKT system eq. (kkt) assembled densely and solved with
              LAPACK; the subtree Hessians P_i and gains K_e by brute force
              from their definitions (Thm. 1, eq. (homogeneous-subtree-value)).
  lifting     the node-control -> edge-control lifting of Sec. II-B
              (Prop. 2) and the native node-control dense KKT.
  plan        the structural-round scheduler and dependency levels of
              Sec. VII (greedy index-order selection, readiness-weighted
              Shannon-Fano-Elias sibling reductions, earliest-start levels).
  algebra     the rake fold and compress composition of Sec. IV-A written
              out literally, for the elimination-identity pins.
  ragged      per-node state and per-edge control dimensions: eq. (kkt)
              assembled densely with rectangular blocks, and the sequential
              recursion with rectangular blocks.
  adjoint     gradients of a scalar loss through the solve: the same solve
              with the seeds as right-hand side (the KKT matrix of eq. (kkt)
              is symmetric) and the outer products of each block's place in
              eq. (kkt).
"""
