"""FP64 CPU oracle for the Poisson coefficient-inversion hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this
package: only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg
of ``bench.py`` use it.  It shares no code with the HIP library; the only
thing both sides consume in common is the seeded input generator in
``synth``.

The oracle is plain and slow on purpose: finite-element matrices are
assembled element by element from vertex coordinates, linear systems are
solved with sparse direct factorizations (SuperLU), and every algorithm of
the paper is written out in the paper's order and notation.

Modules:
  mesh     -- structured right-diagonal triangulation, element assembly of
              A(m), M, K_Theta, boundary mass, observation operator B,
              rectangular mass factor C_M (Appendix C).
  p2       -- quadratic (P2) state space on the same triangles: the state
              discretization of the paper's Poisson experiment (Sec. 5.1).
  model    -- forward, cost, adjoint, gradient, incremental forward/adjoint,
              Hessian action, bilaplacian prior R and R^{-1}, prior sampling
              (Sec. 2, Sec. 4.3, Sec. 5.1 and Appendix A).
  newton   -- inexact Newton-CG with Eisenstat-Walker, Steihaug and Armijo
              (Algorithm 1).
  lowrank  -- double-pass randomized generalized eigensolver (Algorithm 2),
              PreCholQR (Algorithm 4), posterior sampling (Sec. 4.3.2).

Parity status: every function is pinned by a test in tests/test_oracle_*.py
against closed forms, special cases, finite differences or brute force.
"""
