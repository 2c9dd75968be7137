"""CPU FP64 oracle for the SVD-based approximate noisy-circuit simulation.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
this package; only the tests, the smoke check and the benchmark's CPU-baseline
leg do.  It shares no code with the HIP library: its own superoperators, its
own decomposition (LAPACK SVD), its own term enumeration, its own light-cone
reduction and contraction order, all in complex128 / float64.

Modules
  channels  -- matrix representation of a channel, tensor permutation, SVD split
               (Section III, "matrix representation"; Section IV, Fig. 3)
  terms     -- level-l term enumeration and weights (Section IV, Algorithm 1)
  dense     -- exact references: dense density matrix, graded density matrix
  literal   -- Algorithm 1 term by term with both networks contracted as dense
               state vectors (small n)
  network   -- Algorithm 1 term by term with one network per term, contracted
               pairwise with its own light-cone reduction and greedy order
  doubled   -- the exact baseline: the doubled (ket + bra) network with every
               noise as its full superoperator tensor, contracted pairwise
  offdiag   -- off-diagonal elements: density matrix, graded form, cross form of
               Algorithm 1's terms, bond-2 polarization targets
  factored  -- level sums as a product of per-part level polynomials when the
               network splits into independent parts
  trajectories -- the quantum-trajectories estimate (Kraus draws, one network per
               sample), the paper's main comparison
  bounds    -- Theorem 1 (contraction count; error bound in the form its proof
               actually establishes)
  estimate  -- Algorithm 1 end to end: T_u, A(l) for every l' <= l, per-term values
"""
from . import channels, terms, dense, literal, network, doubled, offdiag, factored, trajectories, bounds, estimate  # noqa: F401
