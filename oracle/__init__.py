"""CPU reference (oracle) for the block-sparse PINVIT hot path.  TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke entry point and the benchmark's CPU-baseline leg may
import this package.  The GPU library never calls it and shares no code with it.

Everything here is plain float64 NumPy on full occupation-number vectors of length
2^L (orbital i of the paper is bit i-1 of the index), so it is limited to small L
(about 16).  It follows the paper directly:

* ``fock``    -- Jordan-Wigner annihilation/creation operators (Section 1.1, eq. for
                 a_i and its elementary components), the Hamiltonian (Section 1.1,
                 eq. hamil) applied by its definition, exact diagonalisation of the
                 N-particle sector (eq. Hevp).
* ``tt``      -- particle-number sector blocks of the matricisations (Section 2.3),
                 sequential TT-SVD truncation trunc_eps with a rank cap (Section 2.2,
                 eq. ttsvdquasiopt), block tables rho_{k,n}.
* ``precond`` -- exponential sum S(t) (Thm. expsum), the auxiliary diagonal theta_i
                 (Section 7.1.1), S = alpha_0 S(D/t_min) as a sum of rank-one diagonal
                 terms (Section 4.3), the sorted sequential sum of Lemma truncr.
* ``bounds``  -- a-posteriori quantities of Section 5.4 (b_delta, eq. everrbound).
* ``pinvit``  -- Algorithm 2 (perturbed inverse iteration) in the physical variable
                 psi = S x; Algorithm 3 (outer iteration) on top of it.
* ``subspace`` -- Algorithm 4 (perturbed inverse subspace iteration, Section 6) on D
                 columns kept as separate vectors.
* ``zform``   -- Algorithm 2 on the paper's own variable x: products with A and E summed
                 term by term (eq. exactrq), the residual as the sorted sum of its
                 M^2 terms (Lemma truncr).
* ``learned`` -- learned correction of the preconditioner's diagonal theta_i per (site,
                 particles before it): network forward and backward, Adam training on
                 the misfit to the exact diagonal (an extension, not in the paper).
* ``mps``     -- contraction of an exported block-sparse MPS to its dense vector
                 (eq. mps with the block structure of eq. blockstructure).

Parity status of each function is stated in its docstring; every function is pinned
by a ``-m "not gpu"`` test unless it says "parity unpinned".
"""
