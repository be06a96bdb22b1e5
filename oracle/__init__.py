"""Plain FP64 CPU oracle for the enriched-finite-element (EFE) residual
Chebyshev eigensolver and its SCF support.

THIS PACKAGE IS TEST INFRASTRUCTURE.  Only the test-suite, the smoke check in
``__graft_entry__`` and the ``cpu_baseline`` leg of ``bench.py`` may import it.
The GPU library never calls it and shares no code with it: the two sides only
share seeded inputs (atom positions, random blocks), produced by
``paper_2607_06848_amd.workloads``, which holds none of the method's arithmetic.

Every function follows a passage of the paper (Sircar, Kanungo, Das, Gavini,
"Large-scale pseudopotential DFT calculations using orthogonalized enriched
finite element basis"); the passage is cited in the docstring by section and
equation.  Where the paper is silent or garbled the reading taken is stated in
the docstring.

Modules
  fe       spectral hexahedral elements: GLL/Gauss rules, Lagrange basis,
           mesh tables, lumped mass, cell matrices, assembled CFE operators.
  psp      the synthetic Gaussian pseudopotential, projector, smeared charge
           and atomic density used by the workloads.
  enrich   enrichment functions, orthogonalization against the CFE space,
           overlap/Hamiltonian blocks, Kleinman-Bylander projectors, and the
           explicit EFE matrices H^E, M^E and the approximate inverse of M^E.
  eigen    Chebyshev polynomials, standard and residual Chebyshev filters,
           Rayleigh-Ritz, Lanczos bound, multi-pass driver, dense reference.
  scf      density, Fermi level, PW92 LDA, Poisson by CG, energy, Anderson.
  learned  superposition-of-atomic-densities guess, descriptors and the MLP
           (forward, backward, Adam) of the learned initial density.

Parity pins: see tests/test_oracle_*.py.  Functions without an independent
pin are marked "parity unpinned" in their docstring.
"""
