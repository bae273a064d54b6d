"""FP64 CPU oracle for the LNO fragment solve (test infrastructure only).

This package is a plain, slow reference used by the tests, by the smoke check
and by the CPU-baseline leg of the benchmark.  The library under
``paper_2407_11258_amd`` never imports, links or calls anything here, and
nothing here imports that library.

Contents
  integrals  -- (pq|rs) blocks from three-index DF factors (Eq. 27a)
  ccsd       -- closed-shell CCSD on the fragment Hamiltonian (Eq. 10, the
                step "CCSD with the fragment Hamiltonian" of Sec. II.B),
                MP1 amplitudes / MP2 energy (Eq. 21 with i_F running over all
                occupied), correlation energy (Eq. 7 with tau = t2 + t1 t1)
  triples    -- the (T) energy from the intermediates of SI Sec. S1 and the
                pair energy of Eq. 16 summed at i = i'
  brute      -- determinant-space definitions used to pin the above:
                <mu| e^{-T} H e^{T} |HF>, FCI for two electrons and the
                perturbative triples as a sum over triply excited determinants
"""
