"""Plain, slow FP64 CPU oracle for the spin-adapted two-site DMRG hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the library's product path imports, links
or calls this package; only the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may use it.  It shares no code with the
HIP path: it works on explicit Fock-space vectors (determinants with
Jordan-Wigner signs) and reaches the projected Hamiltonian action by its
definition, H_eff psi = V^T H V psi, where V embeds the two-site variational
space spanned by the MPS into the full Fock space (Sec. "Tensor network states
and density matrix renormalization group"; the Hamiltonian of Sec. "Complete
active space SCF").

Modules
  cg        exact Clebsch-Gordan coefficients (Racah's formula, rational arithmetic)
  fock      determinant space, the Hamiltonian and S^2 acting on it, FCI
  mps_fock  SU(2) MPS -> M-resolved Fock-space vectors, V and V^T
  heff      H_eff psi by definition; dense H_eff for small cases (its lowest
            eigenpair, from numpy's dense eigensolver, is the reference for
            the library's Davidson)
  truncate  Schmidt values of the two-site wavefunction, discarded weight,
            SU(2) multiplet grouping and the dynamic block state selection rule
"""
