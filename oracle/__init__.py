"""CPU FP64 oracle for the VQE state-vector hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or
executes this package; only the test suite, the smoke check and the CPU
baseline leg of the benchmark do.  It shares no code with the GPU library:
its Jordan-Wigner mapping works on Pauli strings with a single-qubit
product table, its simulator applies one gate at a time with NumPy, and its
energy is summed term by term, which is the evaluation order of the paper
(Sec. III-D: the terms are computed individually).

Modules
  hamiltonian  fermionic H (eq. 1) -> Pauli sum (eqs. 2-4) by Jordan-Wigner
  statevector  psi(theta) = U(theta) psi_ref (eq. 6), gate by gate
  expect       <psi|P|psi> per term and E = <psi|H|psi>/<psi|psi> (eq. 7)
  grad         parameter shift, central differences, adjoint reverse sweep
  ed           exact diagonalisation and the free-fermion energy
  slim         Hamiltonian cutoff (Sec. II-D, III-D)
  closed_forms single-gate, one-layer and stabiliser-tableau results
"""
