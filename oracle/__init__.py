"""Plain FP64 CPU oracle for the two-site DMRG effective-Hamiltonian path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check of the
entry module and the CPU-baseline leg of the benchmark may import this
package.  The GPU library never calls it and shares no code with it; the
two meet only through the seeded problem generators of
``paper_2007_14822_amd.inputs`` (operator matrices, MPO tensors, random MPS
tensors, sector tables), which hold none of the method's arithmetic.

Every contraction is written as its plain definition with pairwise
``numpy.einsum(..., optimize=False)`` in float64, in the order the
definition states.  Iterative parts (the eigensolver, the sweep) follow the
steps of the two-site DMRG algorithm of Sec. 7.2 in order.

Modules
  tensor   labelled contraction, the "*" product of Sec. 4 with the
           integer-label interface of Sec. 9.1
  heff     environments, the two-site H_eff matvec, dense helpers
  ed       exact-diagonalisation Hamiltonians used as pins
  dmrg     truncated bond split (Sec. 5), Davidson, two-site sweeps
  qn       quantum-number indices, block enumeration, blockwise H_eff (Sec. 8)
"""
