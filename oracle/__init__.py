"""Plain FP64 CPU oracle for the two-level Schwarz / H_k-GenEO method.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The product path (the
HIP library and its Python binding) never imports, links or calls it, and this
package imports nothing from the product path: the two share no code.  The one
shared module is the seeded input generator ``paper_2406_06283_amd.problems``,
which holds the problem definition only (mesh, coefficients, element and CSR
matrices, loads) and none of the method's arithmetic.

Everything here is written for reading, not speed: each function follows one
definition of the paper (Dolean, Fry, Graham, Langer, "Overlapping Schwarz
methods with GenEO coarse spaces for indefinite and non-self-adjoint problems",
arXiv 2406.06283) and cites it.  Library primitives (sparse/dense LU,
symmetric-definite eigensolver, QZ) serve as steps; there is no blocking,
fusion or reordering beyond the definitions.

Modules:
  decomposition  Def 2.8 (overlap by element layers), Def 2.12 (dof/ovdof),
                 Def 2.13 (partition of unity), the overlap count Lambda (Sec 2.4)
  local          local Dirichlet matrices (eq. 2.22) and the H_k-GenEO local
                 eigenproblem (Def 2.14), eigenvector selection (Def 2.15)
  schwarz        one- and two-level additive Schwarz (eqs. 2.22, 2.23)
  fgmres         right-preconditioned flexible GMRES (Sec. 1, Elman theory)
  reference      direct sparse solve for error statements

Parity pins: every function is checked by tests marked ``not gpu`` against
closed forms, invariants and brute force on tiny inputs; see each module.
"""
