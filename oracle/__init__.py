"""CPU oracle for the directional-preconditioned CFIE solve (test infrastructure).

Plain, slow, float64 numpy/scipy code written from the paper and from the
textbook formulas it relies on.  It exists only to check the HIP library:
only the test suite, the smoke check and the bench's CPU-baseline leg may
import it.  It shares no code with the HIP path; both take their inputs from
the seeded generators in `synth`.

Modules
  special   Hankel functions (scipy as a library primitive) and constants
  nystrom   Kress product quadrature, Maue form of the hypersingular operator,
            dense CFIE assembly, plane-wave data, off-surface field evaluation
  disk      closed forms on the unit disk (eigenvalues, series solutions)
  gmres     textbook restarted GMRES
  precond   the directional preconditioner of Sec. 2 (dense reference)

Parity status of each function is stated in its docstring; every function
here is pinned by a test under tests/ against a closed form, an independent
quadrature, an invariant or a library routine.
"""
