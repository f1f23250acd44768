"""CPU oracle for lowest-order edge-element assembly (test infrastructure only).

This package is the slow, plain reference that the GPU library is checked
against. It is used only by the test suite, by the smoke check and by the
benchmark's CPU-baseline leg; the library itself never imports, links or calls
it, and it shares no code with the library.

What it computes (Anjam & Valdman, "Fast MATLAB assembly of FEM matrices in 2D
and 3D: Edge elements"):

* ``reference``  -- reference elements, the printed reference bases of the
  Raviart-Thomas (Section 2.1) and Nedelec (Section 2.2) elements, their
  div/curl, and a conical-product Gauss-Legendre quadrature on the reference
  triangle / tetrahedron.
* ``topology``   -- global edge/face numbering (rows of edges2nodes /
  faces2nodes are the global degrees of freedom, Section 3) and the orientation
  sign data (Section 2.3, Section 3).
* ``assembly``   -- local mass and stiffness matrices by quadrature of the
  Piola-mapped, sign-adjusted reference basis (Section 2.4), summed element by
  element into a CSR matrix with explicit zeros kept.
* ``gradient``   -- derivative of L = u^T (K(a) + M(b)) u with respect to the
  per-element coefficients (exact) and to the vertex coordinates (complex-step
  differentiation of the per-element quadrature).

Every function is pinned by tests against quantities the paper or the
mathematics fixes (printed table sizes, Euler's formula, exact rational
integrals, de Rham identities, constant-field identities, finite differences).
"""
from . import reference, topology, assembly, gradient  # noqa: F401
from .assembly import assemble, assemble_rows, local_matrices, element_dofs  # noqa: F401
from .topology import build_topology  # noqa: F401
