"""Reference oracle for the face-based ghost penalty y = G(gamma) u.

TEST INFRASTRUCTURE ONLY. Nothing on the product path may import, call or
execute anything in this package: only the tests, the smoke check and the
CPU-baseline leg of the benchmark use it.  It shares no code, tables,
headers or helpers with the HIP library.

What it computes is the plain definition of the ghost penalty of §2.2
(the bilinear form g_F summed over the face set of Fig. 1), assembled face by
face by Gauss quadrature of directly differentiated Lagrange polynomials in
physical coordinates.  It does NOT use the Kronecker factorisation of §2.4 or
the sum-factorised three-step apply of §2.5.1; those are what the GPU path
implements and what the oracle checks.

Two further operators are checked the same way, each from its own definition:
  * the macro-patch stabilisation, the alternative form named in §2.2: the patch integral of the
    difference of the two cells' polynomial extensions (macro.py);
  * the Laplacian on the cells the boundary does not cut: the cell term of §2.1, with the dense cell
    stiffness by quadrature (cell.py).

Modules
  basis     1D nodes, Lagrange polynomials, quadrature (mpmath, 60 digits)
  mesh      cell classification, ghost-face set, lattice numbering
  patch     dense two-cell patch matrix of one face, by quadrature
  macro     dense patch matrix of the macro-patch stabilisation, by quadrature
  cell      dense cell stiffness and the Laplacian on the inside cells
  operator  global apply, sparse assembly, gradients, lumped mass, CG

Parity status: every function is pinned by the CPU tests (closed forms,
invariants, brute force); none is "parity unpinned" except the CG solution
vector beyond its residual (see cg_reference).
"""

from . import basis, mesh, patch, macro, operator, cell  # noqa: F401
