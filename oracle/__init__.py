"""FP64 CPU oracle for DPG element Gram matrices on hexahedra.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the C-ABI library
and its Python binding) may import, call, link or execute anything in this
package; only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py`` use it.  It shares no code with the GPU path.

What it computes is the plain definition of the Gram matrix (2.13) for the
four inner products of the hexahedral exact sequence (2.1):

* H1      (2.28): (u, v) + (grad u, grad v)
* H(curl) (2.65): (E, F) + (curl E, curl F)
* H(div)  (2.46): (V, W) + (div V, div W)
* L2      (2.14): (q, r)

The master-element shape functions are the tensor products of Section 2.2
with the 1D hierarchical basis fixed in Section 2.8.2 (chi_i = integrated
Legendre L_i, nu_i = chi'_{i+1} = P_i, (2.54)).  They are pushed to the
physical element with the Piola maps (2.3)-(2.6) and the integrals are
taken with the L^3 tensor Gauss-Legendre rule of (2.26), i.e. the
conventional algorithm family (Algorithms 1, 4, 6, 8): every entry is
accumulated independently, no sum factorisation, no symmetry assumed.

Modules:
  poly1d        1D Legendre / integrated Legendre families, float and exact
  quadrature    Gauss-Legendre rule on (0, 1)
  geometry      trilinear and affine element maps, Jacobians
  shapes        3D shape functions and their grad / curl / div
  gram          brute-force Gram matrices (full, selected entries, mat-vec)
  closed_forms  the 1D integral chart (2.103)-(2.114) and the Kronecker
                form of Section 2.8.1 for constant Jacobians (pin source)

Readings of the paper that the oracle takes where the text is silent or
garbled are listed in each module's docstring.  Parity is pinned for
every function here (no "parity unpinned" entries): see tests/test_oracle_*.
"""

SPACES = ("H1", "HCURL", "HDIV", "L2")
