"""Plain FP64 CPU oracle of the sliding-mesh spectral difference (SSD) method.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and
the CPU-baseline leg of the benchmark may import this package.  The product
path (the HIP library and its Python binding) never imports, calls or links
anything here, and this package imports nothing from the product.

Written from Zhang & Liang, "A simple, efficient, and high-order accurate
curved sliding-mesh interface approach to spectral difference method on
coupled rotating and stationary domains" (arXiv:1503.02198):

  basis.py     solution/flux points, Lagrange bases, mortar matrices (Sec. 3.1,
               Sec. 3.2 eqs. mortarM, mortarS)
  geometry.py  iso-parametric element maps and metrics (Sec. 2.3, Sec. 3.1)
  physics.py   inviscid, ALE and viscous fluxes, Rusanov flux (Sec. 2.1-2.2,
               Sec. 3.1)
  ssd.py       the residual, the dynamic mortars and SSP-RK3 (Sec. 3)
  exact.py     the isentropic vortex (Sec. 4.1) and Taylor-Couette (Sec. 4.2)
               exact solutions
  subgrid.py   the learned per-element correction (an extension, not in the
               paper): features, restriction of nested meshes, the MLP

Everything is vectorised numpy over elements in float64; numpy routines
(einsum, polynomial algebra, solve) serve as the library primitives.
"""
