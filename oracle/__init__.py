"""Reference oracle for the flux-reconstruction Navier-Stokes right-hand side
with flux anti-aliasing (Akkurt, Witherden & Vincent, "Cache Blocking for Flux
Reconstruction: Extension to Navier-Stokes Equations and Anti-aliasing").

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, unfused CPU
implementation that follows the paper's formulation step by step with dense
operator matrices (section 2.2, "Formulation in Terms of Kernels").  Only the
test-suite, the smoke check and the CPU-baseline leg of the benchmark may
import it.  The product path (the HIP library and its Python binding) never
imports, links or calls anything in here, and this package imports nothing
from the product.

Modules
-------
quadrature  Gauss-Legendre / Gauss-Lobatto / Gauss-Jacobi rules, the
            conical-product triangle, tetrahedron and pyramid rules and the
            triangle, tetrahedron and pyramid node sets.
basis       Bases of the hex, triangle, prism, tet and pyramid solution spaces.
elements    Reference elements (solution, flux and quadrature points, unit
            reference normals) and the dense operator matrices M0..M10.
mesh        Periodic box meshes of hexahedra, split prisms, tetrahedra,
            pyramids and mixtures (hex/prism, prism/tet, hex/pyramid), affine
            metric terms and flux-point pairing by physical coordinates.
physics     Inviscid / viscous fluxes, Rusanov and LDG interface fluxes.
rhs         The semi-discrete right-hand side (the paper's thirteen kernels,
            in PyFR v1.11.0 order) and classical RK4.

Precision: every routine takes the array dtype from its inputs.  The default
is float64 (the paper's precision); float32 and longdouble are used by the
tests to estimate rounding behaviour.

Parity status (pins live in tests/test_oracle_*.py):
  * quadrature, bases, operators: pinned by exactness, closed forms
    (Radau correction polynomials, SBP identities), the paper's printed
    Gauss-Legendre nodes and sum-factorisation identities.
  * rhs: pinned by free-stream preservation, discrete conservation,
    consistency/antisymmetry of the interface fluxes, axis-permutation
    symmetry, one-dimensional reduction, design-order convergence to exact
    time derivatives (entropy wave, heat conduction) and the closed-form
    initial kinetic-energy decay rate of the Taylor-Green vortex.
  * surface-flux anti-aliasing (Mesh(..., surf_aa=True)): the rebuilt lifting
    is pinned against explicit Lagrange polynomials and high-order face
    integration; the right-hand side by free stream, conservation, equality
    with the flux-point form when every interface flux is a face polynomial
    of degree <= p, and design-order convergence (test_oracle_surface_aa.py).
  * tetrahedra (RefElement("tet"), Mesh kinds "tet" and "prism_tet"): the
    conical-product rule against closed-form simplex moments, the node set's
    symmetry and unisolvence, the operator identities above, free stream,
    conservation and entropy-wave convergence (test_oracle_tet.py).
  * pyramids (RefElement("pyr"), Mesh kinds "pyr" and "hex_pyr"): the
    conical-product rule against closed-form pyramid moments, the node set's
    symmetry and unisolvence, the space (gradients, its rational members,
    polynomial face traces), the weak-form divergence taken for pyramids
    (exact for P_p fluxes, conservative), free stream, conservation and
    entropy-wave convergence (test_oracle_pyr.py).
  * curved hexahedra and prisms (Mesh kinds "hex_warp", "prism_warp",
    "mixed_warp": vertex maps of a warped grid, per-point metrics): free
    stream, conservation, the discrete metric identity, equality with the
    affine mesh at zero warp and entropy-wave convergence
    (test_oracle_curved.py).
  * The full right-hand side at a perturbed state has no closed form; it is
    pinned only through the properties above.
"""

from . import quadrature, basis, elements, mesh, physics, rhs  # noqa: F401
from .rhs import Params, rhs as compute_rhs, rk4_step  # noqa: F401
