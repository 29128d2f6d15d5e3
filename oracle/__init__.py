"""FP64 CPU oracle of the FR-PCPF method (Al-Salami, Kamra & Hu, arXiv 2006.10967).

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or execute this
package: only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use it. It shares no code with the GPU library (``paper_2006_10967_amd``):
it builds its own basis, operators, pairing and geometry, and it evaluates every step
with the plain dense operators of the paper's definitions (§3.1 Steps 1-6, §3.2), in
float64, vectorised over elements with torch CPU tensors so that autograd gives the exact
discrete adjoint of the whole map.

Modules
  basis      1D Gauss-Legendre nodal basis, Vandermonde, DG (Radau) correction functions
  operators  dense tensor-product element operators (interpolation, derivative, lifting)
  triangle   the triangle element: points, dense operators, geometry and pairing
  mesh       solution/flux point coordinates, slot pairing by coordinates, affine geometry
  velocity   the analytic velocity fields of §4
  residual   physical residual (§3.1) and preconditioning residual with the sensor (§3.2)
  solver     RK4, reset + pseudo-time preconditioning, the step loop, error measures (§4)

Every function whose result is not pinned to something outside itself says
"parity unpinned" in its docstring.
"""
from .basis import Basis1D
from .operators import ElementOperators
from .mesh import Discretisation
from .solver import Oracle

__all__ = ["Basis1D", "ElementOperators", "Discretisation", "Oracle"]
