"""Plain FP64 CPU oracle of the pseudo-transient topology-optimisation hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the GPU package may import, call or load
anything from here; only the test suite, the smoke check and the bench's CPU
baseline leg use it.  It shares no code with the HIP path: the only common
module is ``workloads`` (seeded inputs, no arithmetic of the method).

What it computes, following the paper (arXiv 2509.06971):

* ``elastic``  -- the staggered-grid linear-elastic energy, its per-cell split and
  its gradient (internal force), for the stress law of Eq. (3.9) with the Lame
  parameters of Eq. (3.10) and the momentum balance of Eq. (3.6).
* ``heat``     -- the cell-centred steady heat-conduction energy and residual of
  Eq. (2.2), with conductivity interpolation as in Eq. (3.1).
* ``assembly`` -- an independent element-by-element sparse assembly of the same
  stiffness, used for direct solves on small grids.
* ``apt``      -- the accelerated pseudo-transient (damped-wave) relaxation of
  Eqs. (2.5)-(2.6) / (3.12), the plain PT iteration of Eqs. (2.4) / (3.11), and the
  residual norm of Eqs. (3.4)-(3.5).
* ``design``   -- compliance (Eq. (2.7) / Eq. (3.7)), its sensitivity (Section 2.3),
  the normalised sensitivity step (Eqs. (3.2)-(3.3)), an explicit Allen-Cahn step
  with the double-well of Eq. (2.15), the volume projection, and the design-step
  workflow of Fig. 4.

Every floating-point operation is FP64.  Parity status of each function is stated
in its docstring; the full design trajectory has no printed values in the paper
("parity unpinned" beyond the invariants the tests check).
"""
from . import elastic, heat, assembly, apt, design  # noqa: F401
