"""Plain, slow CPU FP64 oracle for particle <-> fixed-mesh projection.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path imports, calls or links
anything in this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library (no kernels, headers, helpers, tables or pre/post-processing); the two
meet only in the seeded input generators of ``workloads``.

What it computes (Duque & Espanol, "Rapid convergence for simulations that
project from particles onto a fixed mesh"):

* P2M, eq. (p2m) of Sec. 2.2: alpha_i = sum_mu alpha_mu psi_mu(r_i) with the
  quadratically consistent particle shape functions of App. B, eq. (phiquad):
  psi_mu = phi_mu + sum_{nu sigma} A_{mu nu sigma} phi_nu phi_sigma, where
  phi are linear FE functions on the particles' Delaunay triangulation and the
  A coefficients of each Delaunay edge solve eqs. (A0), (A1), (A2_2) in the
  minimum-norm sense (SVD with rank detection, App. A).
* M2P, eq. (m2p) of Sec. 2.2: alpha_mu = sum_i alpha_i psi^m_i(r_mu) with
  linear FE functions on the fixed uniform mesh.
* Derivatives of both (by transposition for the linear parts, by complex-step
  differentiation of the forward construction for the position dependence).
* The kinematic loop of the paper's transport tests (``advect``): particles
  moved by a prescribed velocity (explicit midpoint rule), their functions
  rebuilt, M2P and P2M every step.
* P2M in the periodic box of the paper's runs (``periodic``): the Delaunay
  triangulation of the cloud tiled by the box periods, the same construction
  on image positions, no closure nodes.

Library routines serve as steps where the paper itself used one: Qhull
(scipy.spatial.Delaunay) for the Delaunay triangulation the paper built with
CGAL, LAPACK SVD (numpy.linalg.svd) for the small solves the paper did with an
Eigen SVD, and a k-d tree for nearest-neighbour queries.

Readings of points the paper leaves open are documented beside the code that
takes them (bounded domain; closure weights at boundary-ring and outside-hull
nodes; support of each edge's coefficients; ordered-pair sum; minimum norm).
"""

from .mesh import Mesh, DomainError  # noqa: F401
from .delaunay import Triangulation, GeometryError  # noqa: F401
from .qcsf import (  # noqa: F401
    edge_system,
    min_norm_svd,
    min_norm_normal,
    barycentric,
    interior_weights_local,
    closure_weights_local,
    NodeStructure,
    P2MOracle,
    CLOSURE_K,
)
from .m2p import m2p_locate, m2p, m2p_matrix, m2p_grad_pos  # noqa: F401
from .periodic import PeriodicP2MOracle  # noqa: F401
