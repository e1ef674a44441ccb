"""Delaunay triangulation of the particles (test infrastructure only).

App. B builds the linear FE functions phi_mu on the Delaunay triangulation of
the particles and calls two particles neighbours when a Delaunay edge joins
them; App. A says the paper used CGAL for it.  The oracle uses Qhull through
scipy.spatial.Delaunay as the equivalent library step.

Two modes:

* ``Triangulation(pos)`` triangulates the whole cloud once (sizes up to a few
  million particles).
* ``Triangulation.local(pos, tree, point, radius)`` triangulates only the
  particles within ``radius`` of one query point and certifies every triangle
  it returns: a triangle of the local triangulation is a triangle of the global
  one when its circumdisk lies inside the gathered disk (no particle outside
  the disk can enter it), so each certified answer equals the global one.
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import Delaunay, QhullError


class GeometryError(ValueError):
    """Duplicate particles or a cloud with no triangle."""


class Triangulation:
    def __init__(self, pos: np.ndarray):
        pos = np.ascontiguousarray(pos, dtype=np.float64)
        self.pos = pos
        try:
            self.dt = Delaunay(pos)
        except QhullError as e:  # flat or too few points
            raise GeometryError(f"no Delaunay triangulation: {e}") from None
        if len(self.dt.coplanar):
            raise GeometryError("duplicate or unused particles (Qhull 'coplanar' set)")
        self.indptr, self.indices = self.dt.vertex_neighbor_vertices

    # -- combinatorics ---------------------------------------------------
    def ring(self, v: int) -> np.ndarray:
        """Delaunay neighbours of particle v (ascending ids)."""
        return np.sort(self.indices[self.indptr[v]:self.indptr[v + 1]])

    def degree(self) -> np.ndarray:
        return np.diff(self.indptr)

    def locate(self, pts: np.ndarray) -> np.ndarray:
        """Index of the triangle containing each point, -1 outside the hull."""
        return self.dt.find_simplex(np.ascontiguousarray(pts, dtype=np.float64))

    def triangle(self, s: int) -> np.ndarray:
        return self.dt.simplices[s]

    @property
    def simplices(self) -> np.ndarray:
        return self.dt.simplices

    def hull_vertices(self) -> np.ndarray:
        return np.unique(self.dt.convex_hull.ravel())


def circumcircle(P: np.ndarray):
    """Circumcentre and radius of triangles P [..., 3, 2]."""
    a, b, c = P[..., 0, :], P[..., 1, :], P[..., 2, :]
    bx, by = b[..., 0] - a[..., 0], b[..., 1] - a[..., 1]
    cx, cy = c[..., 0] - a[..., 0], c[..., 1] - a[..., 1]
    d = 2.0 * (bx * cy - by * cx)
    b2 = bx * bx + by * by
    c2 = cx * cx + cy * cy
    ux = (cy * b2 - by * c2) / d
    uy = (bx * c2 - cx * b2) / d
    centre = np.stack([ux + a[..., 0], uy + a[..., 1]], axis=-1)
    return centre, np.sqrt(ux * ux + uy * uy)


class LocalTriangulation:
    """Delaunay triangulation of the particles within ``radius`` of ``point``.

    ``ids`` maps local vertex numbers to global particle ids.  Only answers
    whose triangles are certified (circumdisk inside the gathered disk with a
    relative margin) are returned; anything else raises ``LookupError`` so the
    caller can retry with a larger radius.
    """

    def __init__(self, pos: np.ndarray, tree, point: np.ndarray, radius: float):
        self.point = np.asarray(point, dtype=np.float64)
        self.radius = float(radius)
        ids = np.sort(np.asarray(tree.query_ball_point(self.point, self.radius), dtype=np.int64))
        if ids.size < 3:
            raise LookupError("too few particles in the local disk")
        self.ids = ids
        self.pos = pos[ids]
        try:
            self.dt = Delaunay(self.pos)
        except QhullError as e:
            raise LookupError(str(e)) from None
        if len(self.dt.coplanar):
            raise GeometryError("duplicate particles in the local disk")
        self.indptr, self.indices = self.dt.vertex_neighbor_vertices
        # vertex -> incident triangles
        self._inc = [[] for _ in range(ids.size)]
        for s, tri in enumerate(self.dt.simplices):
            for v in tri:
                self._inc[v].append(s)
        self._on_hull = np.zeros(ids.size, bool)
        self._on_hull[self.dt.convex_hull.ravel()] = True
        cc, rr = circumcircle(self.pos[self.dt.simplices])
        dist = np.sqrt(((cc - self.point) ** 2).sum(-1))
        self._certified = dist + rr < self.radius * (1.0 - 1e-9)

    def _check(self, simplices) -> None:
        if not np.all(self._certified[list(simplices)]):
            raise LookupError("uncertified triangle; enlarge the disk")

    def locate_point(self) -> int:
        """Local triangle containing the query point, or -1 (outside hull)."""
        s = int(self.dt.find_simplex(self.point[None, :])[0])
        if s >= 0:
            self._check([s])
        else:
            # outside the local hull: certify that it is outside the global one
            # too, i.e. the local hull is not an artefact of the disk boundary
            # (the node would be at least radius away from other particles).
            raise LookupError("point outside the local hull")
        return s

    def ring_global(self, v_local: int) -> np.ndarray:
        # an open local fan may be closed by particles outside the disk
        if self._on_hull[v_local]:
            raise LookupError("vertex on the local hull; its fan is not certified")
        self._check(self._inc[v_local])
        loc = self.indices[self.indptr[v_local]:self.indptr[v_local + 1]]
        return np.sort(self.ids[loc])

    def triangle_global(self, s: int) -> np.ndarray:
        return self.ids[self.dt.simplices[s]]
