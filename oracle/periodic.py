"""P2M in a periodic box (oracle; test infrastructure only).

Every run of the paper takes place in a periodic box, triangulated with
CGAL's periodic Delaunay triangulation (App. A).  The oracle forms that
triangulation as the ordinary Delaunay triangulation of the cloud tiled 3 x 3
by the box periods (Qhull through ``Triangulation``): near the box, the
triangles of the tiling are the periodic triangles, their vertices being the
images of particles across the box sides.  The construction of App. B then
runs unchanged on image positions: the linear FE functions of the triangle
holding the node, the supports ring(nu) U ring(sigma) of its edges and the
minimum-norm solutions of eqs. (A0), (A1), (A2_2), all on the positions of
the images the triangulation joins to the node.  No node is a closure node:
a periodic box has no boundary.

Readings taken here (the paper states none of them):

* The box is [x0, x0 + nx H) x [y0, y0 + ny H).  Mesh arrays keep the
  (nx+1)(ny+1) nodes of the bounded mesh: node (nx, j) is node (0, j) and
  node (i, ny) is node (i, 0), and their rows are those nodes' rows.
* A particle's image is its position plus (a Lx, b Ly), a, b in {-1, 0, 1},
  evaluated in FP64 as one addition per coordinate.
* The box must be large enough that every triangle a node uses has a unique
  set of images near it (a few particle spacings are plenty).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .delaunay import Triangulation
from .mesh import Mesh
from .qcsf import NodeStructure, interior_weights_local

# the tile shifts (a, b); the first is the box itself, so that image k < N is
# particle k
SHIFTS = ((0, 0), (-1, -1), (0, -1), (1, -1), (-1, 0), (1, 0), (-1, 1), (0, 1), (1, 1))


def box_lengths(mesh: Mesh):
    return mesh.nx * mesh.H, mesh.ny * mesh.H


def tiled(pos: np.ndarray, mesh: Mesh):
    """The cloud and its eight translates by the box periods.

    Returns (images [9N, 2], particle id of each image [9N])."""
    Lx, Ly = box_lengths(mesh)
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    n = len(pos)
    parts = []
    for a, b in SHIFTS:
        parts.append(np.stack([pos[:, 0] + a * Lx, pos[:, 1] + b * Ly], axis=1))
    return np.concatenate(parts, axis=0), np.tile(np.arange(n, dtype=np.int64), len(SHIFTS))


def wrapped_nodes(mesh: Mesh) -> np.ndarray:
    """Node positions with the last column and row taken as the first."""
    i = np.arange(mesh.nx + 1) % mesh.nx
    j = np.arange(mesh.ny + 1) % mesh.ny
    X = mesh.x0 + i.astype(np.float64)[None, :] * mesh.H
    Y = mesh.y0 + j.astype(np.float64)[:, None] * mesh.H
    X, Y = np.broadcast_arrays(X, Y)
    return np.stack([X.ravel(), Y.ravel()], axis=1)


def check_in_box(pos: np.ndarray, mesh: Mesh) -> None:
    Lx, Ly = box_lengths(mesh)
    if not np.all(np.isfinite(pos)):
        raise ValueError("non-finite particle position")
    bad = ((pos[:, 0] < mesh.x0) | (pos[:, 0] >= mesh.x0 + Lx) |
           (pos[:, 1] < mesh.y0) | (pos[:, 1] >= mesh.y0 + Ly))
    if np.any(bad):
        raise ValueError(f"{int(bad.sum())} particle(s) outside the periodic box")


class PeriodicP2MOracle:
    """Rows psi_mu(r_i) of every mesh node in a periodic box (eq. p2m)."""

    def __init__(self, pos, mesh: Mesh, h: float):
        self.pos = np.ascontiguousarray(pos, dtype=np.float64)
        self.mesh = mesh
        self.h = float(h)
        check_in_box(self.pos, mesh)
        self.images, self.origin = tiled(self.pos, mesh)
        self.tri = Triangulation(self.images)

    def node_weights(self):
        """(cols, vals, image ids, info) per node: cols are particle ids,
        image ids the tiled vertices they came from."""
        nodes = wrapped_nodes(self.mesh)
        s = self.tri.locate(nodes)
        if np.any(s < 0):
            raise ValueError("a node outside the tiled triangulation")
        triangles = [self.tri.triangle(t) for t in s]
        st = NodeStructure.build(triangles, self.tri.ring)
        P = self.images[st.U]
        w, rank, sig = interior_weights_local(P, st.tri, st.member, st.valid, nodes)
        cols, vals, imgs = [], [], []
        for q in range(len(nodes)):
            m = st.valid[q]
            imgs.append(st.U[q][m])
            cols.append(self.origin[st.U[q][m]])
            vals.append(w[q][m])
        info = {"closure": np.zeros(len(nodes), bool), "edge_rank": rank, "edge_sigma": sig,
                "triangle": self.origin[np.asarray([np.asarray(t) for t in triangles])]}
        return cols, vals, imgs, info

    def matrix(self):
        """Sparse P2M matrix W [n_nodes, N] and the info dict."""
        cols, vals, imgs, info = self.node_weights()
        indptr = np.zeros(len(cols) + 1, np.int64)
        indptr[1:] = np.cumsum([len(c) for c in cols])
        W = sp.csr_matrix((np.concatenate(vals), np.concatenate(cols), indptr),
                          shape=(len(cols), len(self.pos)))
        W.sum_duplicates()
        info["images"] = imgs
        return W, info

    def project(self, vals):
        W, _ = self.matrix()
        return W @ np.asarray(vals, dtype=np.float64)


CS_STEP = 1e-30


def periodic_p2m_grad_pos(orc: PeriodicP2MOracle, vals, gbar_mesh):
    """d/d r of L = sum_{i,c} gbar[i,c] (P2M vals)[i,c] in the periodic box
    (positions only; the triangulation held fixed).

    An image moves with its particle, so the derivative with respect to an
    image position is added to that particle.  Derivatives by complex step of
    the forward construction (normal-equation form of the minimum-norm solve,
    which is holomorphic), as for the bounded box."""
    vals = np.asarray(vals, dtype=np.float64)
    g = np.asarray(gbar_mesh, dtype=np.float64)
    nodes = wrapped_nodes(orc.mesh)
    s = orc.tri.locate(nodes)
    st = NodeStructure.build([orc.tri.triangle(t) for t in s], orc.tri.ring)
    pid = orc.origin[st.U]
    wbar = np.where(st.valid, np.einsum("nkc,nc->nk", vals[pid], g), 0.0)
    P = orc.images[st.U].astype(np.complex128)
    r = nodes.astype(np.complex128)
    grad = np.zeros_like(orc.pos)
    for k in range(st.U.shape[1]):
        for d in range(2):
            Pc = P.copy()
            Pc[:, k, d] += 1j * CS_STEP
            w = interior_weights_local(Pc, st.tri, st.member, st.valid, r, solver="normal")
            contrib = (wbar * (w.imag / CS_STEP)).sum(1)
            m = st.valid[:, k]
            np.add.at(grad[:, d], pid[m, k], contrib[m])
    return grad
