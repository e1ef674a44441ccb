"""M2P with linear FE shape functions of the fixed mesh (oracle; test infrastructure only).

Eq. (m2p) of Sec. 2.2: alpha_mu = sum_i alpha_i psi^m_i(r_mu), here with the
linear finite-element functions of the fixed mesh (App. B: pyramids of height
one at each node on a triangulation).  The Delaunay triangulation of a square
grid is degenerate (App. B notes uniqueness only "except for possible
degeneracies"); the reading taken is the fixed diagonal from (i, j) to
(i+1, j+1) in every cell:

  cell   i = min(floor((x - x0)/H), nx - 1),  j likewise in y
  local  xi = (x - x0)/H - i,  eta = (y - y0)/H - j
  xi >= eta : triangle (i,j), (i+1,j), (i+1,j+1) with weights (1-xi, xi-eta, eta)
  xi <  eta : triangle (i,j), (i+1,j+1), (i,j+1) with weights (1-eta, xi, eta-xi)
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .mesh import Mesh


def m2p_locate(mesh: Mesh, pos):
    """Node ids [N, 3], weights [N, 3] and the lower/upper flag per particle."""
    pos = np.asarray(pos, dtype=np.float64)
    mesh.check_inside(pos)
    tx = (pos[:, 0] - mesh.x0) / mesh.H
    ty = (pos[:, 1] - mesh.y0) / mesh.H
    i = np.minimum(np.floor(tx), mesh.nx - 1).astype(np.int64)
    j = np.minimum(np.floor(ty), mesh.ny - 1).astype(np.int64)
    xi = tx - i
    eta = ty - j
    lower = xi >= eta
    s = mesh.nx + 1
    n00 = j * s + i
    n10 = n00 + 1
    n11 = n00 + s + 1
    n01 = n00 + s
    nodes = np.where(lower[:, None], np.stack([n00, n10, n11], 1), np.stack([n00, n11, n01], 1))
    w = np.where(lower[:, None],
                 np.stack([1.0 - xi, xi - eta, eta], 1),
                 np.stack([1.0 - eta, xi, eta - xi], 1))
    return nodes, w, lower


def m2p(mesh: Mesh, mesh_vals, pos):
    """Eq. (m2p) with linear FE mesh functions; mesh_vals [n_nodes, C] -> [N, C]."""
    nodes, w, _ = m2p_locate(mesh, pos)
    mv = np.asarray(mesh_vals, dtype=np.float64)
    return np.einsum("nk,nkc->nc", w, mv[nodes])


def m2p_matrix(mesh: Mesh, pos):
    """Sparse interpolation matrix [N, n_nodes]; its transpose is the adjoint."""
    nodes, w, _ = m2p_locate(mesh, pos)
    N = nodes.shape[0]
    rows = np.repeat(np.arange(N), 3)
    return sp.csr_matrix((w.ravel(), (rows, nodes.ravel())), shape=(N, mesh.n_nodes))


def m2p_grad_pos(mesh: Mesh, mesh_vals, pos, gbar):
    """d/d r_mu of sum_{mu,c} gbar_mu,c alpha_mu,c: the interpolant's gradient
    on the particle's triangle (constant per triangle), dotted with gbar.

    Lower triangle: d(weights)/dxi = (-1, 1, 0), d/deta = (0, -1, 1).
    Upper triangle: d/dxi = (0, 1, -1), d/deta = (-1, 0, 1).  d/dx = (1/H) d/dxi.
    """
    nodes, _, lower = m2p_locate(mesh, pos)
    mv = np.asarray(mesh_vals, dtype=np.float64)[nodes]          # [N, 3, C]
    dxi = np.where(lower[:, None], np.array([-1.0, 1.0, 0.0]), np.array([0.0, 1.0, -1.0]))
    deta = np.where(lower[:, None], np.array([0.0, -1.0, 1.0]), np.array([-1.0, 0.0, 1.0]))
    gx = np.einsum("nk,nkc->nc", dxi, mv) / mesh.H
    gy = np.einsum("nk,nkc->nc", deta, mv) / mesh.H
    g = np.asarray(gbar, dtype=np.float64)
    return np.stack([(gx * g).sum(1), (gy * g).sum(1)], axis=1)
