"""M2P with quadratically consistent MESH shape functions (oracle; test
infrastructure only).

App. B's construction applied to the fixed mesh instead of the particles:

  psi^m_i(r) = phi^m_i(r) + 2 sum_{edges e = (nu, sigma) of T} phi^m_nu(r) phi^m_sigma(r) A^m_{i e}

for r in the mesh triangle T, with phi^m the mesh's linear FE functions on the
fixed-diagonal triangulation (the reading taken in ``m2p``) and, for each mesh
edge e, A^m_{. e} the minimum-norm solution (SVD with rank detection, App. A)
of eqs. (A0), (A1), (A2_2) over S_e = ring(nu) U ring(sigma), where ring(v)
is v and its neighbours in that triangulation: (i +- 1, j), (i, j +- 1),
(i + 1, j + 1), (i - 1, j - 1), those inside the mesh.  The coefficients
depend on the mesh only.  M2P, eq. (m2p): alpha_mu = sum_i alpha_i psi^m_i(r_mu).

All arithmetic is FP64.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .m2p import m2p_locate
from .mesh import Mesh
from .qcsf import edge_system, min_norm_svd

# offsets of the neighbours of a node in the fixed-diagonal triangulation
RING = ((1, 0), (-1, 0), (0, 1), (0, -1), (1, 1), (-1, -1))


def ring(mesh: Mesh, v: int):
    """Node v and its neighbours inside the mesh, as node ids."""
    s = mesh.nx + 1
    i, j = v % s, v // s
    out = [v]
    for di, dj in RING:
        a, b = i + di, j + dj
        if 0 <= a <= mesh.nx and 0 <= b <= mesh.ny:
            out.append(b * s + a)
    return out


def edge_coefficients(mesh: Mesh, edges):
    """A^m of the given edges [E, 2] (node ids): (support ids [E, K] padded with
    the first id, valid [E, K], A [E, K], rank [E])."""
    edges = np.asarray(edges, dtype=np.int64)
    sups = [np.unique(np.array(ring(mesh, int(a)) + ring(mesh, int(b)))) for a, b in edges]
    K = max(len(u) for u in sups)
    E = len(edges)
    U = np.zeros((E, K), np.int64)
    valid = np.zeros((E, K), bool)
    for e, u in enumerate(sups):
        U[e, :len(u)] = u
        U[e, len(u):] = u[0]
        valid[e, :len(u)] = True
    nu = np.array([np.searchsorted(sups[e], edges[e, 0]) for e in range(E)])
    sg = np.array([np.searchsorted(sups[e], edges[e, 1]) for e in range(E)])
    P = mesh.nodes()[U]
    M, b = edge_system(P, nu, sg, valid)
    A, rank, _ = min_norm_svd(M, b, valid.sum(-1))
    return U, valid, np.where(valid, A, 0.0), rank


def m2p_qcsf_matrix(mesh: Mesh, pos):
    """Sparse [N, n_nodes] matrix of psi^m_i(r_mu)."""
    nodes, phi, _ = m2p_locate(mesh, pos)
    N = len(nodes)
    pairs = ((0, 1), (1, 2), (0, 2))
    ends = np.stack([np.sort(np.stack([nodes[:, p], nodes[:, q]], 1), 1) for p, q in pairs], 1)  # [N, 3, 2]
    uniq, inv = np.unique(ends.reshape(-1, 2), axis=0, return_inverse=True)
    U, valid, A, _ = edge_coefficients(mesh, uniq)
    inv = inv.reshape(N, 3)
    rows, cols, vals = [np.repeat(np.arange(N), 3)], [nodes.ravel()], [phi.ravel()]
    for k, (p, q) in enumerate(pairs):
        c = 2.0 * phi[:, p] * phi[:, q]                       # [N]
        e = inv[:, k]
        rows.append(np.repeat(np.arange(N), U.shape[1]))
        cols.append(U[e].ravel())
        vals.append((c[:, None] * A[e]).ravel())
    W = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, mesh.n_nodes))
    W.sum_duplicates()
    return W


def m2p_qcsf(mesh: Mesh, mesh_vals, pos):
    """Eq. (m2p) with the mesh's quadratically consistent shape functions."""
    return m2p_qcsf_matrix(mesh, pos) @ np.asarray(mesh_vals, dtype=np.float64)


def m2p_qcsf_periodic_matrix(mesh: Mesh, pos):
    """Sparse [N, n_nodes] matrix of psi^m_i(r_mu) in the periodic box.

    The mesh tiled 3 x 3 by the box periods: every edge a particle of the box
    uses is then an interior edge of the tiled mesh, with the periodic box's
    support (the rings wrapped across the sides), and its columns are folded
    back onto node (i mod nx, j mod ny) of the box (the repeated last column
    and row get none)."""
    Lx, Ly = mesh.nx * mesh.H, mesh.ny * mesh.H
    ext = Mesh(3 * mesh.nx, 3 * mesh.ny, mesh.H, mesh.x0 - Lx, mesh.y0 - Ly)
    W = m2p_qcsf_matrix(ext, pos)
    k = np.arange(ext.n_nodes)
    I, J = k % (ext.nx + 1), k // (ext.nx + 1)
    col = ((J - mesh.ny) % mesh.ny) * (mesh.nx + 1) + (I - mesh.nx) % mesh.nx
    F = sp.csr_matrix((np.ones(ext.n_nodes), (k, col)), shape=(ext.n_nodes, mesh.n_nodes))
    return (W @ F).tocsr()


def m2p_qcsf_periodic(mesh: Mesh, mesh_vals, pos):
    """Eq. (m2p) with the mesh's quadratically consistent shape functions in
    the periodic box (mesh values repeat the first column and row)."""
    return m2p_qcsf_periodic_matrix(mesh, pos) @ np.asarray(mesh_vals, dtype=np.float64)
