"""Pins of the oracle's mesh-side quadratically consistent M2P
(oracle/m2p_qcsf.py): exact reproduction of every quadratic at arbitrary
particles (eq. C2, boundary cells included), interpolation at the nodes,
third-order convergence on a smooth field (linear FE: second), and equal
coefficients on equally oriented interior edges (the construction does not
know where an edge is)."""
import numpy as np

from oracle import Mesh
from oracle.m2p import m2p_matrix
from oracle.m2p_qcsf import edge_coefficients, m2p_qcsf_matrix


def test_every_quadratic_is_reproduced_at_any_particle():
    mesh = Mesh(9, 7, 1.0 / 9, x0=0.2, y0=-0.1)
    rng = np.random.default_rng(0)
    p = np.array([0.2, -0.1]) + rng.random((3000, 2)) * np.array([1.0, 7.0 / 9])
    W = m2p_qcsf_matrix(mesh, p)
    nd = mesh.nodes()
    for f in (lambda X: np.ones(len(X)), lambda X: X[:, 0], lambda X: X[:, 1], lambda X: X[:, 0] ** 2,
              lambda X: X[:, 0] * X[:, 1], lambda X: X[:, 1] ** 2):
        assert np.abs(W @ f(nd) - f(p)).max() < 1e-13


def test_interpolates_at_the_nodes():
    mesh = Mesh(6, 6, 1.0 / 6)
    nd = mesh.nodes()
    W = m2p_qcsf_matrix(mesh, nd)
    vals = np.random.default_rng(1).random(len(nd))
    assert np.abs(W @ vals - vals).max() < 1e-14


def test_third_order_against_second_order_for_linear_fe():
    g = lambda X: np.sin(2.3 * X[:, 0] + 0.4) * np.cos(1.7 * X[:, 1] - 0.2)  # noqa: E731
    q = np.random.default_rng(2).random((2000, 2))
    eq, el = [], []
    for n in (16, 32, 64):
        m = Mesh(n, n, 1.0 / n)
        nd = m.nodes()
        eq.append(np.abs(m2p_qcsf_matrix(m, q) @ g(nd) - g(q)).max())
        el.append(np.abs(m2p_matrix(m, q) @ g(nd) - g(q)).max())
    sq = np.log2(eq[0] / eq[2]) / 2
    sl = np.log2(el[0] / el[2]) / 2
    assert sq > 2.7 and 1.8 < sl < 2.2, (sq, sl)


def test_equally_oriented_interior_edges_share_coefficients():
    m = Mesh(10, 10, 0.1)
    s = m.nx + 1
    node = lambda i, j: j * s + i  # noqa: E731
    for d in ((1, 0), (0, 1), (1, 1)):
        E = np.array([[node(3, 3), node(3 + d[0], 3 + d[1])], [node(6, 5), node(6 + d[0], 5 + d[1])]])
        U, valid, A, rank = edge_coefficients(m, E)
        assert np.all(rank == 6) and valid.sum(1)[0] == valid.sum(1)[1] == 10
        # supports sorted by node id: the same offsets in the same order
        assert np.array_equal(U[0] - E[0, 0], U[1] - E[1, 0])
        assert np.abs(A[0] - A[1]).max() < 1e-12


def test_periodic_mesh_functions_are_consistent_in_minimum_image_offsets():
    """Periodic box: sum psi = 1, sum psi d = 0, sum psi d d^t = 0 with d the
    minimum-image offsets of the nodes from the particle (computed here from
    the box's node positions), interpolation at the nodes, and agreement with
    the bounded functions two cells away from the sides."""
    from oracle import Mesh
    from oracle.m2p_qcsf import m2p_qcsf_matrix, m2p_qcsf_periodic_matrix
    m = Mesh(8, 6, 0.25, -1.0, -0.75)
    L = np.array([m.nx * m.H, m.ny * m.H])
    rng = np.random.default_rng(4)
    pos = np.array([m.x0, m.y0]) + rng.random((400, 2)) * L
    W = m2p_qcsf_periodic_matrix(m, pos)
    nodes = m.nodes()
    for p in range(len(pos)):
        r = W.getrow(p)
        d = nodes[r.indices] - pos[p]
        d -= L * np.rint(d / L)
        w = r.data
        assert abs(w.sum() - 1) < 1e-12
        assert np.abs(w @ d).max() < 1e-12
        assert np.abs(np.einsum("k,ka,kb->ab", w, d, d)).max() < 1e-12
    i = np.arange(m.nx); j = np.arange(m.ny)
    kk = (j[:, None] * (m.nx + 1) + i[None, :]).ravel()
    Wn = m2p_qcsf_periodic_matrix(m, nodes[kk]).toarray()
    assert np.abs(Wn[:, kk] - np.eye(len(kk))).max() < 1e-12
    far = ((pos[:, 0] > m.x0 + 2 * m.H) & (pos[:, 0] < m.x0 + L[0] - 2 * m.H) &
           (pos[:, 1] > m.y0 + 2 * m.H) & (pos[:, 1] < m.y0 + L[1] - 2 * m.H))
    assert far.sum() > 50
    Wb = m2p_qcsf_matrix(m, pos[far])
    assert abs(W[np.flatnonzero(far)] - Wb).max() < 1e-12
