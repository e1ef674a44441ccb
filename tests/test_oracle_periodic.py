"""Pins of the periodic-box oracle (CPU only).

The periodic rows are checked against what the method fixes independently of
the oracle's own construction: the consistency conditions (eqs. C0, C1, C2)
in minimum-image offsets computed here from the raw positions, the empty
circumcircle of every node's triangle by brute force over all images,
invariance under a translation of the cloud by one mesh spacing (which moves
particles across the box side), and agreement with the bounded oracle at
nodes far from the box sides.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import Mesh, P2MOracle, PeriodicP2MOracle
from oracle.delaunay import circumcircle
from oracle.periodic import tiled, wrapped_nodes


def _oracle(n=8, ratio=2, jitter=0.25, seed=3, pos=None, voids=False):
    c = wl.periodic_void_cloud(n, 3000, seed) if voids else wl.periodic_tg_cloud(n, ratio, jitter, seed)
    m = Mesh.from_spec(c.mesh)
    return c, m, PeriodicP2MOracle(c.pos if pos is None else pos, m, c.h)


def _min_image(d, L):
    return d - L * np.rint(d / L)


@pytest.mark.parametrize("seed,jitter,voids", [(3, 0.25, False), (4, 0.45, False), (9, 0.0, True)])
def test_consistency_in_minimum_image_offsets(seed, jitter, voids):
    c, m, o = _oracle(n=16 if voids else 8, seed=seed, jitter=jitter, voids=voids)
    cols, vals, imgs, info = o.node_weights()
    L = np.array([m.nx * m.H, m.ny * m.H])
    nodes = wrapped_nodes(m)
    for k, (cc, w, im) in enumerate(zip(cols, vals, imgs)):
        d = _min_image(c.pos[cc] - nodes[k], L)
        # the images used are the nearest ones
        assert np.abs(o.images[im] - nodes[k] - d).max() < 1e-14
        s = d / m.H
        assert abs(w.sum() - 1.0) < 1e-12                                   # C0
        assert np.abs(w @ s).max() < 1e-12                                  # C1
        assert np.abs(np.einsum("k,ka,kb->ab", w, s, s)).max() < 1e-11      # C2
    assert not info["closure"].any()


def test_node_triangles_are_periodic_delaunay():
    c, m, o = _oracle(seed=5)
    imgs, _ = tiled(c.pos, m)
    nodes = wrapped_nodes(m)
    s = o.tri.locate(nodes)
    T = o.tri.simplices[s]
    cc, rr = circumcircle(o.images[T])
    for k in range(len(nodes)):
        d2 = ((imgs - cc[k]) ** 2).sum(1)
        inside = d2 < rr[k] ** 2 * (1 - 1e-12)
        inside[T[k]] = False
        assert not inside.any(), k
        # the node lies in its triangle
        P = o.images[T[k]]
        for a in range(3):
            p, q, r = P[a], P[(a + 1) % 3], P[(a + 2) % 3]
            side = (q[0] - p[0]) * (nodes[k][1] - p[1]) - (q[1] - p[1]) * (nodes[k][0] - p[0])
            ref = (q[0] - p[0]) * (r[1] - p[1]) - (q[1] - p[1]) * (r[0] - p[0])
            assert side * ref >= 0


def test_translation_by_one_cell_shifts_the_rows():
    c, m, o = _oracle(n=10, seed=6)
    pos2 = c.pos.copy()
    pos2[:, 0] += m.H
    L = m.nx * m.H
    pos2[pos2[:, 0] >= m.x0 + L, 0] -= L
    o2 = PeriodicP2MOracle(pos2, m, c.h)
    W1, _ = o.matrix()
    W2, _ = o2.matrix()
    nx1 = m.nx + 1
    for j in range(m.ny + 1):
        for i in range(m.nx + 1):
            r1 = W1.getrow(j * nx1 + i)
            r2 = W2.getrow(j * nx1 + (i + 1) % m.nx)
            assert np.array_equal(np.sort(r1.indices), np.sort(r2.indices))
            assert abs(r1 - r2).max() < 1e-12


def test_seam_rows_repeat_the_first_column_and_row():
    c, m, o = _oracle(seed=7)
    W, _ = o.matrix()
    nx1 = m.nx + 1
    for j in range(m.ny + 1):
        assert abs(W.getrow(j * nx1 + m.nx) - W.getrow(j * nx1)).max() == 0.0
    for i in range(m.nx + 1):
        assert abs(W.getrow(m.ny * nx1 + i) - W.getrow(i)).max() == 0.0


def test_far_from_the_sides_rows_equal_the_bounded_ones():
    c, m, o = _oracle(n=12, seed=8)
    Wp, _ = o.matrix()
    Wb, info = P2MOracle(c.pos, m, c.h).matrix()
    nodes = m.nodes()
    far = ((nodes[:, 0] - m.x0 > 5 * c.h) & (m.x0 + m.nx * m.H - nodes[:, 0] > 5 * c.h) &
           (nodes[:, 1] - m.y0 > 5 * c.h) & (m.y0 + m.ny * m.H - nodes[:, 1] > 5 * c.h))
    assert far.sum() > 20
    for k in np.flatnonzero(far):
        rp, rb = Wp.getrow(k), Wb.getrow(k)
        assert np.array_equal(np.sort(rp.indices), np.sort(rb.indices))
        assert abs(rp - rb).max() < 1e-12


def test_position_gradient_matches_central_differences():
    """The complex-step gradient of sum gbar * P2M(vals) against central
    differences of the periodic forward (retriangulated at each offset) for
    particles next to the box corner and sides, whose images carry the
    dependence across the sides."""
    from oracle.periodic import periodic_p2m_grad_pos
    c, m, o = _oracle(seed=13)
    rng = np.random.default_rng(0)
    g = rng.normal(size=(m.n_nodes, c.vals.shape[1]))
    grad = periodic_p2m_grad_pos(o, c.vals, g)
    L = m.nx * m.H

    def loss(pos):
        W, _ = PeriodicP2MOracle(pos, m, c.h).matrix()
        return float(((W @ c.vals) * g).sum())

    d_side = np.minimum(c.pos - [m.x0, m.y0], [m.x0 + L, m.y0 + L] - c.pos).min(1)
    picks = list(np.argsort(d_side)[:4]) + [int(np.argmax(d_side))]
    step = 1e-6 * c.h
    for p in picks:
        for d in range(2):
            a, b = c.pos.copy(), c.pos.copy()
            a[p, d] += step
            b[p, d] -= step
            fd = (loss(a) - loss(b)) / (2 * step)
            assert abs(fd - grad[p, d]) <= 1e-6 * (1 + abs(fd)), (p, d, fd, grad[p, d])
