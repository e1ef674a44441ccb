"""Pins for the oracle's Delaunay step (Qhull) against exact brute force.

App. B builds phi on the Delaunay triangulation of the particles ("unique
except for possible degeneracies") and defines neighbours as Delaunay edges.
Here Qhull's answer is checked against the definition itself: a triangle is
Delaunay iff no other particle lies strictly inside its circumcircle, decided
in exact integer arithmetic on the (exactly representable) FP64 inputs.
"""
import itertools
from fractions import Fraction

import numpy as np
import pytest

from oracle import Triangulation, GeometryError


def _exact(pos):
    """FP64 coordinates -> exact Python integers (common power-of-two scale)."""
    fr = [[Fraction(float(v)) for v in p] for p in pos]
    den = 1
    for p in fr:
        for v in p:
            den = max(den, v.denominator)
    return [(int(x * den), int(y * den)) for x, y in fr]


def _orient(a, b, c):
    return (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0])


def _incircle(a, b, c, d):
    """> 0 iff d is strictly inside the circle through CCW a, b, c."""
    rows = []
    for p in (a, b, c):
        dx, dy = p[0] - d[0], p[1] - d[1]
        rows.append((dx, dy, dx * dx + dy * dy))
    (a0, a1, a2), (b0, b1, b2), (c0, c1, c2) = rows
    return (a0 * (b1 * c2 - b2 * c1) - a1 * (b0 * c2 - b2 * c0) + a2 * (b0 * c1 - b1 * c0))


def brute_force_delaunay(pos):
    P = _exact(pos)
    n = len(P)
    tris = set()
    for i, j, k in itertools.combinations(range(n), 3):
        o = _orient(P[i], P[j], P[k])
        if o == 0:
            continue
        a, b, c = (i, j, k) if o > 0 else (i, k, j)
        if all(_incircle(P[a], P[b], P[c], P[m]) <= 0 for m in range(n) if m not in (i, j, k)):
            tris.add(frozenset((i, j, k)))
    return tris


def _hull_count(pos):
    P = _exact(pos)
    pts = sorted(set(P))

    def half(seq):
        h = []
        for p in seq:
            while len(h) >= 2 and _orient(h[-2], h[-1], p) <= 0:
                h.pop()
            h.append(p)
        return h

    lo, up = half(pts), half(pts[::-1])
    return len(lo) + len(up) - 2


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("n", [8, 17, 28])
def test_qhull_matches_exact_empty_circle(seed, n):
    rng = np.random.default_rng(1000 + seed)
    if seed % 2:
        pos = rng.uniform(0, 1, (n, 2))
    else:  # jittered lattice fragment, the workloads' structure
        m = int(np.ceil(np.sqrt(n)))
        g = (np.arange(m) + 0.5) / m
        X, Y = np.meshgrid(g, g)
        pos = np.stack([X.ravel(), Y.ravel()], 1)[:n] + rng.uniform(-0.25 / m, 0.25 / m, (n, 2))
    tri = Triangulation(pos)
    qh = {frozenset(map(int, t)) for t in tri.simplices}
    assert qh == brute_force_delaunay(pos)
    # Euler: #triangles = 2N - 2 - #hull vertices (no collinear hull points here)
    assert len(qh) == 2 * n - 2 - _hull_count(pos)
    # rings are symmetric and equal the edge sets of the triangles
    edges = set()
    for t in qh:
        a, b, c = sorted(t)
        edges |= {(a, b), (b, c), (a, c)}
    for v in range(n):
        for u in tri.ring(v):
            assert (min(u, v), max(u, v)) in edges
            assert v in tri.ring(int(u))


def test_duplicate_particles_rejected():
    pos = np.array([[0.1, 0.1], [0.9, 0.1], [0.5, 0.8], [0.4, 0.4], [0.4, 0.4]])
    with pytest.raises(GeometryError):
        Triangulation(pos)


def test_collinear_cloud_rejected():
    pos = np.stack([np.linspace(0.1, 0.9, 10), np.full(10, 0.5)], 1)
    with pytest.raises(GeometryError):
        Triangulation(pos)
