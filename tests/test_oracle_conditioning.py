"""Pins for the oracle's moment-system solves where they are ill-conditioned
or lose rank (App. A: SVD with automatic rank detection; App. B: eqs. A0, A1,
A2_2).

On ``workloads.conic_cloud`` every support lies within a relative delta of
one conic, so cond(M) grows like 1 / delta, and supports of five particles
(ear vertices of the triangulation) are rank-deficient.  Each system the
oracle solves is checked against the same definition evaluated in 60-digit
arithmetic (mpmath), from the same FP64 positions:
  * full rank: A = M^t (M M^t)^-1 b, the minimum-norm solution;
  * K = 5 < 6 columns: A = (M^t M)^-1 M^t b, the least-squares solution (the
    minimum-norm one: M has full column rank);
within 10 eps cond(M) of the largest |A| (the forward error bound of a
backward-stable solve).  The rank the oracle reports must be min(6, K) and
cond(M) must sweep 1e2 .. 1e10 over the deltas.
"""
import mpmath
import numpy as np
import pytest

import workloads as wl
from oracle import Mesh, Triangulation
from oracle.qcsf import NodeStructure, edge_system, min_norm_svd

EPS = np.finfo(np.float64).eps
EDGES = ((0, 1), (1, 2), (2, 0))


def _exact_min_norm(P, nu, sg):
    """Minimum-norm (least-squares if K < 6) solution of eqs. (A0), (A1),
    (A2_2) over the support P [K, 2] in 60-digit arithmetic, written from the
    equations: rows relative to the edge ends, scaled by the edge length."""
    mpmath.mp.dps = 60
    pts = [(mpmath.mpf(float(x)), mpmath.mpf(float(y))) for x, y in P]
    (xn, yn), (xs, ys) = pts[nu], pts[sg]
    s = mpmath.sqrt((xn - xs) ** 2 + (yn - ys) ** 2)
    rows = []
    for x, y in pts:
        ax, ay = (x - xn) / s, (y - yn) / s
        cx, cy = (x - xs) / s, (y - ys) / s
        rows.append([1, ax, ay, ax * cx, (ax * cy + ay * cx) / 2, ay * cy])
    M = mpmath.matrix(rows).T                        # 6 x K
    dx, dy = (xn - xs) / s, (yn - ys) / s
    b = mpmath.matrix([0, 0, 0, -dx * dx / 2, -dx * dy / 2, -dy * dy / 2])
    K = len(pts)
    if K >= 6:
        A = M.T * mpmath.lu_solve(M * M.T, b)
    else:
        A = mpmath.lu_solve(M.T * M, M.T * b)
    return np.array([float(v) for v in A])


@pytest.mark.parametrize("delta", [1e-1, 1e-4, 1e-10])
def test_conic_systems_match_high_precision_definition(delta):
    c = wl.conic_cloud(8, 24, delta, seed=3)
    tri = Triangulation(c.pos)
    om = Mesh.from_spec(c.mesh)
    s = tri.locate(om.nodes())
    ids = np.flatnonzero((s >= 0) & ~om.on_boundary_ring(np.arange(om.n_nodes)))
    st = NodeStructure.build([tri.triangle(t) for t in s[ids]], tri.ring)
    conds = []
    for n in range(len(ids)):
        P = c.pos[st.U[n]]
        for p, q in EDGES:
            S = (st.member[n, p] | st.member[n, q]) & st.valid[n]
            K = int(S.sum())
            M, b = edge_system(P[None], np.array([st.tri[n, p]]), np.array([st.tri[n, q]]), S[None])
            A, rank, sig = min_norm_svd(M, b, np.array([K]))
            assert rank[0] == min(6, K)
            cond = sig[0, 0] / sig[0, rank[0] - 1]
            conds.append(cond)
            sub = np.flatnonzero(S)
            ref = _exact_min_norm(P[sub], int(np.searchsorted(sub, st.tri[n, p])),
                                  int(np.searchsorted(sub, st.tri[n, q])))
            err = np.abs(A[0][sub] - ref).max()
            assert err <= 10.0 * EPS * cond * np.abs(ref).max(), (delta, K, cond, err)
            # columns outside S_e are zero columns of M: zero up to the same bound
            assert np.abs(A[0][~S]).max(initial=0.0) <= 10.0 * EPS * cond * np.abs(ref).max()
    conds = np.array(conds)
    lo, hi = {1e-1: (1e1, 1e3), 1e-4: (1e3, 1e7), 1e-10: (1e8, 1e13)}[delta]
    assert conds.max() >= lo and conds.max() <= hi, (conds.min(), conds.max())
