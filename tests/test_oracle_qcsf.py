"""Pins for the oracle's quadratically consistent P2M (App. B; eq. p2m).

Each test checks the oracle against something the paper or mathematics fixes,
not against a retyped copy of its own formulas:
  * eqs. C0, C1, C2 (partition of unity, linear and quadratic precision);
  * eq. noC2: linear FE alone fail C2 (negative control);
  * the coefficient system of each edge (eqs. A0, A1, condquad) is solved
    exactly and with minimum norm; on an equilateral lattice the result equals
    an exact symbolic computation from the raw eq. (condquad), and a whole
    row equals the exact row built from lattice geometry alone (each edge's
    coefficients over that edge's own S_e = ring(nu) U ring(sigma): the
    node's full support would give another row);
  * interpolation at a particle (psi_mu(r_nu) = delta_mu nu from eq. phiquad);
  * translation/rotation/scale invariance (eq. A2_2);
  * the projection error order of Sec. 2.1 (h^2 for linear FE, h^3 for a
    quadratically consistent scheme) on the Taylor-Green field of Sec. 3.2.
"""
import numpy as np
import pytest
import sympy
from scipy.spatial import cKDTree

import workloads as wl
from oracle import Mesh, P2MOracle, Triangulation, CLOSURE_K
from oracle.qcsf import edge_system, min_norm_svd, psi_at, linear_fe_matrix, closure_weights_local

QUAD = [
    lambda x, y: np.ones_like(x),
    lambda x, y: x,
    lambda x, y: y,
    lambda x, y: x * x,
    lambda x, y: x * y,
    lambda x, y: y * y,
]


def _poly_vals(P):
    return np.stack([f(P[:, 0], P[:, 1]) for f in QUAD], 1)


@pytest.fixture(scope="module")
def c1():
    c = wl.config1()
    mesh = Mesh.from_spec(c.mesh)
    orc = P2MOracle(c.pos, mesh, c.h)
    W, info = orc.matrix()
    return c, mesh, orc, W, info


def test_C0_C1_C2_at_every_node(c1):
    c, mesh, orc, W, info = c1
    nodes = mesh.nodes()
    got = W @ _poly_vals(c.pos)
    want = _poly_vals(nodes)
    assert np.abs(got - want).max() <= 1e-12
    # closure nodes exist (boundary ring) and all systems are full rank
    assert info["closure"].sum() == 4 * 32
    assert info["edge_rank"][~info["closure"]].min() == 6
    assert info["closure_rank"][info["closure"]].min() == 6
    # Lebesgue constants stay moderate (FP32 rounding bound relies on this)
    leb = np.asarray(abs(W).sum(1)).ravel()
    assert leb[~info["closure"]].max() < 3.0
    assert leb.max() < 8.0


def test_C0_C1_C2_at_random_points_and_clusters():
    c = wl.cluster_void_cloud(16, 3000, seed=7)
    tri = Triangulation(c.pos)
    rng = np.random.default_rng(3)
    pts = rng.uniform(0.2, 0.8, (400, 2))
    U, valid, w, rank = psi_at(tri, pts)
    assert rank.min() == 6
    for f in QUAD:
        vals = f(c.pos[:, 0], c.pos[:, 1])[U]
        got = (w * vals).sum(1)
        assert np.abs(got - f(pts[:, 0], pts[:, 1])).max() <= 1e-10


def test_linear_fe_fails_C2_but_keeps_C0_C1(c1):
    c, mesh, _, _, _ = c1
    L, ok = linear_fe_matrix(c.pos, mesh)
    nodes = mesh.nodes()[ok]
    got = (L @ _poly_vals(c.pos))[ok]
    want = _poly_vals(nodes)
    assert np.abs(got[:, :3] - want[:, :3]).max() <= 1e-13      # C0, C1
    err2 = np.abs(got[:, 3:] - want[:, 3:]).max()                # eq. noC2
    assert 1e-6 < err2 < 10 * c.h ** 2


def test_edge_systems_exact_and_minimum_norm(c1):
    c, mesh, orc, _, _ = c1
    tri = orc.tri
    rng = np.random.default_rng(5)
    checked = 0
    for s in rng.choice(len(tri.simplices), 60, replace=False):
        T = tri.simplices[s]
        for a, b in ((0, 1), (1, 2), (2, 0)):
            nu, sg = int(T[a]), int(T[b])
            S = np.union1d(tri.ring(nu), tri.ring(sg))
            assert nu in S and sg in S
            P = c.pos[S][None]
            M, rhs = edge_system(P, np.array([np.searchsorted(S, nu)]),
                                 np.array([np.searchsorted(S, sg)]), np.ones((1, len(S)), bool))
            A, rank, _ = min_norm_svd(M, rhs, np.array([len(S)]))
            assert rank[0] == 6
            A = A[0]
            # eqs. (A0), (A1), (condquad) in raw coordinates
            r = c.pos[S]
            rn, rs = c.pos[nu], c.pos[sg]
            assert abs(A.sum()) < 1e-12
            assert np.abs(r.T @ A).max() < 1e-13
            lhs = np.einsum("m,mi,mj->ij", A, r, r)
            rhs_q = 0.5 * (np.outer(rn, rs) + np.outer(rs, rn) - np.outer(rn, rn) - np.outer(rs, rs))
            assert np.abs(lhs - rhs_q).max() < 1e-13
            # minimum norm: A lies in the row space of the system
            proj = np.linalg.pinv(M[0]) @ (M[0] @ A)
            assert np.abs(proj - A).max() < 1e-12
            checked += 1
    assert checked == 180


def test_equilateral_lattice_matches_exact_symbolic():
    """Unique Delaunay (no four co-circular points); exact A from raw condquad."""
    rt3 = sympy.sqrt(3)
    ij = [(i, j) for j in range(-4, 5) for i in range(-4, 5)]
    exact = {k: (sympy.Integer(k[0]) + sympy.Rational(k[1], 2), k[1] * rt3 / 2) for k in ij}
    pos = np.array([[float(exact[k][0]), float(exact[k][1])] for k in ij])
    tri = Triangulation(pos)
    idx = {k: n for n, k in enumerate(ij)}
    for e in [((0, 0), (1, 0)), ((0, 0), (0, 1)), ((1, 0), (0, 1))]:
        nu, sg = idx[e[0]], idx[e[1]]
        S = np.union1d(tri.ring(nu), tri.ring(sg))
        assert len(S) == 10
        # exact minimum-norm solution of eqs. (A0), (A1), (condquad)
        pts = [exact[ij[m]] for m in S]
        xn, yn = exact[e[0]]
        xs, ys = exact[e[1]]
        Ms = sympy.Matrix([[1] * len(S), [p[0] for p in pts], [p[1] for p in pts],
                           [p[0] ** 2 for p in pts], [p[0] * p[1] for p in pts],
                           [p[1] ** 2 for p in pts]])
        half = sympy.Rational(1, 2)
        bs = sympy.Matrix([0, 0, 0,
                           half * (2 * xn * xs - xn ** 2 - xs ** 2),
                           half * (xn * ys + xs * yn - xn * yn - xs * ys),
                           half * (2 * yn * ys - yn ** 2 - ys ** 2)])
        As = Ms.T * (Ms * Ms.T).LUsolve(bs)
        As = np.array([float(sympy.nsimplify(sympy.simplify(v))) for v in As])
        M, rhs = edge_system(pos[S][None], np.array([np.searchsorted(S, nu)]),
                             np.array([np.searchsorted(S, sg)]), np.ones((1, len(S)), bool))
        A, rank, _ = min_norm_svd(M, rhs, np.array([len(S)]))
        assert rank[0] == 6
        assert np.abs(A[0] - As).max() <= 1e-13


def _lattice_row(q, support_of_edge):
    """Exact row psi_mu(q) on the equilateral lattice (i + j/2, j sqrt(3)/2),
    built from lattice geometry alone (no triangulation): T is the lattice
    triangle holding q, a vertex's ring is its six lattice neighbours, and
    A_e is the exact minimum-norm solution of eqs. (A0), (A1), (condquad)
    over support_of_edge(nu, sigma).  Returns {(i, j): psi}."""
    rt3 = sympy.sqrt(3)
    half = sympy.Rational(1, 2)
    qx, qy = sympy.nsimplify(q[0]), sympy.nsimplify(q[1])   # dyadic, exact
    jf = 2 * qy / rt3
    i_f = qx - jf / 2
    i0, j0 = int(sympy.floor(i_f)), int(sympy.floor(jf))
    if (i_f - i0) + (jf - j0) < 1:
        T = [(i0, j0), (i0 + 1, j0), (i0, j0 + 1)]
    else:
        T = [(i0 + 1, j0), (i0 + 1, j0 + 1), (i0, j0 + 1)]

    def xy(k):
        return (sympy.Integer(k[0]) + half * k[1], k[1] * rt3 / 2)

    # barycentric coordinates of q in T (eqs. C0, C1), exact
    P = [xy(k) for k in T]
    D = (P[1][0] - P[0][0]) * (P[2][1] - P[0][1]) - (P[1][1] - P[0][1]) * (P[2][0] - P[0][0])
    phi = [((P[1][0] - qx) * (P[2][1] - qy) - (P[1][1] - qy) * (P[2][0] - qx)) / D,
           ((qx - P[0][0]) * (P[2][1] - P[0][1]) - (qy - P[0][1]) * (P[2][0] - P[0][0])) / D,
           ((P[1][0] - P[0][0]) * (qy - P[0][1]) - (P[1][1] - P[0][1]) * (qx - P[0][0])) / D]
    row = {}
    for k, f in zip(T, phi):
        row[k] = row.get(k, 0) + f
    for a, b in ((0, 1), (1, 2), (2, 0)):
        nu, sg = T[a], T[b]
        S = sorted(support_of_edge(nu, sg))
        pts = [xy(k) for k in S]
        (xn, yn), (xs, ys) = xy(nu), xy(sg)
        Ms = sympy.Matrix([[1] * len(S), [p[0] for p in pts], [p[1] for p in pts],
                           [p[0] ** 2 for p in pts], [p[0] * p[1] for p in pts],
                           [p[1] ** 2 for p in pts]])
        bs = sympy.Matrix([0, 0, 0,
                           half * (2 * xn * xs - xn ** 2 - xs ** 2),
                           half * (xn * ys + xs * yn - xn * yn - xs * ys),
                           half * (2 * yn * ys - yn ** 2 - ys ** 2)])
        As = Ms.T * (Ms * Ms.T).LUsolve(bs)
        for k, v in zip(S, As):
            row[k] = row.get(k, 0) + 2 * phi[a] * phi[b] * v
    return {k: float(sympy.N(v, 30)) for k, v in row.items()}


def test_equilateral_lattice_whole_row_from_lattice_rings():
    """A whole oracle row equals phi + 2 sum_e phi_nu phi_sigma A_e with each
    A_e solved exactly over its own edge's support ring(nu) U ring(sigma),
    where the rings are the lattice's six neighbours (not the oracle's
    triangulation).  The same construction with the node's full support for
    every edge gives a different row, so the oracle's choice of S_e is what
    this test pins."""
    ij = [(i, j) for j in range(-6, 7) for i in range(-6, 7)]
    rt3 = np.sqrt(3.0)
    pos = np.array([[i + 0.5 * j, 0.5 * rt3 * j] for i, j in ij])
    col = {k: n for n, k in enumerate(ij)}
    # dyadic mesh offsets put the nodes strictly inside lattice triangles
    mesh = Mesh(19, 12, 1.0, -9.75, -5.875)
    nodes = mesh.nodes()
    node_ids = [6 * 20 + 10, 5 * 20 + 9, 7 * 20 + 11]
    W, info = P2MOracle(pos, mesh, 0.5).matrix(np.asarray(node_ids))
    nbr = ((1, 0), (-1, 0), (0, 1), (0, -1), (1, -1), (-1, 1))

    def ring(k):
        return {(k[0] + di, k[1] + dj) for di, dj in nbr}

    for t, k in enumerate(node_ids):
        assert not info["closure"][t]
        got = W[t].toarray().ravel()
        want = np.zeros_like(got)
        for key, v in _lattice_row(nodes[k], lambda a, b: ring(a) | ring(b)).items():
            want[col[key]] = v
        assert np.count_nonzero(got) == np.count_nonzero(want)
        assert np.abs(got - want).max() <= 1e-13
        # negative control: every edge over the node's whole support U
        U = set()
        for key in _lattice_row(nodes[k], lambda a, b: ring(a) | ring(b)):
            U |= {key}
        alt = np.zeros_like(got)
        for key, v in _lattice_row(nodes[k], lambda a, b: U).items():
            alt[col[key]] = v
        assert np.abs(alt - want).max() > 1e-3


def test_interpolates_at_a_particle():
    c = wl.small_cloud(16, 2, 0.25, seed=11)
    mesh = Mesh.from_spec(c.mesh)
    pos = c.pos.copy()
    nodes = mesh.nodes()
    k_node = 7 * 17 + 5
    near = int(np.argmin(((pos - nodes[k_node]) ** 2).sum(1)))
    pos[near] = nodes[k_node]          # a particle exactly on an interior node
    orc = P2MOracle(pos, mesh, c.h)
    W, info = orc.matrix()
    row = W[k_node].toarray().ravel()
    assert not info["closure"][k_node]
    assert abs(row[near] - 1.0) < 1e-14
    row[near] = 0.0
    assert np.abs(row).max() < 1e-14


def test_similarity_invariance():
    c = wl.small_cloud(12, 2, 0.3, seed=21)
    tri = Triangulation(c.pos)
    rng = np.random.default_rng(4)
    pts = rng.uniform(0.25, 0.75, (200, 2))
    U, valid, w, _ = psi_at(tri, pts)
    th = 0.7
    R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    s, t = 3.7, np.array([-2.5, 11.0])
    tri2 = Triangulation(c.pos @ R.T * s + t)
    U2, valid2, w2, _ = psi_at(tri2, pts @ R.T * s + t)
    assert np.array_equal(U, U2) and np.array_equal(valid, valid2)
    assert np.abs(w - w2).max() <= 1e-12


def test_closure_neighbours_match_brute_force_and_are_quadratic_exact():
    c = wl.small_cloud(8, 2, 0.25, seed=3)
    mesh = Mesh.from_spec(c.mesh)
    nodes = mesh.nodes()
    ring = np.flatnonzero(mesh.on_boundary_ring(np.arange(mesh.n_nodes)))
    tree = cKDTree(c.pos)
    _, nn = tree.query(nodes[ring], k=CLOSURE_K)
    for q, k in enumerate(ring):
        d2 = ((c.pos - nodes[k]) ** 2).sum(1)
        assert set(nn[q]) == set(np.argsort(d2, kind="stable")[:CLOSURE_K])
    w, rank, sig = closure_weights_local(c.pos[nn], nodes[ring], c.h)
    assert rank.min() == 6
    for f in QUAD:
        got = (w * f(c.pos[nn][..., 0], c.pos[nn][..., 1])).sum(1)
        assert np.abs(got - f(nodes[ring, 0], nodes[ring, 1])).max() < 1e-12
    assert np.abs(w).sum(1).max() < 8.0
    # the scale used for the monomials does not change the weights
    w2, _, _ = closure_weights_local(c.pos[nn], nodes[ring], 5.0 * c.h)
    assert np.abs(w - w2).max() < 1e-12


def test_local_mode_equals_global_mode(c1):
    c, mesh, _, W, _ = c1
    orl = P2MOracle(c.pos, mesh, c.h, mode="local")
    ids = np.arange(0, mesh.n_nodes, 5)
    Wl, _ = orl.matrix(ids)
    assert abs(Wl - W[ids]).max() <= 1e-13


def _slope(Hs, errs):
    return np.polyfit(np.log(Hs), np.log(errs), 1)[0]


def test_projection_error_order_taylor_green():
    """Sec. 2.1: P2M error ~ h^2 with linear FE, ~ h^3 with the quadratic
    correction, here at fixed h = H/2 on the Taylor-Green u field (Sec. 3.2)."""
    Hs, eq, el = [], [], []
    for n in (16, 32, 64, 128):
        c = wl.small_cloud(n, 2, 0.25, seed=100 + n, channels=("u",))
        mesh = Mesh.from_spec(c.mesh)
        orc = P2MOracle(c.pos, mesh, c.h)
        W, _ = orc.matrix()
        L, ok = linear_fe_matrix(c.pos, mesh)
        nodes = mesh.nodes()
        i, j = mesh.node_ij(np.arange(mesh.n_nodes))
        inner = (i >= 2) & (j >= 2) & (i <= n - 2) & (j <= n - 2)
        exact = wl.tg_u(nodes[:, 0], nodes[:, 1])
        eq.append(np.abs((W @ c.vals[:, 0]) - exact)[inner].max())
        el.append(np.abs((L @ c.vals[:, 0]) - exact)[inner & ok].max())
        Hs.append(1.0 / n)
    sq, sl = _slope(Hs, eq), _slope(Hs, el)
    assert sq >= 2.6, (sq, eq)
    assert 1.7 <= sl <= 2.3, (sl, el)
