"""Quadratically consistent particle shape functions and P2M (oracle; test infrastructure only).

Follows App. B of the paper:

* phi_mu: linear FE functions on the particles' Delaunay triangulation, i.e.
  at a point inside triangle T = (a, b, c) the barycentric coordinates of the
  point in T, zero for every other particle (eqs. C0, C1 hold, eq. noC2 does
  not in general).
* psi_mu = phi_mu + sum over ordered pairs (nu, sigma) of
  A_{mu nu sigma} phi_nu phi_sigma, eq. (phiquad), with A symmetric in its last
  two indices.  Inside T only the three edges of T carry non-zero products, so
  psi_mu(r) = phi_mu(r) + 2 * sum_{edges e=(nu,sigma) of T} phi_nu phi_sigma A_{mu e}.
  (The factor 2 is the ordered-pair sum; it is what makes eq. C2 hold with the
  right-hand side of eq. condquad as printed.)
* For each Delaunay edge e = (nu, sigma) the coefficients A_{mu e} satisfy
  eq. (A0) sum_mu A = 0, eq. (A1) sum_mu r_mu A = 0 and eq. (A2_2)
  sum_mu (r_mu - r_nu)(r_mu - r_sigma)^t A = -1/2 (r_nu - r_sigma)(r_nu - r_sigma)^t,
  the translation/rotation invariant form of eq. (condquad).  A is zero unless
  mu is a Delaunay neighbour of nu or of sigma, so the support of edge e is
  S_e = ring(nu) U ring(sigma) (which contains nu and sigma).  The paper
  defers the exact neighbour rule to its ref. [QCSF]; this union is the reading
  taken here.
* The 6 x |S_e| system is underdetermined; the paper solves it with an SVD
  "with automatic rank detection" (App. A).  The oracle takes the minimum
  Euclidean-norm solution with LAPACK's default rank threshold
  (singular values below eps * max(6, |S_e|) * sigma_max are dropped).
* P2M, eq. (p2m): alpha_i = sum_mu alpha_mu psi_mu(r_i).

Nodes where the construction above is unusable are handled by a reading the
paper does not cover (it only runs periodic boxes, which ``periodic`` forms
without closure nodes): every node on the outer
ring of the mesh and every node outside the particles' convex hull is a
CLOSURE node whose weights are the minimum-norm solution of the six
quadratic moment conditions sum_mu w_mu p(r_mu - r_i) = p(0) over its
CLOSURE_K = 12 nearest particles, p = (1, x, y, x^2, xy, y^2).  These weights
reproduce any quadratic exactly, like psi.

All arithmetic is FP64.  ``min_norm_normal`` / complex inputs exist only for
complex-step differentiation (adjoint tests); values always use the SVD.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np
import scipy.sparse as sp
from scipy.spatial import cKDTree

from .delaunay import LocalTriangulation, Triangulation
from .mesh import Mesh

EPS = np.finfo(np.float64).eps
CLOSURE_K = 12


# --------------------------------------------------------------- algebra ---

def edge_system(P, nu, sg, S):
    """Moment system of one Delaunay edge, eqs. (A0), (A1), (A2_2).

    P  [..., K, 2] candidate positions (real or complex)
    nu, sg [...] index of the edge end points in the K axis
    S  [..., K] bool, True for members of the support S_e (other columns are 0)

    Rows, with s = |r_nu - r_sigma|, a_mu = (r_mu - r_nu)/s,
    c_mu = (r_mu - r_sigma)/s and d = (r_nu - r_sigma)/s:
      (A0)    1                                  = 0
      (A1)    a_mu,x ; a_mu,y                    = 0 ; 0
              (eq. A1 in the form sum (r_mu - r_nu) A = 0, equivalent given A0)
      (A2_2)  a_x c_x ; (a_x c_y + a_y c_x)/2 ; a_y c_y = -d_x^2/2 ; -d_x d_y/2 ; -d_y^2/2
    Dividing by s and s^2 rescales rows only; the solution set is unchanged.
    Returns M [..., 6, K] and b [..., 6].
    """
    P = np.asarray(P)
    rn = np.take_along_axis(P, np.asarray(nu)[..., None, None], axis=-2)[..., 0, :]
    rs = np.take_along_axis(P, np.asarray(sg)[..., None, None], axis=-2)[..., 0, :]
    dvec = rn - rs
    s = np.sqrt(dvec[..., 0] ** 2 + dvec[..., 1] ** 2)
    a = (P - rn[..., None, :]) / s[..., None, None]
    c = (P - rs[..., None, :]) / s[..., None, None]
    d = dvec / s[..., None]
    one = np.ones(P.shape[:-1], dtype=P.dtype)
    rows = [
        one,
        a[..., 0],
        a[..., 1],
        a[..., 0] * c[..., 0],
        0.5 * (a[..., 0] * c[..., 1] + a[..., 1] * c[..., 0]),
        a[..., 1] * c[..., 1],
    ]
    M = np.stack(rows, axis=-2) * S[..., None, :]
    zero = np.zeros(d.shape[:-1], dtype=P.dtype)
    b = np.stack([zero, zero, zero,
                  -0.5 * d[..., 0] ** 2,
                  -0.5 * d[..., 0] * d[..., 1],
                  -0.5 * d[..., 1] ** 2], axis=-1)
    return M, b


def monomials(X):
    """p(x, y) = (1, x, y, x^2, xy, y^2) for X [..., 2] -> [..., 6]."""
    x, y = X[..., 0], X[..., 1]
    return np.stack([np.ones_like(x), x, y, x * x, x * y, y * y], axis=-1)


def min_norm_svd(M, b, k_eff):
    """Minimum-norm solution of M A = b by SVD with rank detection (App. A).

    M [..., 6, K], b [..., 6], k_eff [...] number of real (unpadded) columns.
    Singular values <= eps * max(6, k_eff) * sigma_max are treated as zero
    (LAPACK gelsd's default).  Returns (A [..., K], rank [...], sigma [..., 6]).
    """
    U, sig, Vt = np.linalg.svd(M, full_matrices=False)
    smax = sig[..., 0]
    tol = EPS * np.maximum(6, np.asarray(k_eff)) * smax
    keep = sig > tol[..., None]
    c = np.einsum("...ji,...j->...i", U, b)
    c = np.where(keep, c / np.where(keep, sig, 1.0), 0.0)
    A = np.einsum("...ij,...i->...j", Vt, c)
    if sig.shape[-1] < 6:  # fewer columns than conditions: report 6 values
        sig = np.concatenate([sig, np.zeros(sig.shape[:-1] + (6 - sig.shape[-1],))], axis=-1)
    return A, keep.sum(-1), sig


def min_norm_normal(M, b):
    """A = M^t (M M^t)^{-1} b, the minimum-norm solution for full row rank M.

    Uses plain transposes (no conjugation) so that it is holomorphic and can be
    complex-step differentiated.
    """
    Mt = np.swapaxes(M, -1, -2)
    G = M @ Mt
    y = np.linalg.solve(G, b[..., None])
    return (Mt @ y)[..., 0]


def barycentric(Ptri, r):
    """Linear FE values phi_a, phi_b, phi_c at r inside triangle (a, b, c).

    Solves [x_a x_b x_c; y_a y_b y_c; 1 1 1] phi = [x; y; 1]  (eqs. C0, C1).
    Ptri [..., 3, 2], r [..., 2] -> [..., 3].
    """
    Ptri = np.asarray(Ptri)
    r = np.asarray(r)
    dtype = np.result_type(Ptri, r)
    ones = np.ones(Ptri.shape[:-1], dtype=dtype)
    Amat = np.stack([Ptri[..., 0], Ptri[..., 1], ones], axis=-2)
    rhs = np.stack([r[..., 0], r[..., 1], np.ones(r.shape[:-1], dtype=dtype)], axis=-1)
    return np.linalg.solve(Amat, rhs[..., None])[..., 0]


# ----------------------------------------------------- per-node weights ---

@dataclasses.dataclass
class NodeStructure:
    """Combinatorial data of interior points (all from the triangulation).

    U      [n, K] global particle ids of the point's support
           ring(a) U ring(b) U ring(c), padded with the first id
    valid  [n, K] True for real (unpadded) entries
    tri    [n, 3] positions of T's vertices (a, b, c) inside U
    member [n, 3, K] membership of each U entry in ring(a), ring(b), ring(c)
    """

    U: np.ndarray
    valid: np.ndarray
    tri: np.ndarray
    member: np.ndarray

    @classmethod
    def build(cls, triangles, rings):
        """triangles: list of 3 global ids; rings: callable id -> ring ids."""
        n = len(triangles)
        sets = []
        for T in triangles:
            rs = [np.asarray(rings(int(v)), dtype=np.int64) for v in T]
            U = np.unique(np.concatenate(rs))
            sets.append((T, U, rs))
        K = max(len(U) for _, U, _ in sets) if sets else 1
        Ua = np.zeros((n, K), np.int64)
        valid = np.zeros((n, K), bool)
        tri = np.zeros((n, 3), np.int64)
        member = np.zeros((n, 3, K), bool)
        for t, (T, U, rs) in enumerate(sets):
            k = len(U)
            Ua[t, :k] = U
            Ua[t, k:] = U[0]
            valid[t, :k] = True
            tri[t] = np.searchsorted(U, np.asarray(T, dtype=np.int64))
            for q in range(3):
                member[t, q, :k] = np.isin(U, rs[q])
        return cls(Ua, valid, tri, member)


EDGES = ((0, 1), (1, 2), (2, 0))


def interior_weights_local(P, tri, member, valid, r, solver="svd"):
    """psi_mu(r) for every mu in each point's support, eq. (phiquad).

    P [n, K, 2] support positions, tri [n, 3], member [n, 3, K], valid [n, K],
    r [n, 2] the points.  Returns w [n, K] (zero at padding) and, for the SVD
    solver, the rank and singular values of the three edge systems.
    """
    n, K = valid.shape
    idx = np.arange(n)
    Ptri = P[idx[:, None], tri]                      # [n, 3, 2]
    phi = barycentric(Ptri, r)                       # [n, 3]
    w = np.zeros((n, K), dtype=np.result_type(P, r))
    for q in range(3):
        w[idx, tri[:, q]] += phi[:, q]
    ranks, sigmas = [], []
    for (p, q) in EDGES:
        S = (member[:, p] | member[:, q]) & valid    # support of edge (a_p, a_q)
        M, b = edge_system(P, tri[:, p], tri[:, q], S)
        if solver == "svd":
            A, rank, sig = min_norm_svd(M, b, S.sum(-1))
            ranks.append(rank)
            sigmas.append(sig)
        else:
            A = min_norm_normal(M, b)
        w = w + 2.0 * (phi[:, p] * phi[:, q])[:, None] * A
    w = np.where(valid, w, 0.0)
    if solver == "svd":
        return w, np.stack(ranks, 1), np.stack(sigmas, 1)
    return w


def closure_weights_local(P, r, scale, solver="svd"):
    """Closure weights: minimum-norm w with sum_mu w_mu p((r_mu - r)/scale) = p(0).

    P [n, k, 2] the k nearest particles, r [n, 2], scale: length used to make
    the monomials O(1) (the solution does not depend on it).
    """
    X = (P - r[:, None, :]) / scale
    M = np.swapaxes(monomials(X), -1, -2)            # [n, 6, k]
    b = np.zeros(M.shape[:-1], dtype=M.dtype)
    b[..., 0] = 1.0
    if solver == "svd":
        return min_norm_svd(M, b, np.full(M.shape[0], M.shape[-1]))
    return min_norm_normal(M, b)


# ------------------------------------------------------------------ P2M ---

class P2MOracle:
    """Weights psi_mu(r_i) for the nodes of a fixed mesh (eq. p2m).

    mode="global": one Qhull triangulation of the whole cloud.
    mode="local":  per-node certified local triangulations (for clouds too
                   large to triangulate whole; used on sampled nodes).
    """

    def __init__(self, pos, mesh: Mesh, h: float, mode: str = "global"):
        self.pos = np.ascontiguousarray(pos, dtype=np.float64)
        self.mesh = mesh
        self.h = float(h)
        self.mode = mode
        mesh.check_inside(self.pos)
        self.tree = cKDTree(self.pos)
        if mode == "global":
            self.tri: Optional[Triangulation] = Triangulation(self.pos)
        else:
            d, _ = self.tree.query(self.pos[: min(len(self.pos), 4096)], k=2)
            if np.any(d[:, 1] == 0.0):
                from .delaunay import GeometryError
                raise GeometryError("duplicate particles")
            self.tri = None

    # -- classification ------------------------------------------------
    def _interior_structure(self, node_ids):
        """Return (closure mask, triangles) for the given nodes."""
        nodes = self.mesh.nodes()[node_ids]
        closure = self.mesh.on_boundary_ring(node_ids).copy()
        triangles = [None] * len(node_ids)
        ring_cache = {}
        if self.mode == "global":
            s = self.tri.locate(nodes)
            closure |= s < 0
            for t in np.flatnonzero(~closure):
                triangles[t] = self.tri.triangle(s[t])
            return closure, triangles, self.tri.ring
        for t in np.flatnonzero(~closure):
            for mult in (6.0, 10.0, 16.0):
                try:
                    lt = LocalTriangulation(self.pos, self.tree, nodes[t], mult * self.h)
                    st = lt.locate_point()
                    T = lt.triangle_global(st)
                    loc = lt.dt.simplices[st]
                    for v_loc, v in zip(loc, T):
                        ring_cache[int(v)] = lt.ring_global(int(v_loc))
                    triangles[t] = T
                    break
                except LookupError:
                    continue
            else:
                raise LookupError(f"node {node_ids[t]}: no certified local triangulation")
        return closure, triangles, ring_cache.__getitem__

    def node_weights(self, node_ids=None):
        """Rows of the P2M matrix for ``node_ids`` (all nodes by default).

        Returns (cols list, vals list, info) where cols[t], vals[t] are the
        particle ids and weights of node node_ids[t].
        """
        if node_ids is None:
            node_ids = np.arange(self.mesh.n_nodes)
        node_ids = np.asarray(node_ids, dtype=np.int64)
        nodes = self.mesh.nodes()[node_ids]
        closure, triangles, rings = self._interior_structure(node_ids)
        cols = [None] * len(node_ids)
        vals = [None] * len(node_ids)
        info = {"closure": closure, "edge_rank": np.full((len(node_ids), 3), 6),
                "edge_sigma": np.zeros((len(node_ids), 3, 6)),
                "closure_rank": np.full(len(node_ids), 6),
                "closure_sigma": np.zeros((len(node_ids), 6)),
                "triangle": np.full((len(node_ids), 3), -1, np.int64)}
        it = np.flatnonzero(~closure)
        if it.size:
            st = NodeStructure.build([triangles[t] for t in it], rings)
            P = self.pos[st.U]
            w, rank, sig = interior_weights_local(P, st.tri, st.member, st.valid, nodes[it])
            info["edge_rank"][it] = rank
            info["edge_sigma"][it] = sig
            for q, t in enumerate(it):
                m = st.valid[q]
                cols[t] = st.U[q][m]
                vals[t] = w[q][m]
                info["triangle"][t] = triangles[t]
        ic = np.flatnonzero(closure)
        if ic.size:
            k = min(CLOSURE_K, len(self.pos))
            _, nn = self.tree.query(nodes[ic], k=k)
            nn = np.asarray(nn).reshape(len(ic), k)
            w, rank, sig = closure_weights_local(self.pos[nn], nodes[ic], self.h)
            info["closure_rank"][ic] = rank
            info["closure_sigma"][ic] = sig
            for q, t in enumerate(ic):
                order = np.argsort(nn[q], kind="stable")
                cols[t] = nn[q][order]
                vals[t] = w[q][order]
        return cols, vals, info

    def matrix(self, node_ids=None):
        """Sparse P2M matrix W [len(node_ids), N] and the info dict."""
        cols, vals, info = self.node_weights(node_ids)
        indptr = np.zeros(len(cols) + 1, np.int64)
        indptr[1:] = np.cumsum([len(c) for c in cols])
        W = sp.csr_matrix((np.concatenate(vals), np.concatenate(cols), indptr),
                          shape=(len(cols), len(self.pos)))
        W.sum_duplicates()
        return W, info

    def project(self, vals, node_ids=None):
        """Eq. (p2m): alpha_i = sum_mu psi_mu(r_i) alpha_mu, vals [N, C]."""
        W, _ = self.matrix(node_ids)
        return W @ np.asarray(vals, dtype=np.float64)


def linear_fe_matrix(pos, mesh: Mesh):
    """Linear FE P2M (A = 0) at interior nodes inside the hull: rows are the
    barycentric coordinates of each node in its Delaunay triangle (eqs. C0, C1);
    other rows are empty.  Used as the control that fails eq. C2 (eq. noC2)."""
    tri = Triangulation(pos)
    nodes = mesh.nodes()
    ids = np.arange(mesh.n_nodes)
    s = tri.locate(nodes)
    ok = (~mesh.on_boundary_ring(ids)) & (s >= 0)
    T = tri.simplices[s[ok]]
    phi = barycentric(pos[T], nodes[ok])
    rows = np.repeat(np.flatnonzero(ok), 3)
    return sp.csr_matrix((phi.ravel(), (rows, T.ravel())), shape=(mesh.n_nodes, len(pos))), ok


def psi_at(tri: Triangulation, pts):
    """psi_mu(r) at arbitrary points inside the hull (eq. phiquad).

    Returns (U [n, K] ids, valid [n, K], w [n, K], edge ranks [n, 3]).
    """
    pts = np.ascontiguousarray(pts, dtype=np.float64)
    s = tri.locate(pts)
    if np.any(s < 0):
        raise ValueError("psi_at: point outside the convex hull")
    st = NodeStructure.build([tri.triangle(t) for t in s], tri.ring)
    w, rank, _ = interior_weights_local(tri.pos[st.U], st.tri, st.member, st.valid, pts)
    return st.U, st.valid, w, rank
