"""Derivatives of P2M and M2P (oracle; test infrastructure only).

The paper has no adjoint; these are the derivatives of its forward
construction (eqs. p2m, m2p, phiquad, A0, A1, A2_2):

* w.r.t. particle values: P2M and M2P are linear in the values, so their
  adjoints are the transposed matrices.
* w.r.t. particle positions: the weights psi_mu(r_i) are smooth functions of
  the positions while the combinatorial structure (Delaunay triangle of the
  node, rings, nearest-neighbour set of closure nodes, mesh triangle of a
  particle) stays fixed.  The oracle differentiates its own forward
  construction by complex step: perturb one coordinate by i*delta, evaluate
  the weights in complex arithmetic (normal-equation form of the minimum-norm
  solve, which is holomorphic), and read d w / d x = Im(w) / delta.  This is
  exact to rounding and independent of any hand-derived chain rule.
"""
from __future__ import annotations

import numpy as np

from .m2p import m2p_grad_pos, m2p_matrix
from .qcsf import (NodeStructure, P2MOracle, closure_weights_local,
                   interior_weights_local, CLOSURE_K)

CS_STEP = 1e-30


def p2m_weight_jacobian_contract(orc: P2MOracle, wbar_fn, node_ids=None):
    """sum_i sum_mu wbar[i, mu] * d w[i, mu] / d r_nu for every particle nu.

    ``wbar_fn(node_ids, cols)`` returns wbar for each node's support columns
    (list of arrays aligned with ``cols``).  Returns grad [N, 2].
    """
    if node_ids is None:
        node_ids = np.arange(orc.mesh.n_nodes)
    node_ids = np.asarray(node_ids, dtype=np.int64)
    nodes = orc.mesh.nodes()[node_ids]
    closure, triangles, rings = orc._interior_structure(node_ids)
    grad = np.zeros_like(orc.pos)

    it = np.flatnonzero(~closure)
    if it.size:
        st = NodeStructure.build([triangles[t] for t in it], rings)
        wbar = np.zeros(st.U.shape)
        cols = [st.U[q][st.valid[q]] for q in range(len(it))]
        wb = wbar_fn(node_ids[it], cols)
        for q in range(len(it)):
            wbar[q, : len(cols[q])] = wb[q]
        P = orc.pos[st.U].astype(np.complex128)
        r = nodes[it].astype(np.complex128)
        K = st.U.shape[1]
        for k in range(K):
            for d in range(2):
                Pc = P.copy()
                Pc[:, k, d] += 1j * CS_STEP
                w = interior_weights_local(Pc, st.tri, st.member, st.valid, r, solver="normal")
                dw = w.imag / CS_STEP
                contrib = (wbar * dw).sum(1)
                m = st.valid[:, k]
                np.add.at(grad[:, d], st.U[m, k], contrib[m])

    ic = np.flatnonzero(closure)
    if ic.size:
        k = min(CLOSURE_K, len(orc.pos))
        _, nn = orc.tree.query(nodes[ic], k=k)
        nn = np.asarray(nn).reshape(len(ic), k)
        wb = np.stack(wbar_fn(node_ids[ic], [nn[q] for q in range(len(ic))]))
        P = orc.pos[nn].astype(np.complex128)
        r = nodes[ic].astype(np.complex128)
        for s in range(k):
            for d in range(2):
                Pc = P.copy()
                Pc[:, s, d] += 1j * CS_STEP
                w = closure_weights_local(Pc, r, orc.h, solver="normal")
                dw = w.imag / CS_STEP
                np.add.at(grad[:, d], nn[:, s], (wb * dw).sum(1))
    return grad


def p2m_grad_pos(orc: P2MOracle, vals, gbar_mesh, node_ids=None):
    """d/d r of L = sum_{i,c} gbar[i,c] * (P2M vals)[i,c] (positions only)."""
    vals = np.asarray(vals, dtype=np.float64)
    if node_ids is None:
        node_ids = np.arange(orc.mesh.n_nodes)
    g = np.asarray(gbar_mesh, dtype=np.float64)
    lookup = {int(n): q for q, n in enumerate(np.asarray(node_ids))}

    def wbar_fn(ids, cols):
        return [vals[c] @ g[lookup[int(i)]] for i, c in zip(ids, cols)]

    return p2m_weight_jacobian_contract(orc, wbar_fn, node_ids)


def p2m_grad_vals(W, gbar_mesh):
    """Adjoint of eq. (p2m) w.r.t. particle values: W^t gbar."""
    return W.T @ np.asarray(gbar_mesh, dtype=np.float64)


def m2p_grad_mesh(mesh, pos, gbar_particles):
    """Adjoint of eq. (m2p) w.r.t. mesh values: M^t gbar."""
    return m2p_matrix(mesh, pos).T @ np.asarray(gbar_particles, dtype=np.float64)


def roundtrip(orc: P2MOracle, f_mesh, g_mesh):
    """Loss L = 1/2 sum_{i,c} (P2M(M2P(f))_{i,c} - g_{i,c})^2 and its gradients.

    Returns dict with the loss, the particle values a = M2P(f), the mesh result,
    dL/da (gradient w.r.t. the particle values), dL/dr (positions, through both
    operators) and dL/df (mesh input).
    """
    mesh, pos = orc.mesh, orc.pos
    Mm = m2p_matrix(mesh, pos)
    a = Mm @ np.asarray(f_mesh, dtype=np.float64)
    W, _ = orc.matrix()
    out = W @ a
    resid = out - np.asarray(g_mesh, dtype=np.float64)
    loss = 0.5 * float((resid * resid).sum())
    ga = W.T @ resid
    gpos = p2m_grad_pos(orc, a, resid) + m2p_grad_pos(mesh, f_mesh, pos, ga)
    gf = Mm.T @ ga
    return {"loss": loss, "a": a, "out": out, "resid": resid,
            "grad_vals": ga, "grad_pos": gpos, "grad_mesh": gf}
