"""Full-size GPU parity of the two largest workloads, sampled against the
oracle (it cannot triangulate millions of particles whole, so it builds the
rows of sampled nodes from certified local triangulations, App. B).

* 512 x 512 mesh, 2048^2 jittered lattice (4.2 M particles): M2P -> P2M ->
  loss -> full backward, FP64 and mixed (FP32 values, FP64 geometry).
* 1024 x 1024 mesh, 4096^2 lattice advected 200 Euler steps (16.8 M
  particles), BF16 particle storage: forward P2M and M2P, backward of a P2M
  loss, against the oracle on the BF16-rounded inputs (arithmetic error)
  and on the unrounded FP64 inputs (quantisation included).

Gradients at a sampled particle need every node whose support holds it;
supports reach about 4h from the node, so the rows of all nodes within
2.5 H (10h at h = H/4) of the particle are built, which makes the sampled
gradient exact.
"""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle import Mesh as OMesh, P2MOracle, m2p as o_m2p, m2p_grad_pos as o_m2p_grad_pos, m2p_matrix
from oracle.adjoint import p2m_grad_pos as o_p2m_grad_pos
from paper_1610_05266_amd import autograd, ops
from tests._util import assert_close, rel_errs

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _g(a, dt=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dt)


def _sample_particles(c, om, tree, rng, n):
    """Half uniformly drawn particles, half the nearest particle of a random
    interior node (those always carry weight; a particle in no node's support
    has zero gradient and would test nothing)."""
    inner = np.flatnonzero(~om.on_boundary_ring(np.arange(om.n_nodes)))
    near = tree.query(om.nodes()[rng.choice(inner, n - n // 2, replace=False)])[1]
    return np.unique(np.concatenate([rng.choice(c.N, n // 2, replace=False), near]))


def _nodes_near(om, pts, R):
    """Ids of the nodes inside the square of half-width R around each point."""
    out = []
    for x, y in np.atleast_2d(pts):
        i0 = max(0, int(np.floor((x - om.x0 - R) / om.H)))
        i1 = min(om.nx, int(np.ceil((x - om.x0 + R) / om.H)))
        j0 = max(0, int(np.floor((y - om.y0 - R) / om.H)))
        j1 = min(om.ny, int(np.ceil((y - om.y0 + R) / om.H)))
        jj, ii = np.meshgrid(np.arange(j0, j1 + 1), np.arange(i0, i1 + 1), indexing="ij")
        out.append((jj * (om.nx + 1) + ii).ravel())
    return np.unique(np.concatenate(out))


@pytest.fixture(scope="module")
def c4():
    c = wl.config4()
    om = OMesh.from_spec(c.mesh)
    print(f"C4: N={c.N} nodes={om.n_nodes}", flush=True)
    return c, om, P2MOracle(c.pos, om, c.h, mode="local")


def _roundtrip(c, dtype):
    mesh = ops.Mesh.of(c.mesh)
    pos = _g(c.pos).requires_grad_(True)
    fm = _g(c.extra["f_mesh"], dtype).requires_grad_(True)
    a = autograd.m2p(fm, pos, mesh)
    out = autograd.p2m(pos, a, mesh, c.h)
    loss = 0.5 * ((out.double() - _g(c.extra["g_mesh"])) ** 2).sum()
    loss.backward()
    return (out.detach().double().cpu().numpy(), pos.grad.cpu().numpy(), fm.grad.double().cpu().numpy(),
            loss.item())


def test_c4_full_backward_sampled_against_oracle(c4):
    c, om, orc = c4
    out64, gp64, gf64, L64 = _roundtrip(c, torch.float64)
    out32, gp32, gf32, L32 = _roundtrip(c, torch.float32)
    assert abs(L32 - L64) <= 1e-5 * L64
    rng = np.random.default_rng(4)
    parts = _sample_particles(c, om, orc.tree, rng, 16)
    snodes = np.unique(np.concatenate([rng.choice(om.n_nodes, 8, replace=False),
                                       [0, om.nx // 2, om.n_nodes - 1]]))
    # nodes whose residual the sampled gradients need (see module docstring);
    # the mesh-input gradient at a node needs the particles of its six
    # triangles (within H), hence nodes within 3.5 H
    nodes = np.union1d(_nodes_near(om, c.pos[parts], 2.5 * om.H),
                       _nodes_near(om, om.nodes()[snodes], 3.5 * om.H))
    W, _ = orc.matrix(nodes)
    g = c.extra["g_mesh"]
    f64 = c.extra["f_mesh"]
    # The mixed path stores the mesh input and the particle values of M2P in
    # FP32: its reference is the oracle on those FP32-rounded arrays (the
    # mesh input rounded, the oracle's M2P rounded once, as the GPU's M2P
    # rounds its FP64 sum once).  Rounding either array moves dL/dpos by
    # ~1e-5 of its terms (see below), which is the storage's doing, not the
    # arithmetic's: that total is reported, and bounded, separately.
    f32 = f64.astype(np.float32).astype(np.float64)
    near = np.flatnonzero(np.asarray(abs(m2p_matrix(om, c.pos)[:, snodes]).sum(1)).ravel() > 0)
    a64 = o_m2p(om, f64, c.pos)
    a32 = o_m2p(om, f32, c.pos).astype(np.float32).astype(np.float64)
    ref_terms = {}
    for f, a, out_g, gp_g, gf_g, tol, gtol, what in (
            (f64, a64, out64, gp64, gf64, 1e-12, 1e-10, "FP64"),
            (f32, a32, out32, gp32, gf32, 1e-5, 1e-5, "mixed")):
        out = W @ a
        r = out - g[nodes]
        assert_close(out_g[nodes], out, tol, f"C4 P2M(M2P f) at sampled nodes, {what}")
        abar = W.T @ r
        g_p2m = o_p2m_grad_pos(orc, a, r, node_ids=nodes)[parts]
        g_m2p = o_m2p_grad_pos(om, f, c.pos[parts], abar[parts])
        gp = g_p2m + g_m2p
        # The weight term and the M2P term of dL/dpos nearly cancel (P2M(M2P f)
        # follows f as particles move), by about three orders of magnitude
        # here, so the error is measured against the size of the two terms.
        scale = np.abs(g_p2m) + np.abs(g_m2p)
        d = gp_g[parts] - gp
        nrm = np.linalg.norm(d) / np.linalg.norm(scale)
        mx = np.abs(d).max() / scale.max()
        print(f"C4 dL/dpos {what}: normwise {nrm:.3e}, max {mx:.3e} (of the terms)", flush=True)
        assert nrm <= gtol and mx <= gtol, f"C4 dL/dpos {what}: {nrm:.3e} {mx:.3e} > {gtol:.1e}"
        if what == "FP64":
            assert_close(gp64[parts], gp, 1e-7, "C4 dL/dpos, FP64, relative to the sum")
            ref_terms = dict(gp=gp, scale=scale)
        gf = m2p_matrix(om, c.pos[near])[:, snodes].T @ abar[near]
        assert_close(gf_g[snodes], gf, gtol, f"C4 dL/df, {what}")
    # the mixed form against the unrounded FP64 reference: the storage
    # rounding included (measured ~1.5e-5 of the terms; bounded at 1e-4)
    d = gp32[parts] - ref_terms["gp"]
    tot = (np.linalg.norm(d) / np.linalg.norm(ref_terms["scale"]), np.abs(d).max() / ref_terms["scale"].max())
    print(f"C4 dL/dpos mixed vs unrounded FP64 reference (storage included): {tot[0]:.3e}, {tot[1]:.3e}", flush=True)
    assert max(tot) <= 1e-4


def test_c4_recompute_mode_gives_the_stored_mode_gradients(c4):
    """At full size the autograd P2M may keep no weights between forward and
    backward (rebuilt in backward); the build is deterministic, so the
    forward is bitwise the same and the position gradient equal up to the
    order of its atomic sums."""
    c, om, _ = c4
    mesh = ops.Mesh.of(c.mesh)
    res = []
    for rec in (False, True):
        pos = _g(c.pos).requires_grad_(True)
        a = _g(c.vals, torch.float32).requires_grad_(True)
        out = autograd.p2m(pos, a, mesh, c.h, recompute=rec)
        (0.5 * ((out.double() - _g(c.extra["g_mesh"])) ** 2).sum()).backward()
        res.append((out.detach(), pos.grad))
    assert torch.equal(res[0][0], res[1][0])
    assert torch.allclose(res[0][1], res[1][1], rtol=0, atol=1e-12 * res[0][1].abs().max().item())


def test_c4_full_size_properties(c4):
    """Every node reproduces a quadratic; the FP64 build is bitwise
    repeatable; the diagnostics are clean."""
    c, om, _ = c4
    pos = _g(c.pos)
    w = ops.p2m_build_weights(c.mesh, c.h, pos)
    d = w.diag()
    assert d["status"] == 0 and d["failed_nodes"] == 0 and d["rank_deficient"] == 0
    assert d["interior_nodes"] + d["closure_nodes"] == om.n_nodes
    q = wl.quad_q(c.pos[:, 0], c.pos[:, 1])[:, None]
    mq = ops.p2m_project(w, _g(q)).cpu().numpy()[:, 0]
    ref = wl.quad_q(*om.nodes().T)
    assert np.abs(mq - ref).max() <= 1e-10 * np.abs(ref).max()
    i1, x1, _, _ = w.export()
    w2 = ops.p2m_build_weights(c.mesh, c.h, pos)
    i2, x2, _, _ = w2.export()
    assert torch.equal(i1, i2) and torch.equal(x1, x2)


@pytest.fixture(scope="module")
def c5():
    # input generation only: the advection runs on torch (on the GPU for speed)
    c = wl.config5(device=DEV)
    om = OMesh.from_spec(c.mesh)
    print(f"C5: N={c.N} nodes={om.n_nodes}", flush=True)
    return c, om, P2MOracle(c.pos, om, c.h, mode="local")


def test_c5_bf16_forward_backward_sampled_against_oracle(c5):
    c, om, orc = c5
    mesh = ops.Mesh.of(c.mesh)
    vb = _g(c.vals, torch.bfloat16)
    vr = vb.double().cpu().numpy()            # the BF16-rounded inputs
    nodes_xy = om.nodes()
    target = np.stack([wl.tg_u(nodes_xy[:, 0] - 0.05, nodes_xy[:, 1] + 0.03),
                       wl.tg_v(nodes_xy[:, 0] - 0.05, nodes_xy[:, 1] + 0.03),
                       wl.tg_p(nodes_xy[:, 0] - 0.05, nodes_xy[:, 1] + 0.03)], 1)
    pos = _g(c.pos).requires_grad_(True)
    v = vb.clone().requires_grad_(True)
    out = autograd.p2m(pos, v, mesh, c.h)
    assert out.dtype == torch.float32
    back = autograd.m2p(out.detach(), pos.detach(), mesh, bf16_out=True)
    loss = 0.5 * ((out.double() - _g(target)) ** 2).sum()
    loss.backward()
    out = out.detach().double().cpu().numpy()
    gp = pos.grad.cpu().numpy()
    gv = v.grad.double().cpu().numpy()

    rng = np.random.default_rng(5)
    parts = _sample_particles(c, om, orc.tree, rng, 16)
    snodes = np.unique(np.concatenate([rng.choice(om.n_nodes, 48, replace=False), [0, om.n_nodes - 1]]))
    nodes = np.union1d(_nodes_near(om, c.pos[parts], 2.5 * om.H), snodes)
    W, _ = orc.matrix(nodes)
    ref = W @ vr
    assert_close(out[nodes], ref, 1e-5, "C5 P2M vs oracle on BF16-rounded inputs")
    e_total = rel_errs(out[nodes], W @ c.vals)
    print(f"C5 P2M vs oracle on unrounded inputs (BF16 quantisation): {e_total}", flush=True)
    assert max(e_total) <= 1e-2
    # M2P of the P2M result, BF16 output storage, every particle
    ob = back.float().cpu().numpy()
    assert_close(ob, o_m2p(om, out, c.pos), 8e-3, "C5 M2P, BF16 output")
    r = ref - target[nodes]
    gv_ref = (W.T @ r)[parts]
    assert_close(gv[parts], gv_ref, 1e-2, "C5 dL/dvals (BF16 gradient storage)")
    gp_ref = o_p2m_grad_pos(orc, vr, r, node_ids=nodes)[parts]
    assert_close(gp[parts], gp_ref, 1e-5, "C5 dL/dpos")
