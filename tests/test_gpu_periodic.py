"""GPU parity of the periodic box (P2M_PERIODIC) against the periodic oracle.

The paper's runs are periodic (App. A: a periodic Delaunay triangulation):
a particle enters a node's weights at its image nearest to the node, there
are no closure nodes, and the mesh keeps the bounded layout with node
(nx, j) = (0, j) and (i, ny) = (i, 0).  Rows, triangles and P2M values are
compared element by element with the oracle on the paper's Taylor-Green box
(-1, 1)^2 with k = pi.  FP64 bar 1e-12 (as the bounded build), FP32 1e-5.
"""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle import Mesh as OMesh, PeriodicP2MOracle
from paper_1610_05266_amd import ops
from tests._util import assert_close, ell_to_csr

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _gpu(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dtype)


def _case(n, ratio, jitter, seed):
    c = wl.periodic_tg_cloud(n, ratio, jitter, seed)
    W, info = PeriodicP2MOracle(c.pos, OMesh.from_spec(c.mesh), c.h).matrix()
    return c, W, info


def _check_rows(c, W, info, w):
    d = w.diag()
    assert d["failed_nodes"] == 0 and d["closure_nodes"] == 0 and d["outside_hull_nodes"] == 0, d
    assert d["interior_nodes"] == c.mesh.n_nodes
    idx, wt, cnt, tri = w.export()
    G = ell_to_csr(idx.numpy(), wt.numpy(), cnt.numpy(), c.N)
    assert ((G != 0).astype(int) != (W != 0).astype(int)).nnz == 0
    assert abs(G - W).max() <= 1e-12
    assert np.array_equal(np.sort(tri.numpy(), 1), np.sort(info["triangle"], 1))
    return d, idx, wt, cnt, tri


@pytest.fixture(scope="module")
def small():
    return _case(16, 2, 0.3, 11)


@pytest.fixture(scope="module")
def medium():
    # 64 x 64 cells: most nodes take the fast pass, those whose search window
    # reaches a box side the exact path, whose regions wrap
    return _case(64, 2, 0.3, 12)


def test_periodic_rows_match_oracle_small(small):
    c, W, info = small
    print(f"[gpu] periodic build {c.name} N={c.N}", flush=True)
    w = ops.p2m_build_weights(c.mesh, c.h, _gpu(c.pos), ops.P2M_PERIODIC)
    _check_rows(c, W, info, w)


def test_periodic_rows_match_oracle_with_fast_tiles(medium):
    c, W, info = medium
    print(f"[gpu] periodic build {c.name} N={c.N}", flush=True)
    w = ops.p2m_build_weights(c.mesh, c.h, _gpu(c.pos), ops.P2M_PERIODIC)
    d, *_ = _check_rows(c, W, info, w)
    assert 0 < d["slow_nodes"] < d["interior_nodes"] - 1000, d


def test_periodic_p2m_values_and_seam(medium):
    c, W, info = medium
    pos = _gpu(c.pos)
    w = ops.p2m_build_weights(c.mesh, c.h, pos, ops.P2M_PERIODIC | ops.P2M_WEIGHTS_F32)
    got = ops.p2m_project(w, _gpu(c.vals)).cpu().numpy()
    assert_close(got, W @ c.vals, 1e-12, "periodic P2M FP64")
    got32 = ops.p2m_project(w, _gpu(c.vals, torch.float32)).cpu().numpy()
    assert_close(got32, W @ c.vals, 1e-5, "periodic P2M FP32")
    # the seam nodes repeat the first column and row bit for bit
    n1 = c.mesh.nx + 1
    g = got.reshape(c.mesh.ny + 1, n1, -1)
    assert np.array_equal(g[:, -1], g[:, 0]) and np.array_equal(g[-1], g[0])
    # the projection of the periodic Taylor-Green field is close to the field
    nodes = OMesh.from_spec(c.mesh).nodes()
    want = np.stack([wl.tg_u(nodes[:, 0], nodes[:, 1]), wl.tg_v(nodes[:, 0], nodes[:, 1])], 1)
    assert np.abs(got[:, :2] - want).max() < 2e-3


def test_periodic_round_trip_with_m2p(small):
    """M2P needs no flag on the repeated-seam layout: the round trip of a
    periodic mesh field equals the oracle's W @ M2P."""
    from oracle import m2p as o_m2p
    c, W, info = small
    om = OMesh.from_spec(c.mesh)
    nodes = om.nodes()
    f = np.stack([wl.tg_u(nodes[:, 0], nodes[:, 1]), wl.tg_p(nodes[:, 0], nodes[:, 1])], 1)
    pos = _gpu(c.pos)
    w = ops.p2m_build_weights(c.mesh, c.h, pos, ops.P2M_PERIODIC)
    a = ops.m2p_interpolate(c.mesh, _gpu(f), pos)
    assert_close(ops.p2m_project(w, a).cpu().numpy(), W @ o_m2p(om, f, c.pos), 1e-12, "periodic round trip")


@pytest.mark.parametrize("fast_radius,region_h", [(1.5, 1.0), (3.0, 6.0)])
def test_periodic_options_change_no_bit(medium, fast_radius, region_h):
    c, W, info = medium
    pos = _gpu(c.pos)
    ref = ops.p2m_build_weights(c.mesh, c.h, pos, ops.P2M_PERIODIC).export()
    saved = {k: ops.p2m_get_option(k) for k in ("fast_radius", "region_h")}
    try:
        ops.p2m_set_option("fast_radius", fast_radius)
        ops.p2m_set_option("region_h", region_h)
        got = ops.p2m_build_weights(c.mesh, c.h, pos, ops.P2M_PERIODIC).export()
    finally:
        for k, v in saved.items():
            ops.p2m_set_option(k, v)
    for g, r, name in zip(got, ref, ("idx", "w", "cnt", "tri")):
        assert torch.equal(g, r), name


def test_periodic_linear_rows(small):
    c, W, info = small
    w = ops.p2m_build_weights(c.mesh, c.h, _gpu(c.pos), ops.P2M_PERIODIC | ops.P2M_LINEAR)
    idx, wt, cnt, tri = w.export()
    assert np.array_equal(np.sort(tri.numpy(), 1), np.sort(info["triangle"], 1))
    assert (cnt.numpy() == 3).all()
    G = ell_to_csr(idx.numpy(), wt.numpy(), cnt.numpy(), c.N)
    assert np.abs(np.asarray(G.sum(1)).ravel() - 1.0).max() < 1e-12


def test_periodic_batched_equals_single_builds():
    cs = [wl.periodic_tg_cloud(8, 2, 0.3, 21), wl.periodic_tg_cloud(12, 3, 0.25, 22)]
    off = np.cumsum([0] + [c.N for c in cs])
    b = ops.Batch([c.mesh for c in cs], [c.h for c in cs], off)
    pos = _gpu(np.concatenate([c.pos for c in cs]))
    wb = ops.p2m_build_weights_batched(b, pos, ops.P2M_PERIODIC)
    ib, xb, cb, tb = (t.numpy() for t in wb.export())
    for s, c in enumerate(cs):
        n0, n1 = b.node_offsets[s], b.node_offsets[s + 1]
        ws = ops.p2m_build_weights(c.mesh, c.h, _gpu(c.pos), ops.P2M_PERIODIC)
        i1, x1, c1, t1 = (t.numpy() for t in ws.export())
        p0 = b.offsets[s]
        assert np.array_equal(cb[n0:n1], c1)
        assert np.array_equal(xb[:, n0:n1], x1)
        assert np.array_equal(np.where(i1 >= 0, i1 + p0, -1), ib[:, n0:n1])
        assert np.array_equal(np.where(t1 >= 0, t1 + p0, -1), tb[n0:n1])


def test_periodic_position_gradient_matches_oracle(small):
    """d/dr of sum gbar * P2M(vals) through the periodic weights: the
    adjoint kernels against the oracle's complex-step derivative on image
    positions (FP64 gradients, 1e-10)."""
    from oracle.periodic import periodic_p2m_grad_pos
    c, W, info = small
    orc = PeriodicP2MOracle(c.pos, OMesh.from_spec(c.mesh), c.h)
    gmesh = np.random.default_rng(3).normal(size=(c.mesh.n_nodes, c.vals.shape[1]))
    pos = _gpu(c.pos)
    w = ops.p2m_build_weights(c.mesh, c.h, pos, ops.P2M_PERIODIC)
    _, gw = ops.p2m_project_backward(w, _gpu(gmesh), _gpu(c.vals), want_vals=False, want_w=True)
    gp = ops.p2m_build_weights_backward(w, pos, gw).cpu().numpy()
    assert_close(gp, periodic_p2m_grad_pos(orc, c.vals, gmesh), 1e-10, "periodic P2M grad pos")


def test_periodic_rejections():
    c = wl.periodic_tg_cloud(16, 2, 0.3, 11)
    pos = _gpu(c.pos)
    small = wl.MeshSpec(3, 3, 2.0 / 3, -1.0, -1.0)
    with pytest.raises(ops.P2MError):
        ops.p2m_build_weights(small, c.h, pos, ops.P2M_PERIODIC)


@pytest.fixture(scope="module")
def full():
    # the benchmark's periodic workload: 256 x 256 cells on (-1, 1)^2, a
    # 1024 x 1024 jittered lattice (h = H/4, jitter 0.3h, seed 2)
    c = wl.periodic_tg_cloud(256, 4, 0.30, 2)
    pos = _gpu(c.pos)
    print(f"[gpu] periodic build {c.name} N={c.N}", flush=True)
    w = ops.p2m_build_weights(c.mesh, c.h, pos, ops.P2M_PERIODIC)
    return c, pos, w


def test_periodic_full_size_consistency(full):
    """Eqs. C0, C1, C2 at every node in minimum-image offsets (a wrong image
    is off by a period, 256 mesh spacings)."""
    c, pos, w = full
    d = w.diag()
    assert d["failed_nodes"] == 0 and d["closure_nodes"] == 0 and d["interior_nodes"] == c.mesh.n_nodes
    idx, wt, cnt, tri = (t.numpy() for t in w.export())
    m = OMesh.from_spec(c.mesh)
    from oracle.periodic import wrapped_nodes
    nodes = wrapped_nodes(m)
    L = np.array([m.nx * m.H, m.ny * m.H])
    valid = np.arange(idx.shape[0])[:, None] < cnt[None, :]
    P = c.pos[np.where(valid, idx, 0)]
    off = P - nodes[None]
    off -= L * np.rint(off / L)
    s = off / m.H
    ww = np.where(valid, wt, 0.0)
    assert np.abs(ww.sum(0) - 1.0).max() < 1e-12
    assert np.abs(np.einsum("kn,kna->na", ww, s)).max() < 1e-10
    assert np.abs(np.einsum("kn,kna,knb->nab", ww, s, s)).max() < 1e-10


def test_periodic_full_size_sampled_oracle_rows(full):
    """Sampled nodes (box corners and sides among them) against the oracle's
    certified local triangulation of the cloud translated by half a period,
    which puts the node far from every side of the bounded box."""
    from oracle import P2MOracle
    c, pos, w = full
    idx, wt, cnt, tri = (t.numpy() for t in w.export())
    m = OMesh.from_spec(c.mesh)
    L = m.nx * m.H
    shifted = c.pos + L / 2
    shifted[shifted >= m.x0 + L] -= L
    orc = P2MOracle(shifted, m, c.h, mode="local")
    rng = np.random.default_rng(5)
    # (translated by half a period, nodes near the middle of the box would
    # land next to the bounded box's sides: they are not sampled)
    ij = [(0, 0), (1, 0), (0, 1), (255, 255), (256, 3), (7, 256), (256, 256), (100, 0), (0, 200)]
    ij += [tuple(v) for v in rng.integers(0, 257, size=(40, 2)) if min(abs(v % 256 - 128)) > 10][:12]
    n1 = m.nx + 1
    ks = [j * n1 + i for i, j in ij]
    kshift = [((j % m.ny + m.ny // 2) % m.ny) * n1 + (i % m.nx + m.nx // 2) % m.nx for i, j in ij]
    cols, vals, _ = orc.node_weights(np.asarray(kshift))
    for k, cc, vv in zip(ks, cols, vals):
        n = cnt[k]
        got = dict(zip(idx[:n, k].tolist(), wt[:n, k].tolist()))
        assert sorted(got) == sorted(cc.tolist()), k
        assert max(abs(got[u] - x) for u, x in zip(cc.tolist(), vv.tolist())) < 1e-11, k


def test_periodic_voids_across_the_sides():
    """Voids centred on the box corner and on a side, and a cluster across
    the right side: searches escalate through wrapped regions (up to the
    whole box at nearest images) and still match the oracle."""
    c = wl.periodic_void_cloud(16, 3000, 9)
    W, info = PeriodicP2MOracle(c.pos, OMesh.from_spec(c.mesh), c.h).matrix()
    print(f"[gpu] periodic build {c.name} N={c.N}", flush=True)
    w = ops.p2m_build_weights(c.mesh, c.h, _gpu(c.pos), ops.P2M_PERIODIC)
    d = w.diag()
    assert d["failed_nodes"] == 0 and d["closure_nodes"] == 0 and d["escalated_nodes"] > 0, d
    idx, wt, cnt, tri = w.export()
    assert np.array_equal(np.sort(tri.numpy(), 1), np.sort(info["triangle"], 1))
    got = ops.p2m_project(w, _gpu(c.vals)).cpu().numpy()
    assert_close(got, W @ c.vals, 1e-12, "periodic voids P2M")
