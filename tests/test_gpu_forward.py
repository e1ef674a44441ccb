"""GPU parity of the forward path against the CPU FP64 oracle (small sizes).

P2M (eq. p2m with the App. B shape functions) and M2P (eq. m2p with linear FE
mesh functions) through the C ABI, compared element by element with the
oracle on the same seeded inputs.  FP64 bar: 1e-12 normwise and max-relative.
"""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle import Mesh as OMesh, P2MOracle, m2p as o_m2p
from paper_1610_05266_amd import ops
from tests._util import assert_close, ell_to_csr

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
TOL64 = 1e-12
TOL32 = 1e-5


def _gpu(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dtype)


def _build(cloud, flags=0):
    print(f"[gpu] build {cloud.name} N={cloud.N} nodes={cloud.mesh.n_nodes}", flush=True)
    pos = _gpu(cloud.pos)
    w = ops.p2m_build_weights(cloud.mesh, cloud.h, pos, flags)
    return w, pos


@pytest.fixture(scope="module")
def c1():
    c = wl.config1()
    orc = P2MOracle(c.pos, OMesh.from_spec(c.mesh), c.h)
    W, info = orc.matrix()
    return c, orc, W, info


def test_c1_weights_and_triangles_match_oracle(c1):
    c, orc, W, info = c1
    w, pos = _build(c)
    d = w.diag()
    assert d["near_degenerate"] == 0 and d["failed_nodes"] == 0 and d["rank_deficient"] == 0
    assert d["closure_nodes"] == int(info["closure"].sum())
    assert d["interior_nodes"] == c.mesh.n_nodes - d["closure_nodes"]
    idx, wt, cnt, tri = w.export()
    G = ell_to_csr(idx.numpy(), wt.numpy(), cnt.numpy(), c.N)
    # same support (integer-exact) and weights to FP64 rounding
    assert ((G != 0).astype(int) != (W != 0).astype(int)).nnz == 0
    assert abs(G - W).max() <= 1e-12
    inter = ~info["closure"]
    gt = np.sort(tri.numpy()[inter], axis=1)
    ot = np.sort(info["triangle"][inter], axis=1)
    assert np.array_equal(gt, ot)


def test_c1_p2m_values_fp64_and_quadratic(c1):
    c, orc, W, info = c1
    w, pos = _build(c)
    vals = _gpu(c.vals)
    got = ops.p2m_project(w, vals).cpu().numpy()
    assert_close(got, W @ c.vals, TOL64, "P2M FP64")
    # quadratic reproduction on the GPU (eq. C2) at every node, closure included
    nodes = OMesh.from_spec(c.mesh).nodes()
    q = _gpu(np.stack([c.pos[:, 0] ** 2, c.pos[:, 0] * c.pos[:, 1], c.pos[:, 1] ** 2,
                       np.ones(c.N)], 1))
    got = ops.p2m_project(w, q).cpu().numpy()
    want = np.stack([nodes[:, 0] ** 2, nodes[:, 0] * nodes[:, 1], nodes[:, 1] ** 2, np.ones(len(nodes))], 1)
    assert np.abs(got - want).max() <= 1e-10


def test_c1_m2p_fp64(c1):
    c, *_ = c1
    om = OMesh.from_spec(c.mesh)
    nodes = om.nodes()
    mv = np.stack([wl.tg_u(nodes[:, 0], nodes[:, 1]), wl.tg_v(nodes[:, 0], nodes[:, 1]),
                   wl.quad_q(nodes[:, 0], nodes[:, 1])], 1)
    got = ops.m2p_interpolate(c.mesh, _gpu(mv), _gpu(c.pos)).cpu().numpy()
    assert_close(got, o_m2p(om, mv, c.pos), TOL64, "M2P FP64")


def test_c1_round_trip_fp64_and_mixed(c1):
    c, orc, W, info = c1
    om = OMesh.from_spec(c.mesh)
    nodes = om.nodes()
    f = np.stack([wl.tg_u(nodes[:, 0], nodes[:, 1]), wl.tg_v(nodes[:, 0], nodes[:, 1])], 1)
    ref = W @ o_m2p(om, f, c.pos)
    pos = _gpu(c.pos)
    w = ops.p2m_build_weights(c.mesh, c.h, pos, ops.P2M_WEIGHTS_F32)
    a64 = ops.m2p_interpolate(c.mesh, _gpu(f), pos)
    assert_close(ops.p2m_project(w, a64).cpu().numpy(), ref, TOL64, "round trip FP64")
    a32 = ops.m2p_interpolate(c.mesh, _gpu(f, torch.float32), pos)
    assert_close(ops.p2m_project(w, a32).cpu().numpy(), ref, TOL32, "round trip FP32")


def test_h_is_only_a_hint_and_builds_are_deterministic():
    c = wl.small_cloud(24, 2, 0.25, seed=5)
    pos = _gpu(c.pos)
    vals = _gpu(c.vals)
    outs = []
    for h in (c.h, c.h, 0.5 * c.h, 2.7 * c.h):
        w = ops.p2m_build_weights(c.mesh, h, pos)
        outs.append(ops.p2m_project(w, vals).cpu().numpy())
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


def test_cluster_and_void_cloud():
    c = wl.cluster_void_cloud(16, 3000, seed=7)
    om = OMesh.from_spec(c.mesh)
    orc = P2MOracle(c.pos, om, c.h)
    W, info = orc.matrix()
    w, pos = _build(c)
    d = w.diag()
    assert d["failed_nodes"] == 0
    got = ops.p2m_project(w, _gpu(c.vals)).cpu().numpy()
    assert_close(got, W @ c.vals, TOL64, "cluster P2M")


@pytest.mark.parametrize("fast_radius,region_h,bin_scale,min_slow_share",
                         [(1.5, 1.0, 1.0, 0.5), (2.8, 4.0, 1.0, 0.0), (3.0, 6.0, 1.0, 0.0),
                          (2.6, 4.0, 0.25, 0.99)])
def test_c1_build_options_change_no_bit(c1, fast_radius, region_h, bin_scale, min_slow_share):
    """The build options change only which pass certifies a node: the rows,
    weights and triangles equal the default build's (2.6h, 7 candidate slots
    per lane) bit for bit.  With the smallest first-pass radius most interior
    nodes take the exact wave path, and a first region of one h makes it
    double its regions; 2.8h and 3h run the fast pass with 8 and 10 slots;
    bins of h/8 make every tile's region too wide to stage, so every node
    takes the exact path."""
    c, orc, W, info = c1
    w0, pos = _build(c)
    ref = w0.export()
    saved = {k: ops.p2m_get_option(k) for k in ("fast_radius", "region_h", "bin_scale")}
    try:
        ops.p2m_set_option("fast_radius", fast_radius)
        ops.p2m_set_option("region_h", region_h)
        ops.p2m_set_option("bin_scale", bin_scale)
        w1, _ = _build(c)
        d = w1.diag()
        got = w1.export()
    finally:
        for k, v in saved.items():
            ops.p2m_set_option(k, v)
    assert d["failed_nodes"] == 0
    assert d["slow_nodes"] >= min_slow_share * d["interior_nodes"], d
    for g, r, name in zip(got, ref, ("idx", "w", "cnt", "tri")):
        assert torch.equal(g, r), name
    G = ell_to_csr(got[0].numpy(), got[1].numpy(), got[2].numpy(), c.N)
    assert abs(G - W).max() <= 1e-12


@pytest.mark.parametrize("C", [1, 3, 5])
def test_m2p_particles_per_thread_change_no_bit(C):
    """The M2P option m2p_ppt (particles per thread) changes only the launch
    shape: the same bits for 1, 2 and 4 at a particle count that is no
    multiple of any block's share, and the oracle's values at 1e-12."""
    rng = np.random.default_rng(C)
    mesh = wl.MeshSpec(20, 17, 1.0 / 20)
    N = 3 * 1024 + 77
    pos = rng.uniform([0.0, 0.0], [1.0, 17.0 / 20], size=(N, 2))
    mv = rng.normal(size=(mesh.n_nodes, C))
    ref = o_m2p(OMesh.from_spec(mesh), mv, pos)
    saved = ops.p2m_get_option("m2p_ppt")
    outs = []
    try:
        for ppt in (1, 2, 4):
            ops.p2m_set_option("m2p_ppt", ppt)
            outs.append(ops.m2p_interpolate(mesh, _gpu(mv), _gpu(pos)).cpu())
    finally:
        ops.p2m_set_option("m2p_ppt", saved)
    for o in outs[1:]:
        assert torch.equal(o, outs[0])
    assert_close(outs[0].numpy(), ref, 1e-12, "M2P")
