"""GPU parity of the batched driver: many independent particle sets, each
with its own mesh and spacing, built, projected and interpolated by one
launch sequence.  Each set must give what the oracle gives for it alone
(eqs. p2m, m2p, App. B), and exactly what a single-set build gives."""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle import Mesh as OMesh, P2MOracle, m2p as o_m2p, m2p_grad_pos as o_m2p_grad_pos
from oracle.adjoint import p2m_grad_pos as o_p2m_grad_pos
from paper_1610_05266_amd import ops
from paper_1610_05266_amd._lib import P2M_WEIGHTS_F32
from tests._util import assert_close, ell_to_csr

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _g(a, dt=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dt)


def _offset_cloud(seed):
    rng = np.random.default_rng(seed)
    mesh = wl.MeshSpec(9, 6, 0.07, -0.3, 2.1)
    N = 700
    pos = np.stack([rng.uniform(-0.3, -0.3 + 9 * 0.07, N), rng.uniform(2.1, 2.1 + 6 * 0.07, N)], 1)
    h = float(np.sqrt(9 * 6 * 0.07 ** 2 / N))
    return mesh, h, pos


@pytest.fixture(scope="module")
def mixed_batch():
    """Five sets: two lattice ratios, different sizes, an offset rectangle
    with uniform random particles, and a three-cell set."""
    sets = []
    for n, ratio, jit, seed in ((10, 2, 0.25, 1), (7, 4, 0.3, 2), (16, 2, 0.25, 3), (3, 2, 0.25, 4)):
        c = wl.small_cloud(n, ratio, jit, seed)
        sets.append((c.mesh, c.h, c.pos))
    sets.insert(2, _offset_cloud(5))
    offs = np.cumsum([0] + [s[2].shape[0] for s in sets])
    b = ops.Batch([s[0] for s in sets], [s[1] for s in sets], offs)
    pos = np.concatenate([s[2] for s in sets])
    rng = np.random.default_rng(9)
    vals = rng.normal(size=(pos.shape[0], 3))
    oracles = [P2MOracle(p, OMesh.from_spec(m), h) for m, h, p in sets]
    return sets, b, pos, vals, oracles


def test_batch_shape(mixed_batch):
    sets, b, pos, _, _ = mixed_batch
    assert b.S == len(sets) and b.N == pos.shape[0]
    sizes = [(m.nx + 1) * (m.ny + 1) for m, _, _ in sets]
    assert b.node_offsets == list(np.cumsum([0] + sizes))
    assert b.n_nodes == sum(sizes)


def test_batched_weights_match_oracle_per_set(mixed_batch):
    sets, b, pos, vals, oracles = mixed_batch
    w = ops.p2m_build_weights_batched(b, _g(pos))
    d = w.diag()
    assert d["status"] == 0 and d["failed_nodes"] == 0
    idx, wts, cnt, tri = w.export()
    idx, wts, cnt, tri = idx.numpy(), wts.numpy(), cnt.numpy(), tri.numpy()
    mesh_vals = ops.p2m_project(w, _g(vals)).cpu().numpy()
    for s, (orc, (m, h, p)) in enumerate(zip(oracles, sets)):
        n0, n1 = b.node_offsets[s], b.node_offsets[s + 1]
        p0, p1 = b.offsets[s], b.offsets[s + 1]
        W, info = orc.matrix()
        # batch-global particle ids of the set's rows, shifted to set-local
        got = ell_to_csr(idx[:, n0:n1] - np.where(idx[:, n0:n1] >= 0, p0, 0), wts[:, n0:n1], cnt[n0:n1],
                         p.shape[0])
        assert np.all((idx[:, n0:n1] < 0) | ((idx[:, n0:n1] >= p0) & (idx[:, n0:n1] < p1)))
        assert_close(got.toarray(), W.toarray(), 1e-12, f"set {s} weights")
        assert_close(mesh_vals[n0:n1], W @ vals[p0:p1], 1e-12, f"set {s} P2M")
        inter = ~info["closure"]
        t = tri[n0:n1][inter] - p0
        assert np.array_equal(np.sort(t, 1), np.sort(info["triangle"][inter], 1)), f"set {s} triangles"


def test_batched_equals_single_set_builds_bitwise(mixed_batch):
    sets, b, pos, vals, _ = mixed_batch
    wb = ops.p2m_build_weights_batched(b, _g(pos), P2M_WEIGHTS_F32)
    ib, xb, cb, tb = (t.numpy() for t in wb.export())
    mb = ops.p2m_project(wb, _g(vals, torch.float32)).cpu().numpy()
    for s, (m, h, p) in enumerate(sets):
        n0, n1 = b.node_offsets[s], b.node_offsets[s + 1]
        p0, p1 = b.offsets[s], b.offsets[s + 1]
        ws = ops.p2m_build_weights(m, h, _g(p), P2M_WEIGHTS_F32)
        i1, x1, c1, t1 = (t.numpy() for t in ws.export())
        assert np.array_equal(c1, cb[n0:n1])
        assert np.array_equal(np.where(i1 >= 0, i1 + p0, -1), ib[:, n0:n1])
        assert np.array_equal(x1, xb[:, n0:n1])
        assert np.array_equal(np.where(t1 >= 0, t1 + p0, -1), tb[n0:n1])
        ms = ops.p2m_project(ws, _g(vals[p0:p1], torch.float32)).cpu().numpy()
        assert np.array_equal(ms, mb[n0:n1])


def test_batched_m2p_and_adjoint(mixed_batch):
    sets, b, pos, _, _ = mixed_batch
    rng = np.random.default_rng(11)
    f = rng.normal(size=(b.n_nodes, 2))
    g = rng.normal(size=(b.N, 2))
    out = ops.m2p_interpolate_batched(b, _g(f), _g(pos)).cpu().numpy()
    gp = torch.zeros((b.N, 2), dtype=torch.float64, device=DEV)
    gm, gp = ops.m2p_interpolate_backward_batched(b, _g(f), _g(pos), _g(g), want_mesh=True, grad_pos=gp)
    gm, gp = gm.cpu().numpy(), gp.cpu().numpy()
    for s, (m, h, p) in enumerate(sets):
        n0, n1 = b.node_offsets[s], b.node_offsets[s + 1]
        p0, p1 = b.offsets[s], b.offsets[s + 1]
        om = OMesh.from_spec(m)
        assert_close(out[p0:p1], o_m2p(om, f[n0:n1], p), 1e-13, f"set {s} M2P")
        assert_close(gp[p0:p1], o_m2p_grad_pos(om, f[n0:n1], p, g[p0:p1]), 1e-12, f"set {s} M2P grad pos")
        single, _ = ops.m2p_interpolate_backward(m, None, _g(p), _g(g[p0:p1]), want_mesh=True)
        assert_close(gm[n0:n1], single.cpu().numpy(), 1e-13, f"set {s} M2P^T")


def test_batched_build_backward_matches_oracle(mixed_batch):
    sets, b, pos, vals, oracles = mixed_batch
    rng = np.random.default_rng(12)
    gmesh = rng.normal(size=(b.n_nodes, 3))
    w = ops.p2m_build_weights_batched(b, _g(pos))
    gv, gw = ops.p2m_project_backward(w, _g(gmesh), _g(vals), want_vals=True, want_w=True)
    gp = ops.p2m_build_weights_backward(w, _g(pos), gw).cpu().numpy()
    gv = gv.cpu().numpy()
    for s, orc in enumerate(oracles):
        n0, n1 = b.node_offsets[s], b.node_offsets[s + 1]
        p0, p1 = b.offsets[s], b.offsets[s + 1]
        W, _ = orc.matrix()
        assert_close(gv[p0:p1], W.T @ gmesh[n0:n1], 1e-12, f"set {s} P2M^T")
        ref = o_p2m_grad_pos(orc, vals[p0:p1], gmesh[n0:n1])
        assert_close(gp[p0:p1], ref, 1e-10, f"set {s} grad pos")


def test_batch_handle_rebuild_with_other_batch(mixed_batch):
    """A weights handle built from one batch, then a single set, then the
    batch again gives the same bits every time (device set table refresh)."""
    sets, b, pos, vals, _ = mixed_batch
    w = ops.p2m_build_weights_batched(b, _g(pos))
    first = ops.p2m_project(w, _g(vals)).cpu().numpy()
    m, h, p = sets[1]
    ops.p2m_build_weights(m, h, _g(p), weights=w)
    ops.p2m_build_weights_batched(b, _g(pos), weights=w)
    again = ops.p2m_project(w, _g(vals)).cpu().numpy()
    assert np.array_equal(first, again)


@pytest.fixture(scope="module")
def c3():
    sets = wl.config3()
    offs = np.cumsum([0] + [c.N for c in sets])
    b = ops.Batch([c.mesh for c in sets], [c.h for c in sets], offs)
    pos = np.concatenate([c.pos for c in sets])
    vals = np.concatenate([c.vals for c in sets])
    return sets, b, pos, vals


def test_c3_full_batch_quadratic_exact_and_sampled_oracle(c3):
    """64 sets, ~10 M particles, one launch sequence: every node of every set
    reproduces a quadratic (eqs. C0-C2, closure included), and sampled nodes
    of eight sets match the oracle."""
    sets, b, pos, vals = c3
    print(f"C3: S={b.S} N={b.N} nodes={b.n_nodes}", flush=True)
    P = _g(pos)
    w = ops.p2m_build_weights_batched(b, P, P2M_WEIGHTS_F32)
    d = w.diag()
    assert d["status"] == 0 and d["failed_nodes"] == 0 and d["rank_deficient"] == 0
    assert d["interior_nodes"] + d["closure_nodes"] == b.n_nodes
    q = wl.quad_q(pos[:, 0], pos[:, 1])[:, None]
    mq = ops.p2m_project(w, _g(q)).cpu().numpy()[:, 0]
    ref = np.concatenate([wl.quad_q(*OMesh.from_spec(c.mesh).nodes().T) for c in sets])
    assert np.abs(mq - ref).max() <= 1e-10 * np.abs(ref).max()
    m64 = ops.p2m_project(w, _g(vals)).cpu().numpy()
    m32 = ops.p2m_project(w, _g(vals, torch.float32)).cpu().numpy()
    assert_close(m32, m64, 1e-5, "C3 mixed vs FP64")
    rng = np.random.default_rng(3)
    for s in rng.choice(b.S, 8, replace=False):
        c = sets[s]
        n0, p0, p1 = b.node_offsets[s], b.offsets[s], b.offsets[s + 1]
        om = OMesh.from_spec(c.mesh)
        sample = np.unique(np.concatenate([rng.choice(om.n_nodes, 24, replace=False), [0, om.n_nodes - 1]]))
        Ws, _ = P2MOracle(c.pos, om, c.h, mode="local").matrix(sample)
        assert_close(m64[n0 + sample], Ws @ vals[p0:p1], 1e-12, f"C3 set {s} sampled nodes")
    # M2P of the P2M result, every particle, against the oracle formula per set
    out = ops.m2p_interpolate_batched(b, _g(m64), P).cpu().numpy()
    for s in rng.choice(b.S, 4, replace=False):
        c = sets[s]
        n0, n1, p0, p1 = b.node_offsets[s], b.node_offsets[s + 1], b.offsets[s], b.offsets[s + 1]
        assert_close(out[p0:p1], o_m2p(OMesh.from_spec(c.mesh), m64[n0:n1], c.pos), 1e-13, f"C3 set {s} M2P")


@pytest.mark.parametrize("bin_scale", [0.75, 0.5])
def test_c3_finer_binning_grids_change_no_bit(c3, bin_scale):
    """Finer binning grids over the 64-set batch (thousands of super-bins:
    the partition pass's LDS plan and the local pass's staging at their
    limits) give the default grid's projection bit for bit."""
    sets, b, pos, vals = c3
    P = _g(pos)
    v = _g(vals, torch.float32)
    ref = ops.p2m_project(ops.p2m_build_weights_batched(b, P, P2M_WEIGHTS_F32), v)
    saved = ops.p2m_get_option("bin_scale")
    try:
        ops.p2m_set_option("bin_scale", bin_scale)
        w = ops.p2m_build_weights_batched(b, P, P2M_WEIGHTS_F32)
        print(f"C3 bin_scale={bin_scale}: {w.diag()['slow_nodes']} slow nodes", flush=True)
        got = ops.p2m_project(w, v)
    finally:
        ops.p2m_set_option("bin_scale", saved)
    assert torch.equal(got, ref)
