"""GPU parity for supports longer than the ELL width (32 entries).

A node's support is the union of the Delaunay rings of its triangle's three
vertices (App. B), so a particle of high Delaunay degree gives long rows.
``workloads.hub_cloud`` rings a particle with 40 or 50 others (and a
particle with 56 in a second cloud); every mesh node inside such a ring has
a support of 43..60 particles.  The first 32 entries of such a row stay in
the ELL arrays, the rest go to an overflow row of the handle, and the row is
solved by the wave solver (one support entry per lane).  Checked against the
oracle, which has no support cap:
  * the supports (same particle sets) and the weights element by element;
  * P2M in FP64 and FP32, P2M^t and grad_w (p2m_project_backward);
  * the position adjoint through those rows (oracle complex-step
    derivatives);
  * a ring of 70 particles (supports above 63): exactly the rows whose
    support exceeds the cap fail, and are reported; the others are whole.
"""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle import Mesh as OMesh, P2MOracle
from oracle.adjoint import p2m_grad_pos as o_p2m_grad_pos
from paper_1610_05266_amd import ops
from tests._util import assert_close, ell_to_csr

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
EPS = np.finfo(np.float64).eps
ELL = 32

HUBS = {
    "hub40_50": ((0.37, 0.41, 40), (0.66, 0.63, 50)),
    "hub56": ((0.37, 0.41, 56),),
}


def _g(a, dt=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dt)


def _row_cond(info, t):
    if info["closure"][t]:
        s, r = info["closure_sigma"][t], info["closure_rank"][t]
        return s[0] / s[r - 1]
    return max(s[0] / s[r - 1] for s, r in zip(info["edge_sigma"][t], info["edge_rank"][t]))


@pytest.mark.parametrize("name", sorted(HUBS))
def test_long_rows_match_oracle(name):
    c = wl.hub_cloud(16, HUBS[name], seed=21)
    om = OMesh.from_spec(c.mesh)
    print(f"[gpu] long rows {name} N={c.N}", flush=True)
    orc = P2MOracle(c.pos, om, c.h)
    cols, _, info = orc.node_weights()
    W, _ = orc.matrix()
    sizes = np.array([len(u) for u in cols])
    n_long = int((sizes > ELL).sum())
    assert n_long > 0
    w = ops.p2m_build_weights(c.mesh, c.h, _g(c.pos), ops.P2M_WEIGHTS_F32)
    d = w.diag()
    assert d["failed_nodes"] == 0 and d["cap_overflow"] == 0
    assert d["long_rows"] == n_long
    assert d["support_max"] == sizes.max()
    idx, wt, cnt, _ = w.export()
    cnt = cnt.numpy()
    idx = idx.numpy()
    assert (cnt == sizes).all()
    for t in np.flatnonzero(sizes > ELL):
        assert sorted(idx[: cnt[t], t].tolist()) == sorted(cols[t].tolist()), t
    G = ell_to_csr(idx, wt.numpy(), cnt, c.N)
    for t in range(om.n_nodes):
        ref = W[t].toarray().ravel()
        got = G[t].toarray().ravel()
        tol = max(1e-12, 10.0 * EPS * _row_cond(info, t))
        assert np.abs(got - ref).max() <= tol * np.abs(ref).max(), (t, sizes[t])
    # P2M, FP64 and FP32 weights
    ref = W @ c.vals
    assert_close(ops.p2m_project(w, _g(c.vals)).cpu().numpy(), ref, 1e-12, "P2M FP64, long rows")
    got32 = ops.p2m_project(w, _g(c.vals, torch.float32)).cpu().numpy()
    assert_close(got32, ref, 1e-5, "P2M FP32, long rows")
    # P2M^t and grad_w
    rng = np.random.default_rng(22)
    gmesh = rng.normal(size=(om.n_nodes, 3))
    gv, gw = ops.p2m_project_backward(w, _g(gmesh), _g(c.vals), want_vals=True, want_w=True)
    assert_close(gv.cpu().numpy(), W.T @ gmesh, 1e-12, "P2M^t, long rows")
    gw = gw.cpu().numpy()
    gvals = gmesh @ c.vals.T  # [n_nodes, N]: d L / d W[i, j]
    for t in np.flatnonzero(sizes > ELL):
        want = gvals[t, idx[: cnt[t], t]]
        assert np.abs(gw[: cnt[t], t] - want).max() <= 1e-12 * np.abs(want).max(), t
        assert (gw[cnt[t]:, t] == 0.0).all()


def test_long_rows_position_adjoint():
    c = wl.hub_cloud(16, HUBS["hub40_50"], seed=21)
    om = OMesh.from_spec(c.mesh)
    print(f"[gpu] long rows adjoint N={c.N}", flush=True)
    orc = P2MOracle(c.pos, om, c.h)
    pos = _g(c.pos)
    w = ops.p2m_build_weights(c.mesh, c.h, pos)
    assert w.diag()["long_rows"] > 0
    rng = np.random.default_rng(23)
    gmesh = rng.normal(size=(om.n_nodes, 3))
    _, gw = ops.p2m_project_backward(w, _g(gmesh), _g(c.vals), want_vals=False, want_w=True)
    gp = ops.p2m_build_weights_backward(w, pos, gw).cpu().numpy()
    assert w.diag()["bwd_rank_deficient"] == 0
    assert_close(gp, o_p2m_grad_pos(orc, c.vals, gmesh), 1e-10, "P2M grad pos, long rows")


def test_support_above_cap_is_reported():
    c = wl.hub_cloud(16, ((0.37, 0.41, 70),), seed=24)
    om = OMesh.from_spec(c.mesh)
    print(f"[gpu] support above the cap N={c.N}", flush=True)
    orc = P2MOracle(c.pos, om, c.h)
    cols, _, info = orc.node_weights()
    W, _ = orc.matrix()
    sizes = np.array([len(u) for u in cols])
    over = sizes > ops.MAX_SUPPORT
    assert over.any()
    w = ops.p2m_build_weights(c.mesh, c.h, _g(c.pos), check_diag=False)
    d = w.diag(check_status=False)
    assert d["cap_overflow"] > 0
    # exactly the rows whose support exceeds the cap fail; the rest are whole
    assert d["failed_nodes"] == int(over.sum())
    idx, wt, cnt, _ = w.export()
    cnt = cnt.numpy()
    assert ((cnt == 0) == over).all()
    G = ell_to_csr(idx.numpy(), wt.numpy(), cnt, c.N)
    for t in np.flatnonzero(~over):
        ref = W[t].toarray().ravel()
        got = G[t].toarray().ravel()
        tol = max(1e-12, 10.0 * EPS * _row_cond(info, t))
        assert np.abs(got - ref).max() <= tol * np.abs(ref).max(), (t, sizes[t])
    with pytest.raises(ops.P2MError):
        ops.p2m_build_weights(c.mesh, c.h, _g(c.pos))
