"""GPU parity of the linear FE particle functions (P2M_LINEAR) against the
oracle: at an interior node the row is phi_mu alone, the barycentric
coordinates of the node in its particle Delaunay triangle (App. B, eqs. C0,
C1); closure nodes keep their quadratic-moment weights.  FP64 bar 1e-12."""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle import Mesh as OMesh, P2MOracle
from oracle.qcsf import linear_fe_matrix
from paper_1610_05266_amd import ops
from tests._util import assert_close, ell_to_csr

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, torch.float64)


@pytest.fixture(scope="module")
def c1_linear():
    c = wl.config1()
    mesh = OMesh.from_spec(c.mesh)
    W, info = P2MOracle(c.pos, mesh, c.h).matrix()
    L, ok = linear_fe_matrix(c.pos, mesh)
    print(f"[gpu] linear build {c.name} N={c.N}", flush=True)
    pos = _gpu(c.pos)
    wq = ops.p2m_build_weights(c.mesh, c.h, pos, 0)
    wl_ = ops.p2m_build_weights(c.mesh, c.h, pos, ops.P2M_LINEAR)
    return c, mesh, W, info, L, ok, wq, wl_, pos


def test_c1_linear_rows_match_the_linear_fe_oracle(c1_linear):
    c, mesh, W, info, L, ok, wq, wl_, pos = c1_linear
    d = wl_.diag()
    assert d["failed_nodes"] == 0 and d["rank_deficient"] == 0
    closure = info["closure"]
    assert np.array_equal(ok, ~closure)
    idx, wt, cnt, tri = wl_.export()
    G = ell_to_csr(idx.numpy(), wt.numpy(), cnt.numpy(), c.N)
    # interior: three entries, the oracle's barycentric coordinates
    assert np.all(cnt.numpy()[ok] == 3)
    assert abs(G[ok] - L[ok]).max() <= 1e-12
    # closure nodes: the quadratic closure rows
    assert abs(G[closure] - W[closure]).max() <= 1e-12
    # the same triangles as the quadratic build's
    tq = wq.export()[3].numpy()
    assert np.array_equal(np.sort(tri.numpy()[ok], 1), np.sort(tq[ok], 1))


def test_c1_linear_p2m_reproduces_linear_fields_only(c1_linear):
    c, mesh, W, info, L, ok, wq, wl_, pos = c1_linear
    nodes = mesh.nodes()
    lin = _gpu(np.stack([np.ones(c.N), c.pos[:, 0], c.pos[:, 1]], 1))
    got = ops.p2m_project(wl_, lin).cpu().numpy()
    want = np.stack([np.ones(len(nodes)), nodes[:, 0], nodes[:, 1]], 1)
    assert np.abs(got - want).max() <= 1e-12
    # eq. C2 does not hold: x^2 is off at interior nodes by about h^2
    x2 = ops.p2m_project(wl_, _gpu(c.pos[:, :1] ** 2)).cpu().numpy()[:, 0]
    assert np.abs(x2[ok] - nodes[ok, 0] ** 2).max() > 1e-6
    assert_close(ops.p2m_project(wl_, _gpu(c.vals)).cpu().numpy()[ok], (L @ c.vals)[ok], 1e-12, "linear P2M")


def test_linear_weights_refuse_position_gradients(c1_linear):
    c, mesh, W, info, L, ok, wq, wl_, pos = c1_linear
    gw = torch.zeros((ops.MAX_SUPPORT, mesh.n_nodes), dtype=torch.float64, device=DEV)
    gp = torch.zeros((c.N, 2), dtype=torch.float64, device=DEV)
    with pytest.raises(ops.P2MError, match="P2M_LINEAR"):
        ops.p2m_build_weights_backward(wl_, pos, gw, gp)
