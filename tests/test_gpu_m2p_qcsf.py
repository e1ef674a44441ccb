"""GPU parity of M2P with the mesh's quadratically consistent functions
(m2p_interpolate_qcsf) against the oracle (oracle/m2p_qcsf.py): FP64 bar
1e-12, FP32 5e-6; every quadratic field reproduced at the particles."""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle import Mesh as OMesh
from oracle.m2p_qcsf import m2p_qcsf_matrix
from paper_1610_05266_amd import ops
from tests._util import assert_close

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _gpu(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dtype)


def _cases():
    c = wl.config1()
    rect = wl.MeshSpec(9, 7, 1.0 / 9, x0=0.2, y0=-0.1)
    rng = np.random.default_rng(3)
    p = np.array([0.2, -0.1]) + rng.random((5000, 2)) * np.array([1.0, 7.0 / 9])
    # particles on the walls and at the corners too
    om = OMesh.from_spec(rect)
    p = np.concatenate([p, om.nodes()[[0, rect.nx, -1, -rect.nx - 1]], om.nodes()[: rect.nx + 1] + [0.3 / 9, 0.0]])
    p[:, 0] = np.minimum(p[:, 0], om.x0 + om.nx * om.H)
    return [(c.mesh, c.pos), (rect, p)]


@pytest.mark.parametrize("case", [0, 1])
def test_m2p_qcsf_matches_the_oracle_and_reproduces_quadratics(case):
    spec, pos_np = _cases()[case]
    print(f"[gpu] m2p qcsf case {case} N={len(pos_np)}", flush=True)
    om = OMesh.from_spec(spec)
    W = m2p_qcsf_matrix(om, pos_np)
    nodes = om.nodes()
    rng = np.random.default_rng(7)
    mv = rng.standard_normal((om.n_nodes, 3))
    q = ops.MeshQCSF(spec, DEV)
    pos = _gpu(pos_np)
    got = q.interpolate(_gpu(mv), pos).cpu().numpy()
    assert_close(got, W @ mv, 1e-12, "M2P QCSF FP64")
    got32 = q.interpolate(_gpu(mv, torch.float32), pos).cpu().numpy()
    assert_close(got32, W @ mv, 5e-6, "M2P QCSF FP32")
    quad = np.stack([np.ones(len(nodes)), nodes[:, 0], nodes[:, 1], nodes[:, 0] ** 2, nodes[:, 0] * nodes[:, 1],
                     nodes[:, 1] ** 2], 1)
    want = np.stack([np.ones(len(pos_np)), pos_np[:, 0], pos_np[:, 1], pos_np[:, 0] ** 2,
                     pos_np[:, 0] * pos_np[:, 1], pos_np[:, 1] ** 2], 1)
    got_q = q.interpolate(_gpu(quad), pos).cpu().numpy()
    assert np.abs(got_q - want).max() <= 1e-12


def test_periodic_mesh_qcsf_matches_the_oracle():
    """The periodic box: every particle, next to the sides too, against the
    oracle's tiled-mesh functions (FP64 1e-12, FP32 5e-6)."""
    import workloads as wl
    from oracle import Mesh as OMesh
    from oracle.m2p_qcsf import m2p_qcsf_periodic
    c = wl.periodic_tg_cloud(16, 2, 0.3, 11)
    om = OMesh.from_spec(c.mesh)
    nodes = om.nodes()
    f = np.stack([wl.tg_u(nodes[:, 0], nodes[:, 1]), wl.tg_p(nodes[:, 0], nodes[:, 1])], 1)
    # the repeated last column and row hold the first's values
    n1 = om.nx + 1
    g = f.reshape(om.ny + 1, n1, -1)
    g[:, -1] = g[:, 0]
    g[-1] = g[0]
    f = g.reshape(-1, f.shape[1])
    want = m2p_qcsf_periodic(om, f, c.pos)
    print("[gpu] periodic mesh qcsf", flush=True)
    q = ops.MeshQCSF(c.mesh, DEV, periodic=True)
    pos = torch.from_numpy(c.pos).to(DEV)
    got = q.interpolate(torch.from_numpy(f).to(DEV), pos).cpu().numpy()
    assert_close(got, want, 1e-12, "periodic QCSF M2P FP64")
    got32 = q.interpolate(torch.from_numpy(f).to(DEV, torch.float32), pos).cpu().numpy()
    assert_close(got32, want, 5e-6, "periodic QCSF M2P FP32")
    with pytest.raises(ops.P2MError):
        ops.MeshQCSF(wl.MeshSpec(3, 3, 2.0 / 3, -1.0, -1.0), DEV, periodic=True)
