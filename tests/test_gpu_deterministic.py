"""The deterministic adjoints of P2M (handles built with P2M_DETERMINISTIC).

The entries of the weights are indexed by particle at build time, and the
transpose of eq. (p2m) and the position adjoint of the App. B weights are
summed per particle in a fixed order instead of by atomics.  Checked:
  * P2M^t against the oracle's W^t g (1e-12 FP64, 1e-5 FP32), bit for bit
    the same on repeated calls and on a rebuilt handle;
  * the position gradient against the oracle's complex-step derivatives
    (1e-10) and against the atomic form of the same call (1e-12 of the
    largest component), bit for bit the same on repeated calls;
  * rows longer than the ELL width and the periodic box;
  * the 1,048,576-particle workload: both gradients bit-stable and equal to
    the atomic forms within rounding.
"""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle import Mesh as OMesh, P2MOracle
from oracle.adjoint import p2m_grad_pos as o_p2m_grad_pos
from paper_1610_05266_amd import ops
from paper_1610_05266_amd._lib import P2M_DETERMINISTIC, P2M_PERIODIC, P2M_WEIGHTS_F32
from tests._util import assert_close

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
DET = P2M_DETERMINISTIC | P2M_WEIGHTS_F32


def _g(a, dt=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dt)


def _grads(w, pos, gmesh, vals):
    gv, gw = ops.p2m_project_backward(w, gmesh, vals, want_vals=True, want_w=True)
    gp = ops.p2m_build_weights_backward(w, pos, gw)
    return gv, gp


@pytest.mark.parametrize("cloud", ["small", "hub"])
def test_deterministic_adjoints_match_oracle_and_repeat_bitwise(cloud):
    if cloud == "small":
        c = wl.small_cloud(12, 2, 0.25, seed=41, channels=("u", "v", "q"))
    else:
        c = wl.hub_cloud(16, ((0.37, 0.41, 40), (0.66, 0.63, 50)), seed=21)
    om = OMesh.from_spec(c.mesh)
    print(f"[gpu] deterministic adjoints {c.name} N={c.N}", flush=True)
    orc = P2MOracle(c.pos, om, c.h)
    W, _ = orc.matrix()
    rng = np.random.default_rng(5)
    gmesh = rng.normal(size=(om.n_nodes, 3))
    pos = _g(c.pos)
    w = ops.p2m_build_weights(c.mesh, c.h, pos, DET)
    gv, gp = _grads(w, pos, _g(gmesh), _g(c.vals))
    assert_close(gv.cpu().numpy(), W.T @ gmesh, 1e-12, "P2M^t gathered")
    assert w.diag()["bwd_rank_deficient"] == 0
    assert_close(gp.cpu().numpy(), o_p2m_grad_pos(orc, c.vals, gmesh), 1e-10, "grad pos gathered")
    # FP32 values and weights
    gv32, _ = ops.p2m_project_backward(w, _g(gmesh, torch.float32), _g(c.vals, torch.float32), want_vals=True)
    assert_close(gv32.cpu().numpy(), W.T @ gmesh, 1e-5, "P2M^t gathered FP32")
    # the same bits on every call, and on a rebuilt handle
    for _ in range(2):
        gv2, gp2 = _grads(w, pos, _g(gmesh), _g(c.vals))
        assert torch.equal(gv2, gv) and torch.equal(gp2, gp)
    w2 = ops.p2m_build_weights(c.mesh, c.h, pos, DET)
    gv3, gp3 = _grads(w2, pos, _g(gmesh), _g(c.vals))
    assert torch.equal(gv3, gv) and torch.equal(gp3, gp)
    # the atomic form of the same calls agrees to rounding
    wa = ops.p2m_build_weights(c.mesh, c.h, pos, P2M_WEIGHTS_F32)
    gva, gpa = _grads(wa, pos, _g(gmesh), _g(c.vals))
    assert_close(gva.cpu().numpy(), gv.cpu().numpy(), 1e-13, "gathered vs atomic P2M^t")
    assert_close(gpa.cpu().numpy(), gp.cpu().numpy(), 1e-12, "gathered vs atomic grad pos")


def test_deterministic_adjoints_in_the_periodic_box():
    c = wl.periodic_tg_cloud(16, 2, 0.25, seed=12)
    print(f"[gpu] deterministic adjoints periodic N={c.N}", flush=True)
    rng = np.random.default_rng(6)
    gmesh = _g(rng.normal(size=(c.mesh.n_nodes, 3)))
    pos = _g(c.pos)
    w = ops.p2m_build_weights(c.mesh, c.h, pos, P2M_PERIODIC | DET)
    wa = ops.p2m_build_weights(c.mesh, c.h, pos, P2M_PERIODIC | P2M_WEIGHTS_F32)
    gv, gp = _grads(w, pos, gmesh, _g(c.vals))
    gva, gpa = _grads(wa, pos, gmesh, _g(c.vals))
    assert_close(gv.cpu().numpy(), gva.cpu().numpy(), 1e-13, "periodic gathered vs atomic P2M^t")
    assert_close(gp.cpu().numpy(), gpa.cpu().numpy(), 1e-12, "periodic gathered vs atomic grad pos")
    gv2, gp2 = _grads(w, pos, gmesh, _g(c.vals))
    assert torch.equal(gv2, gv) and torch.equal(gp2, gp)


def test_deterministic_adjoints_at_a_million_particles():
    c = wl.config2()
    print(f"[gpu] deterministic adjoints C2 N={c.N}", flush=True)
    rng = np.random.default_rng(7)
    gmesh = _g(rng.normal(size=(c.mesh.n_nodes, 3)))
    pos = _g(c.pos)
    vals = _g(c.vals)
    w = ops.p2m_build_weights(c.mesh, c.h, pos, DET)
    gv, gp = _grads(w, pos, gmesh, vals)
    gv2, gp2 = _grads(w, pos, gmesh, vals)
    assert torch.equal(gv2, gv) and torch.equal(gp2, gp)
    wa = ops.p2m_build_weights(c.mesh, c.h, pos, P2M_WEIGHTS_F32)
    gva, gpa = _grads(wa, pos, gmesh, vals)
    assert_close(gva.cpu().numpy(), gv.cpu().numpy(), 1e-13, "C2 gathered vs atomic P2M^t")
    assert_close(gpa.cpu().numpy(), gp.cpu().numpy(), 1e-12, "C2 gathered vs atomic grad pos")
    # every particle's entries are indexed: P2M^t of a constant field is the
    # column sum of the weights, which the rows fix (sum_mu of each row is 1)
    ones = torch.ones((c.mesh.n_nodes, 1), dtype=torch.float64, device=DEV)
    g1, _ = ops.p2m_project_backward(w, ones, want_vals=True)
    assert abs(float(g1.sum()) - c.mesh.n_nodes) <= 1e-9 * c.mesh.n_nodes
