"""The M2P adjoint gathered per node through a weights handle's binning
(m2p_interpolate_backward_binned) against the oracle's transpose of the M2P
matrix (eq. m2p, linear FE on the fixed mesh): FP64 at 1e-12, FP32 storage
at 1e-6 (FP64 sums, one rounding); particles placed exactly on cell sides,
on nodes and on the walls (the bin of such a particle and the cell it is
located in can differ); a batch of sets; the same bits on every call; the
position gradient equal to m2p_interpolate_backward's bit for bit."""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle import Mesh as OMesh, m2p_grad_pos as o_m2p_grad_pos, m2p_matrix
from paper_1610_05266_amd import ops
from paper_1610_05266_amd._lib import P2M_WEIGHTS_F32
from tests._util import assert_close

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _g(a, dt=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dt)


def _edge_cloud():
    """A jittered lattice with particles moved exactly onto cell sides, mesh
    nodes and the walls."""
    c = wl.small_cloud(8, 2, 0.25, seed=71)
    pos = c.pos.copy()
    H = c.mesh.H
    rng = np.random.default_rng(72)
    pick = rng.choice(c.N, 40, replace=False)
    for t, p in enumerate(pick):
        if t < 15:
            pos[p, 0] = round(pos[p, 0] / H) * H          # on a vertical cell side
        elif t < 25:
            pos[p, 1] = round(pos[p, 1] / H) * H          # on a horizontal side
        elif t < 33:
            pos[p] = np.round(pos[p] / H) * H              # on a node
        else:
            pos[p, t % 2] = 1.0 if t % 3 else 0.0          # on a wall
    # keep particles distinct
    _, keep = np.unique(pos, axis=0, return_index=True)
    pos = pos[np.sort(keep)]
    return c.mesh, c.h, pos


@pytest.mark.parametrize("dt,tol", [(torch.float64, 1e-12), (torch.float32, 1e-6)])
def test_binned_m2p_adjoint_matches_oracle_and_is_deterministic(dt, tol):
    for mesh, h, pos in (_edge_cloud(), (wl.config1().mesh, wl.config1().h, wl.config1().pos)):
        om = OMesh.from_spec(mesh)
        print(f"[gpu] binned M2P adjoint N={len(pos)} nodes={om.n_nodes} {dt}", flush=True)
        rng = np.random.default_rng(73)
        gb = rng.normal(size=(len(pos), 3))
        f = rng.normal(size=(om.n_nodes, 3))
        P = _g(pos)
        w = ops.p2m_build_weights(mesh, h, P, P2M_WEIGHTS_F32)
        gbt, ft = _g(gb, dt), _g(f, dt)
        gpa = torch.zeros_like(P)
        gm1, gpa = ops.m2p_interpolate_backward_binned(w, ft, P, gbt, want_mesh=True, grad_pos=gpa)
        gm2, _ = ops.m2p_interpolate_backward_binned(w, ft, P, gbt, want_mesh=True)
        torch.cuda.synchronize()
        assert torch.equal(gm1, gm2)
        gbr = gbt.double().cpu().numpy()
        ref = m2p_matrix(om, pos).T @ gbr
        assert_close(gm1.double().cpu().numpy(), ref, tol, "binned M2P adjoint")
        gpb = torch.zeros_like(P)
        _, gpb = ops.m2p_interpolate_backward(mesh, ft, P, gbt, want_mesh=False, grad_pos=gpb)
        assert torch.equal(gpa, gpb)
        assert_close(gpa.cpu().numpy(), o_m2p_grad_pos(om, ft.double().cpu().numpy(), pos, gbr),
                     1e-12 if dt == torch.float64 else 1e-6, "grad pos")


def test_binned_m2p_adjoint_of_a_batch():
    sets = [wl.small_cloud(n, 2, 0.25, seed=80 + n) for n in (6, 11, 9)]
    offs = np.concatenate([[0], np.cumsum([c.N for c in sets])])
    b = ops.Batch([c.mesh for c in sets], [c.h for c in sets], offs)
    pos = np.concatenate([c.pos for c in sets])
    P = _g(pos)
    w = ops.p2m_build_weights_batched(b, P, 0)
    rng = np.random.default_rng(81)
    gb = rng.normal(size=(b.N, 2))
    gm, _ = ops.m2p_interpolate_backward_binned(w, None, P, _g(gb), want_mesh=True)
    gm = gm.cpu().numpy()
    for s, c in enumerate(sets):
        om = OMesh.from_spec(c.mesh)
        n0, n1, p0, p1 = b.node_offsets[s], b.node_offsets[s + 1], offs[s], offs[s + 1]
        assert_close(gm[n0:n1], m2p_matrix(om, c.pos).T @ gb[p0:p1], 1e-12, f"set {s}")


def test_binned_m2p_adjoint_in_dense_clusters():
    """Clusters dense enough that some tiles' windows hold more particles
    than the kernel keeps in LDS (those tiles locate per node) beside sparse
    tiles that stage their windows: both kinds against the oracle, and the
    same bits on every call."""
    c = wl.cluster_void_cloud(32, 24000, seed=74)
    om = OMesh.from_spec(c.mesh)
    # particles per tile window (cells of the tile and one around it, plus a
    # bin of margin): the densest exceed the 2048 held in LDS, the sparsest
    # do not
    ij = np.floor(c.pos / om.H).astype(int)
    counts = []
    for ty in range((om.ny + 1 + 7) // 8):
        for tx in range((om.nx + 1 + 7) // 8):
            inx = (ij[:, 0] >= 8 * tx - 2) & (ij[:, 0] <= 8 * tx + 8)
            iny = (ij[:, 1] >= 8 * ty - 2) & (ij[:, 1] <= 8 * ty + 8)
            counts.append(int((inx & iny).sum()))
    assert max(counts) > 2 * 2048 and min(counts) < 2048 // 2
    print(f"[gpu] binned M2P adjoint, clusters N={c.N} window counts {min(counts)}..{max(counts)}", flush=True)
    rng = np.random.default_rng(75)
    gb = rng.normal(size=(c.N, 2))
    P = _g(c.pos)
    w = ops.p2m_build_weights(c.mesh, c.h, P, 0, check_diag=False)
    gm1, _ = ops.m2p_interpolate_backward_binned(w, None, P, _g(gb), want_mesh=True)
    gm2, _ = ops.m2p_interpolate_backward_binned(w, None, P, _g(gb), want_mesh=True)
    assert torch.equal(gm1, gm2)
    assert_close(gm1.cpu().numpy(), m2p_matrix(om, c.pos).T @ gb, 1e-12, "binned M2P adjoint, clusters")
