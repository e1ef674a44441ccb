"""The no-allocation form p2m_project_fused_noalloc against the allocating
p2m_project_fused (same build kernels, weights in the library's static
workspace): calls in a row, each on a smaller input than the one before
(the middle one with rows longer than the ELL width), FP64 and mixed; and
the host-side rejections beyond the workspace's limits."""
import numpy as np
import pytest
import torch

import workloads as wl
from paper_1610_05266_amd import ops
from paper_1610_05266_amd._lib import P2MError, P2M_EINVAL
from tests._util import assert_close

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _g(a, dt=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dt)


@pytest.mark.parametrize("dt,tol", [(torch.float64, 1e-12), (torch.float32, 1e-5)])
def test_noalloc_equals_fused_on_two_calls(dt, tol):
    # the middle call holds rows longer than the ELL width (overflow store)
    for c in (wl.small_cloud(32, 2, 0.25, seed=61), wl.hub_cloud(16, ((0.37, 0.41, 40), (0.66, 0.63, 50)), seed=21),
              wl.small_cloud(12, 2, 0.3, seed=62)):
        print(f"[gpu] noalloc {c.name} N={c.N} nodes={c.mesh.n_nodes} {dt}", flush=True)
        pos = _g(c.pos)
        vals = _g(c.vals, dt)
        mdt = torch.float64 if dt == torch.float64 else torch.float32
        out = torch.full((c.mesh.n_nodes, vals.shape[1]), float("nan"), dtype=mdt, device=DEV)
        ops.p2m_project_fused_noalloc(c.mesh, c.h, pos, vals, out)
        ref = ops.p2m_project_fused(c.mesh, c.h, pos, vals)
        torch.cuda.synchronize()
        got, want = out.double().cpu().numpy(), ref.double().cpu().numpy()
        assert np.isfinite(got).all()
        assert_close(got, want, tol, f"noalloc vs fused, {c.name}")
        print(f"  bitwise equal: {bool(np.array_equal(got, want))}", flush=True)


def test_noalloc_rejects_sizes_beyond_the_workspace():
    c = wl.small_cloud(12, 2, 0.3, seed=63)
    pos = _g(c.pos)
    vals = _g(c.vals)
    # a mesh of 26 x 26 node tiles
    big = wl.MeshSpec(200, 200, 1.0 / 200)
    out = torch.empty((big.n_nodes, vals.shape[1]), dtype=torch.float64, device=DEV)
    with pytest.raises(P2MError) as e:
        ops.p2m_project_fused_noalloc(big, c.h, pos, vals, out)
    assert e.value.code == P2M_EINVAL and "static workspace" in str(e.value)
    # too many particles
    n = (1 << 17) + 1
    posn = torch.rand((n, 2), dtype=torch.float64, device=DEV)
    valn = torch.zeros((n, 1), dtype=torch.float64, device=DEV)
    out = torch.empty((c.mesh.n_nodes, 1), dtype=torch.float64, device=DEV)
    with pytest.raises(P2MError) as e:
        ops.p2m_project_fused_noalloc(c.mesh, c.h, posn, valn, out)
    assert e.value.code == P2M_EINVAL
