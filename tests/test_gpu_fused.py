"""The fused recompute form p2m_project_fused: the weights pass adds every
row of the fast path into its node's weighted sum (eq. p2m) as it weighs it
and stores no weights for it; rows of the exact path and of the
rank-revealing solver keep stored weights and are projected afterwards.  The
summation order is the stored-weights projection's, so the result must equal
p2m_build_weights + p2m_project bit for bit:
  * every value type (FP64, FP32, BF16 values) and channel counts 1..5 (five
    takes the unfused build + project);
  * clouds whose rows take the exact path, the rank-revealing solver, and
    rows longer than the ELL width;
  * the 1,048,576-particle workload.
The fused workspace then holds no weights: project and export on it are
refused."""
import numpy as np
import pytest
import torch

import workloads as wl
from paper_1610_05266_amd import ops
from paper_1610_05266_amd._lib import P2M_WEIGHTS_F32

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _g(a, dt=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dt)


def _stored(c, pos, vals):
    flags = 0 if vals.dtype == torch.float64 else P2M_WEIGHTS_F32
    w = ops.p2m_build_weights(c.mesh, c.h, pos, flags, check_diag=False)
    return ops.p2m_project(w, vals), w.diag(check_status=False)


@pytest.mark.parametrize("dt", [torch.float64, torch.float32, torch.bfloat16])
@pytest.mark.parametrize("C", [1, 2, 3, 4, 5])
def test_fused_equals_stored_bitwise(dt, C):
    c = wl.small_cloud(24, 2, 0.3, seed=71)
    print(f"[gpu] fused vs stored {dt} C={C}", flush=True)
    rng = np.random.default_rng(C)
    pos = _g(c.pos)
    vals = _g(rng.normal(size=(c.N, C)), dt)
    ref, _ = _stored(c, pos, vals)
    out = ops.p2m_project_fused(c.mesh, c.h, pos, vals, check_diag=True)
    assert torch.equal(out, ref)


@pytest.mark.parametrize("cloud", ["cluster", "conic", "hub"])
def test_fused_equals_stored_on_exact_and_rank_revealing_rows(cloud):
    if cloud == "cluster":
        c = wl.cluster_void_cloud(32, 6000, seed=72)
    elif cloud == "conic":
        c = wl.conic_cloud(8, 24, 1e-8, seed=3)
    else:
        c = wl.hub_cloud(16, ((0.37, 0.41, 40), (0.66, 0.63, 50)), seed=21)
    print(f"[gpu] fused vs stored {c.name} N={c.N}", flush=True)
    pos = _g(c.pos)
    for dt in (torch.float64, torch.float32):
        vals = _g(c.vals, dt)
        ref, d = _stored(c, pos, vals)
        out = ops.p2m_project_fused(c.mesh, c.h, pos, vals)
        assert torch.equal(out, ref), dt
        fd = ops.fused_diag()
        assert fd["slow_nodes"] == d["slow_nodes"] and fd["svd_systems"] == d["svd_systems"]
    # the workload exercises the listed rows
    assert d["slow_nodes"] > 0 or d["svd_systems"] > 0 or d["long_rows"] > 0


def test_fused_equals_stored_at_a_million_particles():
    c = wl.config2()
    print(f"[gpu] fused vs stored C2 N={c.N}", flush=True)
    pos = _g(c.pos)
    for dt in (torch.float64, torch.float32):
        vals = _g(c.vals, dt)
        ref, d = _stored(c, pos, vals)
        assert d["slow_nodes"] > 0
        out = ops.p2m_project_fused(c.mesh, c.h, pos, vals, check_diag=True)
        assert torch.equal(out, ref), dt


def test_fused_workspace_keeps_no_weights():
    import ctypes

    from paper_1610_05266_amd._lib import load
    c = wl.small_cloud(12, 2, 0.25, seed=73)
    pos = _g(c.pos)
    lib = load()
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    cnt = torch.empty((c.mesh.n_nodes,), dtype=torch.int32, device=DEV)
    ops.p2m_project_fused(c.mesh, c.h, pos, _g(c.vals))
    h = ctypes.c_void_p(lib.p2m_fused_handle())
    assert h.value
    rc = lib.p2m_weights_export(h, None, None, ctypes.c_void_p(cnt.data_ptr()), None, st)
    assert rc != 0 and b"keeps no weights" in lib.p2m_last_error()
    # the recompute backward rebuilds the workspace with stored weights
    g = _g(np.random.default_rng(4).normal(size=(c.mesh.n_nodes, 3)))
    gv, _ = ops.p2m_backward_fused(c.mesh, c.h, pos, _g(c.vals), g, want_vals=True)
    assert torch.isfinite(gv).all()
    assert lib.p2m_weights_export(h, None, None, ctypes.c_void_p(cnt.data_ptr()), None, st) == 0
    torch.cuda.synchronize()
    assert int(cnt.min()) > 0


def test_handle_regrowth_keeps_the_fp32_weights_sized():
    """A handle built with FP32 weights, rebuilt larger without them and then
    larger again with them must hold FP32 weights for every slot (their
    capacity is tracked on its own): the projection equals a fresh
    handle's."""
    small = wl.small_cloud(12, 2, 0.25, seed=74)
    big = wl.small_cloud(40, 2, 0.25, seed=75)
    pos_s, pos_b = _g(small.pos), _g(big.pos)
    v32 = _g(big.vals, torch.float32)
    w = ops.p2m_build_weights(small.mesh, small.h, pos_s, P2M_WEIGHTS_F32)
    w = ops.p2m_build_weights(big.mesh, big.h, pos_b, 0, weights=w)
    w = ops.p2m_build_weights(big.mesh, big.h, pos_b, P2M_WEIGHTS_F32, weights=w)
    fresh = ops.p2m_build_weights(big.mesh, big.h, pos_b, P2M_WEIGHTS_F32)
    assert torch.equal(ops.p2m_project(w, v32), ops.p2m_project(fresh, v32))
    # the same sequence through the fused workspace
    for c, dt in ((small, torch.float32), (big, torch.float64), (big, torch.float32)):
        pos = _g(c.pos)
        vals = _g(c.vals, dt)
        ref, _ = _stored(c, pos, vals)
        assert torch.equal(ops.p2m_project_fused(c.mesh, c.h, pos, vals), ref)
