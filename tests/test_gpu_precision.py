"""The mixed path's P2M error taken apart (eq. p2m), on the 1,048,576-particle
workload: the FP32 result against the FP64 one is split into
  * the values' storage: values rounded to FP32, summed in FP64 with FP64
    weights (the GPU's FP64 path);
  * the weights' storage: the exported FP64 weights rounded to FP32, summed in
    FP64 on the host with the rounded values;
  * the FP32 arithmetic: the GPU's FP32 path against that host sum,
and each share is checked node by node against its a priori bound, with
u = 2^-24 and S_i = sum_k |w_k| |v_k| over node i's row of K_i entries:
  storage of values  <= u S_i          (every |v32 - v| <= u |v|)
  storage of weights <= u S_i (1 + u)  (every |w32 - w| <= u |w|)
  FP32 arithmetic    <= (2 K_i + 2) u S_i (1 + u)
                        (a rounded product and a rounded sum per entry, two
                        more sums across the quad; any order)
plus 1e-14 S_i for the FP64 sums on either side."""
import numpy as np
import pytest
import torch

import workloads as wl
from paper_1610_05266_amd import ops
from paper_1610_05266_amd._lib import P2M_WEIGHTS_F32

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
U = 2.0 ** -24


def test_fp32_error_shares_of_p2m():
    c = wl.config2()
    print(f"[gpu] FP32 error shares, C2 N={c.N}", flush=True)
    pos = torch.from_numpy(c.pos).to(DEV)
    w = ops.p2m_build_weights(c.mesh, c.h, pos, P2M_WEIGHTS_F32)
    v64 = c.vals
    v32 = v64.astype(np.float32)
    ref = ops.p2m_project(w, torch.from_numpy(v64).to(DEV)).cpu().numpy()
    a = ops.p2m_project(w, torch.from_numpy(v32.astype(np.float64)).to(DEV)).cpu().numpy()
    b = ops.p2m_project(w, torch.from_numpy(v32).to(DEV)).double().cpu().numpy()
    idx, wt, cnt, _ = (t.numpy() for t in w.export())
    K, nn = wt.shape
    live = np.arange(K)[:, None] < cnt[None, :]
    ids = np.where(live, idx, 0)
    w64 = np.where(live, wt, 0.0)
    w32 = w64.astype(np.float32).astype(np.float64)
    vv = v32.astype(np.float64)[ids]                      # [K, n_nodes, C]
    c_host = np.einsum("kn,knc->nc", w32, vv)
    S = np.einsum("kn,knc->nc", np.abs(w64), np.abs(v64[ids]) * (1.0 + U))
    tiny = 1e-14 * S
    shares = {
        "values' storage": (np.abs(a - ref), U * S),
        "weights' storage": (np.abs(c_host - a), U * S * (1.0 + U)),
        "FP32 arithmetic": (np.abs(b - c_host), (2 * cnt[:, None] + 2) * U * S * (1.0 + U)),
    }
    scale = np.abs(ref).max()
    for name, (err, bound) in shares.items():
        print(f"  {name}: max {err.max() / scale:.3e} of max|ref|, "
              f"max err/bound {np.max(err / np.maximum(bound + tiny, 1e-300)):.3f}", flush=True)
        assert np.all(err <= bound + tiny), name
    # the three shares add up to the mixed path's error, within the bar
    assert np.abs(b - ref).max() <= 1e-5 * scale
