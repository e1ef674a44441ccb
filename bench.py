#!/usr/bin/env python3
"""Benchmark of the particle <-> mesh projection round trip on one MI355X.

One step = the whole forward hot path over one synthetic particle set, with
the particle shape functions rebuilt every step (the method recomputes them
whenever particles move): binning, weight build (Delaunay + moment solves),
P2M (eq. p2m) and M2P (eq. m2p) of the P2M result.  Workload: 256x256 mesh,
1024x1024 jittered lattice (h = H/4, jitter 0.3h), 3 channels (Taylor-Green
u, v, p), randomly permuted particle order, inputs resident in HBM.

Prints one JSON line.  ``value`` is the round-trip rate of the mixed form
(FP32 values, weights and sums; FP64 geometry and solves); the plain FP64
form is timed in the same run and reported beside it.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

METRIC = "P2M+M2P round-trip Mparticles/s + % HBM roofline; FP32-mixed vs FP64 at ≤1e-5"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_VECTOR_PEAK_TFS = 78.6    # MI355X FP64 vector
# VALU issue: 256 CUs x 4 SIMDs, one wave64 instruction per SIMD every 4
# cycles at 2.4 GHz
VALU_ISSUE_PEAK_G = 256 * 4 * 2.4 / 4
# algorithmic FP64 work of the weight build per node (moment assembly of the
# three edge systems, Gram/Cholesky/solve with one refinement, weights)
# algorithmic FP64 work of the weight build per node, by kernel:
#   fast pass (certified local Delaunay): ~20 gift-wrap steps over ~25
#     candidates at ~12 flop per bisector key, plus one nearest search;
#     boundary-ring nodes: 12 nearest-particle rounds over ~25 candidates;
#   weights: three edge systems (moments, Cholesky, one refinement step,
#     weights), or one closure system.
FAST_FLOP_INTERIOR = 6000.0
FAST_FLOP_RING = 900.0
WEIGHTS_FLOP_INTERIOR = 2100.0
WEIGHTS_FLOP_CLOSURE = 700.0
TRAFFIC_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                            "roundtrip_256x256_1M_hbm_traffic.md")
# FP64 instruction counts of the build kernels (rocprofv3 SQ counters):
# 64 x (2 FMA + ADD + MUL) wave instructions per launch
COUNTERS_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                             "build_kernels_256x256_1M_counters.md")


def parse(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip timing the CPU oracle")
    ap.add_argument("--no-oracle-check", action="store_true", help="skip the sampled oracle comparison")
    ap.add_argument("--no-tune", action="store_true", help="keep the library's default build options")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the linear-FE and kinematic-loop measurements (profiles of the headline step)")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the batched (64 sets), 4.2M-particle and 16.8M-particle BF16 measurements")
    ap.add_argument("--only-large", action="store_true",
                    help="time the large workloads only (profiles of their kernels)")
    ap.add_argument("--set", action="append", default=[], metavar="NAME=VALUE",
                    help="set a build option (p2m_set_option) instead of autotuning")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="end with one plain device copy of MIB MiB (calibrates profiler byte counters)")
    ap.add_argument("--no-graph", action="store_true",
                    help="launch every step from the host instead of replaying a captured HIP graph")
    ap.add_argument("--cpu-side", type=float, default=1.0,
                    help="side of the sub-square of the workload the CPU oracle is timed on")
    return ap.parse_args(argv)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def rel_errs(got, ref):
    import numpy as np

    d = np.asarray(got, np.float64) - np.asarray(ref, np.float64)
    return (float(np.linalg.norm(d) / np.linalg.norm(ref)), float(np.abs(d).max() / np.abs(ref).max()))


def source_digest():
    """Digest of the HIP sources the measured kernels are built from."""
    import hashlib

    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1610_05266_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".h")):
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def counted_flops(kernel):
    """FP64 flops per launch of `kernel` counted by the committed rocprofv3
    instruction counters, or None when there are none or the sources changed
    since they were taken."""
    try:
        text = open(COUNTERS_FILE).read()
    except OSError:
        return None
    import re

    m = re.search(r"^source_digest: (\w+)$", text, flags=re.M)
    if not m or m.group(1) != source_digest():
        return None
    m = re.search(r"^fp64_flop_per_launch " + re.escape(kernel.replace(" ", "")) + r" (\d+)$", text, flags=re.M)
    return int(m.group(1)) if m else None


def counted_valu(kernel):
    """VALU wave instructions per launch of `kernel` from the committed
    instruction counters (SQ_INSTS_VALU), or None when stale or absent."""
    try:
        text = open(COUNTERS_FILE).read()
    except OSError:
        return None
    import re

    m = re.search(r"^source_digest: (\w+)$", text, flags=re.M)
    if not m or m.group(1) != source_digest():
        return None
    m = re.search(r"^valu_insts_per_launch " + re.escape(kernel.replace(" ", "")) + r" (\d+)$", text, flags=re.M)
    return int(m.group(1)) if m else None


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, calibrated on a plain copy), or None
    when there is none or the sources changed since it was taken."""
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    import re

    m = re.search(r"^source_digest: (\w+)$", text, flags=re.M)
    if not m or m.group(1) != source_digest():
        return None
    m = re.search(r"^traffic_bytes_per_launch " + re.escape(kernel.replace(" ", "")) + r" (\d+)$", text, flags=re.M)
    return int(m.group(1)) if m else None


def cpu_baseline(cloud, side):
    """Time the CPU oracle (as it stands) on the sub-square [0, side]^2 of the
    same workload: P2M weights + P2M + M2P of the result."""
    import numpy as np

    import oracle
    from oracle import Mesh as OMesh, P2MOracle

    m = cloud.mesh
    n_sub = int(round(side / m.H))
    side = n_sub * m.H
    keep = (cloud.pos[:, 0] <= side) & (cloud.pos[:, 1] <= side)
    pos = cloud.pos[keep]
    vals = cloud.vals[keep]
    om = OMesh(n_sub, n_sub, m.H)
    try:
        from threadpoolctl import threadpool_info

        threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count() or 1
    t0 = time.perf_counter()
    orc = P2MOracle(pos, om, cloud.h)
    W, _ = orc.matrix()
    t1 = time.perf_counter()
    mesh_vals = W @ vals
    t2 = time.perf_counter()
    oracle.m2p(om, mesh_vals, pos)
    t3 = time.perf_counter()
    t = t3 - t0
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {
        "value": round(pos.shape[0] / t / 1e6, 4),
        "unit": "Mparticles/s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": (f"sub-square [0,{side:g}]^2 of the workload: {pos.shape[0]} particles, "
                   f"{om.nx}x{om.ny} cells; FP64 Qhull (1 thread) + LAPACK SVD weights + P2M + M2P, "
                   f"{t:.1f} s"),
        "phases_s": {"build": round(t1 - t0, 3), "project": round(t2 - t1, 4), "interpolate": round(t3 - t2, 4)},
        "cpu_model": model,
        "logical_cpus": os.cpu_count(),
    }


def hbm_entry(nbytes, ms):
    gbs = nbytes / (ms * 1e-3) / 1e9
    return {"algorithmic_bytes": int(nbytes), "achieved_GBs": round(gbs, 2), "frac": round(gbs / HBM_PEAK_GBS, 5)}


def large_workloads(a, dev, time_loop, as_graph, check_replay, phase_times, graph_notes, tuning, log):
    """The other measured workloads, each timed as HIP graph replays:
    * 64 independent sets (~10 M particles, h = H/2) built, projected and
      interpolated in one launch sequence, with the build options tuned on it;
    * the 4.2 M-particle differentiation workload: M2P -> P2M -> loss
      residual -> full backward (grad of values, positions and mesh input);
    * the 16.8 M-particle advected cloud with BF16 particle storage: P2M (and
      M2P of its result) forward, P2M backward to values and positions.
    Algorithmic bytes: forward N (2*16 + (v_in + v_out) C) + N_m C (v_out +
    v_in); a backward adds N (2 C v + 16 + 16) + 2 N_m C v (gradients of values
    in and out, positions read and gradient written, mesh gradients)."""
    import numpy as np
    import torch

    import workloads as wl
    from paper_1610_05266_amd import ops, tune
    from paper_1610_05266_amd._lib import P2M_DETERMINISTIC, P2M_WEIGHTS_F32

    out = {}
    # ---- 64 sets in one launch sequence
    log("large: 64-set batch")
    sets = wl.config3()
    offs = np.concatenate([[0], np.cumsum([c.N for c in sets])])
    b = ops.Batch([c.mesh for c in sets], [c.h for c in sets], offs)
    P = torch.from_numpy(np.concatenate([c.pos for c in sets])).to(dev)
    V = torch.from_numpy(np.concatenate([c.vals for c in sets])).to(dev, torch.float32)
    C3 = V.shape[1]
    wb = ops.p2m_build_weights_batched(b, P, P2M_WEIGHTS_F32)
    dgb = wb.diag()
    key = tune.workload_key(torch.cuda.get_device_name(dev), b.N, b.n_nodes, 0.5, P2M_WEIGHTS_F32) + "|64 sets"
    tres = None
    if not a.no_tune and not a.set:
        tres = tune.autotune(lambda: ops.p2m_build_weights_batched(b, P, P2M_WEIGHTS_F32, weights=wb,
                                                                   check_diag=False),
                             lambda hd: ops.p2m_project(hd, V), key)
        log(f"large: batch tuning {tres.options} {tres.median_ms:.4f} ms (default {tres.default_ms:.4f})")
    bm = torch.empty((b.n_nodes, C3), dtype=torch.float32, device=dev)
    bo = torch.empty_like(V)

    def step3():
        ops.p2m_build_weights_batched(b, P, P2M_WEIGHTS_F32, weights=wb, check_diag=False)
        ops.p2m_project(wb, V, out=bm)
        ops.m2p_interpolate_batched(b, bm, P, out=bo)

    run3 = as_graph(step3)
    if run3 is not step3:
        check_replay(run3, step3, [bm, bo])
    ms3 = time_loop(run3, "batch64", steps=max(3, a.steps // 2), warmup=2)
    ph3 = phase_times(step3)
    B3 = b.N * (2 * 16 + 8 * C3) + b.n_nodes * C3 * 8
    out["batch64"] = {
        "workload": f"64 independent sets, {b.N} particles, {b.n_nodes} nodes, meshes 64^2..384^2 (h=H/2), "
                    "4 FP32 channels, seeded; build + P2M + M2P of all sets in one launch sequence",
        "ms_per_step": round(ms3, 5), "Mparticles_per_s": round(b.N / (ms3 * 1e-3) / 1e6, 3),
        "round_trip_hbm": hbm_entry(B3, ms3), "kernels_ms": {k: round(v, 5) for k, v in ph3.items()},
        "diag": {k: dgb[k] for k in ("slow_nodes", "failed_nodes", "rank_deficient", "svd_systems")},
        "tuning": None if tres is None else {"options": tres.options, "build_ms_tuned": round(tres.median_ms, 5),
                                             "build_ms_default": round(tres.default_ms, 5), "cached": tres.cached}}
    log(f"large: batch64 {ms3:.4f} ms/step")
    if tres is not None and tuning is not None:
        tune.apply_options(tuning["options"])
    del wb, P, V, bm, bo, b, sets

    # ---- 4.2 M particles: M2P -> P2M -> loss -> full backward
    log("large: 4.2M round trip with backward")
    c = wl.config4()
    mesh = ops.Mesh.of(c.mesh)
    N, nn = c.N, mesh.n_nodes
    pos = torch.from_numpy(c.pos).to(dev)
    f32 = torch.from_numpy(c.extra["f_mesh"]).to(dev, torch.float32)
    g32 = torch.from_numpy(c.extra["g_mesh"]).to(dev, torch.float32)
    C4 = f32.shape[1]
    w4 = ops.p2m_build_weights(mesh, c.h, pos, P2M_WEIGHTS_F32)
    a32 = torch.empty((N, C4), dtype=torch.float32, device=dev)
    o32 = torch.empty((nn, C4), dtype=torch.float32, device=dev)
    gpos = torch.zeros_like(pos)

    def fwd4():
        ops.m2p_interpolate(mesh, f32, pos, out=a32)
        ops.p2m_build_weights(mesh, c.h, pos, P2M_WEIGHTS_F32, weights=w4, check_diag=False)
        ops.p2m_project(w4, a32, out=o32)

    def step4():
        fwd4()
        r = o32 - g32
        gv, gw = ops.p2m_project_backward(w4, r, a32, want_vals=True, want_w=True)
        gpos.zero_()
        ops.p2m_build_weights_backward(w4, pos, gw, grad_pos=gpos)
        # the M2P adjoint gathered per node through the build's binning (the
        # handle was built from the same positions): no atomics
        ops.m2p_interpolate_backward_binned(w4, f32, pos, gv, want_mesh=True, grad_pos=gpos)

    # the same step with the deterministic adjoints: the build also indexes
    # the entries by particle, P2M^t and the position adjoint gather per
    # particle (no atomics)
    w4d = ops.p2m_build_weights(mesh, c.h, pos, P2M_WEIGHTS_F32 | P2M_DETERMINISTIC)

    def step4d():
        ops.m2p_interpolate(mesh, f32, pos, out=a32)
        ops.p2m_build_weights(mesh, c.h, pos, P2M_WEIGHTS_F32 | P2M_DETERMINISTIC, weights=w4d, check_diag=False)
        ops.p2m_project(w4d, a32, out=o32)
        r = o32 - g32
        gv, gw = ops.p2m_project_backward(w4d, r, a32, want_vals=True, want_w=True)
        gpos.zero_()
        ops.p2m_build_weights_backward(w4d, pos, gw, grad_pos=gpos)
        ops.m2p_interpolate_backward_binned(w4d, f32, pos, gv, want_mesh=True, grad_pos=gpos)

    steps = max(3, a.steps // 2)
    run4f = as_graph(fwd4)
    msf4 = time_loop(run4f, "c4_forward", steps=steps, warmup=2)
    run4 = as_graph(step4)
    ms4 = time_loop(run4, "c4_forward_backward", steps=steps, warmup=2)
    ph4 = phase_times(step4)
    ms4d = time_loop(as_graph(step4d), "c4_forward_backward_deterministic", steps=steps, warmup=2)
    ph4d = phase_times(step4d)
    Bf4 = N * (2 * 16 + 8 * C4) + nn * C4 * 8
    Bb4 = Bf4 + N * (8 * C4 + 32) + 2 * nn * C4 * 4
    out["c4"] = {
        "workload": f"512x512 mesh, 2048x2048 jittered lattice ({N} particles, h=H/4, jitter 0.25h, seed 4), "
                    "2 FP32 channels: M2P of a mesh field, P2M (weights rebuilt), loss residual, backward to "
                    "values, positions and the mesh input",
        "forward_ms": round(msf4, 5), "forward_Mparticles_per_s": round(N / (msf4 * 1e-3) / 1e6, 3),
        "forward_hbm": hbm_entry(Bf4, msf4),
        "ms_per_step": round(ms4, 5), "Mparticles_per_s": round(N / (ms4 * 1e-3) / 1e6, 3),
        "forward_backward_hbm": hbm_entry(Bb4, ms4), "kernels_ms": {k: round(v, 5) for k, v in ph4.items()},
        "backward_kernels_hbm": {
            "m2p_bwd": hbm_entry(N * (16 + 4 * C4 + 16) + nn * C4 * 4, ph4["m2p_bwd"]),
            "project_bwd": hbm_entry(nn * C4 * 4 + N * C4 * 4, ph4["project_bwd"])},
        "deterministic": {"note": "built with P2M_DETERMINISTIC: P2M^t and the position adjoint gathered per "
                                  "particle in a fixed order (the build indexes the entries by particle)",
                          "ms_per_step": round(ms4d, 5), "Mparticles_per_s": round(N / (ms4d * 1e-3) / 1e6, 3),
                          "kernels_ms": {k: round(v, 5) for k, v in ph4d.items()}}}
    log(f"large: c4 forward {msf4:.4f} ms, forward+backward {ms4:.4f} ms (deterministic {ms4d:.4f} ms)")
    del w4, w4d, pos, f32, g32, a32, o32, gpos

    # ---- 16.8 M particles, BF16 particle storage: forward and backward
    log("large: 16.8M BF16 workload (generating)")
    c = wl.config5(device=str(dev))
    mesh = ops.Mesh.of(c.mesh)
    N, nn = c.N, mesh.n_nodes
    pos = torch.from_numpy(c.pos).to(dev)
    vb = torch.from_numpy(c.vals).to(dev, torch.bfloat16)
    C5 = vb.shape[1]
    nodes = np.asarray(c.mesh.node_xy())
    tgt = torch.from_numpy(np.stack([wl.tg_u(nodes[:, 0] - 0.05, nodes[:, 1] + 0.03),
                                     wl.tg_v(nodes[:, 0] - 0.05, nodes[:, 1] + 0.03),
                                     wl.tg_p(nodes[:, 0] - 0.05, nodes[:, 1] + 0.03)], 1)).to(dev, torch.float32)
    w5 = ops.p2m_build_weights(mesh, c.h, pos, P2M_WEIGHTS_F32)
    t5 = None
    if not a.no_tune and not a.set:
        # the advected cloud is sheared: its own build options
        key5 = tune.workload_key(torch.cuda.get_device_name(dev), N, nn, c.h / mesh.H, P2M_WEIGHTS_F32) + "|advected"
        t5 = tune.autotune(lambda: ops.p2m_build_weights(mesh, c.h, pos, P2M_WEIGHTS_F32, weights=w5,
                                                         check_diag=False),
                           lambda hd: ops.p2m_project(hd, vb), key5)
        log(f"large: c5 tuning {t5.options} {t5.median_ms:.4f} ms (default {t5.default_ms:.4f})")
        ops.p2m_build_weights(mesh, c.h, pos, P2M_WEIGHTS_F32, weights=w5)
    d5 = w5.diag()
    o5 = torch.empty((nn, C5), dtype=torch.float32, device=dev)
    back5 = torch.empty((N, C5), dtype=torch.bfloat16, device=dev)
    gp5 = torch.zeros_like(pos)

    def fwd5():
        ops.p2m_build_weights(mesh, c.h, pos, P2M_WEIGHTS_F32, weights=w5, check_diag=False)
        ops.p2m_project(w5, vb, out=o5)
        ops.m2p_interpolate(mesh, o5, pos, out=back5, bf16_out=True)

    def step5():
        fwd5()
        r = o5 - tgt
        gv, gw = ops.p2m_project_backward(w5, r, vb, want_vals=True, want_w=True)
        gp5.zero_()
        ops.p2m_build_weights_backward(w5, pos, gw, grad_pos=gp5)

    w5d = ops.p2m_build_weights(mesh, c.h, pos, P2M_WEIGHTS_F32 | P2M_DETERMINISTIC)

    def step5d():
        ops.p2m_build_weights(mesh, c.h, pos, P2M_WEIGHTS_F32 | P2M_DETERMINISTIC, weights=w5d, check_diag=False)
        ops.p2m_project(w5d, vb, out=o5)
        ops.m2p_interpolate(mesh, o5, pos, out=back5, bf16_out=True)
        r = o5 - tgt
        gv, gw = ops.p2m_project_backward(w5d, r, vb, want_vals=True, want_w=True)
        gp5.zero_()
        ops.p2m_build_weights_backward(w5d, pos, gw, grad_pos=gp5)

    steps = max(3, a.steps // 4)
    msf5 = time_loop(as_graph(fwd5), "c5_forward", steps=steps, warmup=1)
    ms5 = time_loop(as_graph(step5), "c5_forward_backward", steps=steps, warmup=1)
    ph5 = phase_times(step5)
    ms5d = time_loop(as_graph(step5d), "c5_forward_backward_deterministic", steps=steps, warmup=1)
    ph5d = phase_times(step5d)
    Bf5 = N * (2 * 16 + 2 * C5 + 2 * C5) + nn * C5 * 8
    Bb5 = Bf5 + N * (2 * C5 + 4 * C5 + 16 + 16) + nn * C5 * 4
    out["c5"] = {
        "workload": f"1024x1024 mesh, 4096x4096 jittered lattice advected 200 Euler steps through the steady "
                    f"vortex ({N} particles, h=H/4), 3 channels in BF16 particle storage, FP32 sums, FP64 "
                    "geometry: P2M (weights rebuilt) and M2P of its result (BF16 out), P2M backward to values "
                    "and positions",
        "forward_ms": round(msf5, 5), "forward_Mparticles_per_s": round(N / (msf5 * 1e-3) / 1e6, 3),
        "forward_hbm": hbm_entry(Bf5, msf5),
        "ms_per_step": round(ms5, 5), "Mparticles_per_s": round(N / (ms5 * 1e-3) / 1e6, 3),
        "forward_backward_hbm": hbm_entry(Bb5, ms5), "kernels_ms": {k: round(v, 5) for k, v in ph5.items()},
        "diag": {k: d5[k] for k in ("slow_nodes", "failed_nodes", "rank_deficient", "svd_systems",
                                    "max_gram_cond")},
        "tuning": None if t5 is None else {"options": t5.options, "build_ms_tuned": round(t5.median_ms, 5),
                                           "build_ms_default": round(t5.default_ms, 5), "cached": t5.cached},
        "deterministic": {"note": "built with P2M_DETERMINISTIC: P2M^t and the position adjoint gathered per "
                                  "particle in a fixed order (the build indexes the entries by particle)",
                          "ms_per_step": round(ms5d, 5), "Mparticles_per_s": round(N / (ms5d * 1e-3) / 1e6, 3),
                          "kernels_ms": {k: round(v, 5) for k, v in ph5d.items()}}}
    log(f"large: c5 forward {msf5:.4f} ms, forward+backward {ms5:.4f} ms (deterministic {ms5d:.4f} ms)")
    if t5 is not None and tuning is not None:
        tune.apply_options(tuning["options"])
    del w5, w5d, pos, vb, o5, back5, gp5
    torch.cuda.synchronize()
    return out


def main(argv=None):
    a = parse(argv)
    if a.only_large:
        a.no_extras = a.no_cpu_baseline = a.no_oracle_check = True
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); the multi-GPU design is "
              "described in DESIGN.md and is not built.", file=sys.stderr)
        return 2
    import numpy as np
    import torch

    import workloads as wl
    from paper_1610_05266_amd import load, ops
    from paper_1610_05266_amd._lib import P2M_WEIGHTS_F32

    lib = load()
    dev = torch.device("cuda:0")
    log("generating workload")
    cloud = wl.config2()
    mesh = ops.Mesh.of(cloud.mesh)
    N, C, nn = cloud.N, cloud.vals.shape[1], mesh.n_nodes
    pos = torch.from_numpy(cloud.pos).to(dev)
    v64 = torch.from_numpy(cloud.vals).to(dev)
    v32 = v64.float().contiguous()
    mesh64 = torch.empty((nn, C), dtype=torch.float64, device=dev)
    mesh32 = torch.empty((nn, C), dtype=torch.float32, device=dev)
    out64 = torch.empty((N, C), dtype=torch.float64, device=dev)
    out32 = torch.empty((N, C), dtype=torch.float32, device=dev)
    w = ops.Weights()
    ops.p2m_build_weights(mesh, cloud.h, pos, P2M_WEIGHTS_F32, weights=w, check_diag=True)
    diag = w.diag()
    log(f"diag {diag}")

    tuning = None
    if a.set:
        for kv in a.set:
            k, v = kv.split("=", 1)
            ops.p2m_set_option(k, float(v))
        tuning = {"options": dict(kv.split("=", 1) for kv in a.set), "fixed": True}
    elif not a.no_tune:
        from paper_1610_05266_amd import tune

        log("autotuning the build options")
        key = tune.workload_key(torch.cuda.get_device_name(dev), N, nn, cloud.h / mesh.H, P2M_WEIGHTS_F32)
        tuning_key = key
        res = tune.autotune(
            lambda: ops.p2m_build_weights(mesh, cloud.h, pos, P2M_WEIGHTS_F32, weights=w, check_diag=False),
            lambda h: ops.p2m_project(h, v32), key)
        tuning = {"options": res.options, "build_ms_tuned": round(res.median_ms, 5),
                  "build_ms_default": round(res.default_ms, 5), "cached": res.cached}
        log(f"tuning {tuning}")
        # M2P's particles per thread, on the mesh field of this workload
        ops.p2m_build_weights(mesh, cloud.h, pos, P2M_WEIGHTS_F32, weights=w, check_diag=False)
        ops.p2m_project(w, v32, out=mesh32)
        tuning["m2p"] = tune.choose(tune.m2p_variants(), lambda: ops.m2p_interpolate(mesh, mesh32, pos, out=out32),
                                    lambda: [out32], key + "|m2p")
        log(f"m2p tuning {tuning['m2p']}")

    def step(mixed):
        ops.p2m_build_weights(mesh, cloud.h, pos, P2M_WEIGHTS_F32 if mixed else 0, weights=w, check_diag=False)
        if mixed:
            ops.p2m_project(w, v32, out=mesh32)
            ops.m2p_interpolate(mesh, mesh32, pos, out=out32)
        else:
            ops.p2m_project(w, v64, out=mesh64)
            ops.m2p_interpolate(mesh, mesh64, pos, out=out64)

    def step_fused(mixed):
        # the recompute form: the fast path's rows projected as they are
        # weighted, no weights kept for them (the same bits as step)
        if mixed:
            ops.p2m_project_fused(mesh, cloud.h, pos, v32, out=mesh32)
            ops.m2p_interpolate(mesh, mesh32, pos, out=out32)
        else:
            ops.p2m_project_fused(mesh, cloud.h, pos, v64, out=mesh64)
            ops.m2p_interpolate(mesh, mesh64, pos, out=out64)

    def eager_cached(mixed):
        if mixed:
            ops.p2m_project(w, v32, out=mesh32)
            ops.m2p_interpolate(mesh, mesh32, pos, out=out32)
        else:
            ops.p2m_project(w, v64, out=mesh64)
            ops.m2p_interpolate(mesh, mesh64, pos, out=out64)

    graph_notes = []

    def as_graph(fn):
        """fn captured as a HIP graph (replays without host launch overhead),
        or fn itself when graphs are off or capture fails."""
        if a.no_graph:
            return fn
        try:
            side = torch.cuda.Stream()
            side.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(side):
                fn()
            torch.cuda.current_stream().wait_stream(side)
            torch.cuda.synchronize()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                fn()
            torch.cuda.synchronize()
            graphs.append(g)
            return g.replay
        except Exception as exc:  # noqa: BLE001 - report and time eagerly
            graph_notes.append(f"graph capture failed ({exc}); eager launches timed")
            torch.cuda.synchronize()
            return fn

    graphs = []

    def check_replay(run, fn, outs):
        """Every replay must reproduce the eager step bit for bit."""
        fn()
        torch.cuda.synchronize()
        ref = [o.clone() for o in outs]
        for _ in range(3):
            run()
            torch.cuda.synchronize()
            for o, r in zip(outs, ref):
                if not torch.equal(o, r):
                    raise RuntimeError("graph replay differs from the eager step")
            fn()
            torch.cuda.synchronize()

    step_stats = {}

    def time_loop(run, label=None, steps=None, warmup=None):
        """Mean ms per step of `steps` runs after `warmup` untimed ones; an
        event between consecutive runs gives the per-step median and IQR
        (kept in step_stats[label])."""
        steps = a.steps if steps is None else steps
        warmup = a.warmup if warmup is None else warmup
        for _ in range(warmup):
            run()
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        ev[0].record()
        for k in range(steps):
            run()
            ev[k + 1].record()
        torch.cuda.synchronize()
        per = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(steps)])
        mean = ev[0].elapsed_time(ev[steps]) / steps
        if label:
            q25, q50, q75 = np.percentile(per, [25, 50, 75])
            step_stats[label] = {"mean_ms": round(mean, 5), "median_ms": round(float(q50), 5),
                                 "iqr_ms": [round(float(q25), 5), round(float(q75), 5)], "steps": steps}
        return mean

    def timed(mixed):
        import ctypes

        fn = (lambda: step(mixed))
        run = as_graph(fn)
        if run is not fn:
            try:
                check_replay(run, fn, [mesh32, out32] if mixed else [mesh64, out64])
            except RuntimeError as exc:
                graph_notes.append(f"{exc}; eager launches timed")
                run = fn
        ms = time_loop(run, "mixed" if mixed else "fp64")
        # per-kernel GPU times from the library's own events, in a separate
        # eager pass so that the event records do not perturb the timed loop
        return ms, phase_times(lambda: step(mixed))

    def phase_times(fn, names=("bin", "build", "project", "m2p", "build_fast", "build_slow", "weights",
                               "k_weights", "k_weights_rd", "m2p_bwd", "project_bwd", "build_bwd")):
        """Average ms per launch of each kernel group over a.steps eager runs
        of fn, from the library's events on the stream each group runs on."""
        import ctypes

        lib.p2m_profile_enable(1)
        for _ in range(a.steps):
            fn()
        torch.cuda.synchronize()
        phases = {}
        for ph in names:
            tot, cnt = ctypes.c_double(), ctypes.c_int64()
            lib.p2m_profile_read(ph.encode(), ctypes.byref(tot), ctypes.byref(cnt))
            if cnt.value:
                phases[ph] = tot.value / cnt.value
        lib.p2m_profile_enable(0)
        return phases

    def cached(mixed):
        """P2M + M2P with the weights of the last build (no rebuild)."""
        fn = (lambda: eager_cached(mixed))
        run = as_graph(fn)
        if run is not fn:
            try:
                check_replay(run, fn, [mesh32, out32] if mixed else [mesh64, out64])
            except RuntimeError as exc:
                graph_notes.append(f"{exc}; eager launches timed")
                run = fn
        return time_loop(run, "cached_mixed" if mixed else "cached_fp64")

    log("timing FP64 form")
    ms64, ph64 = timed(False)
    log(f"FP64 {ms64:.4f} ms/step phases {ph64}")
    log("timing mixed form")
    ms32, ph32 = timed(True)
    log(f"mixed {ms32:.4f} ms/step phases {ph32}")
    ref_mesh = {True: mesh32.clone(), False: None}
    step(False)
    ref_mesh[False] = mesh64.clone()
    step(True)  # the handle holds the mixed build again (the cached timings use it)

    def timed_fused(mixed):
        fn = (lambda: step_fused(mixed))
        fn()
        torch.cuda.synchronize()
        # the fused form must give the stored form's bits
        if not torch.equal(mesh32 if mixed else mesh64, ref_mesh[mixed]):
            raise RuntimeError("fused projection differs from the stored-weights projection")
        run = as_graph(fn)
        if run is not fn:
            try:
                check_replay(run, fn, [mesh32, out32] if mixed else [mesh64, out64])
            except RuntimeError as exc:
                graph_notes.append(f"fused: {exc}; eager launches timed")
                run = fn
        ms = time_loop(run, "fused_mixed" if mixed else "fused_fp64")
        return ms, phase_times(fn)

    log("timing the fused forms")
    fms64, fph64 = timed_fused(False)
    fms32, fph32 = timed_fused(True)
    log(f"fused: mixed {fms32:.4f} ms/step, FP64 {fms64:.4f} ms/step; phases {fph32}")
    stored = {"mixed_ms": round(ms32, 5), "fp64_ms": round(ms64, 5)}
    fused = {"mixed_ms": round(fms32, 5), "fp64_ms": round(fms64, 5),
             "phases_ms": {k: round(v, 5) for k, v in fph32.items()}}
    # the headline takes the faster library form of the same step: the
    # tuner's choice between the two (timed on graph replays, results equal
    # bit for bit, cached), or the faster of the timings above untuned
    if tuning is not None and not tuning.get("fixed"):
        from paper_1610_05266_amd import tune

        form = ["stored"]
        tuning["form"] = tune.choose(
            {"stored": lambda: form.__setitem__(0, "stored"), "fused": lambda: form.__setitem__(0, "fused")},
            lambda: (step if form[0] == "stored" else step_fused)(True), lambda: [mesh32, out32],
            tuning_key + "|form")
        log(f"form tuning {tuning['form']}")
        head_form = tuning["form"]["choice"]
        step(True)  # the handle holds the mixed build again (the cached timings use it)
    else:
        head_form = "fused" if fms32 < ms32 else "stored"
    ms32_head = ms32 if head_form == "stored" else fms32
    ms64_head = ms64 if head_form == "stored" else fms64
    # the weights handle now holds the mixed build (FP64 and FP32 weights)
    cms32 = cached(True)
    cms64 = cached(False)
    log(f"cached weights: mixed {cms32:.4f} ms, FP64 {cms64:.4f} ms per round trip")
    torch.cuda.synchronize()

    lms32 = kms32 = qms32 = qsetup = pms32 = pkms32 = None
    pdiag, pkdiag = {}, {}
    pktuning = None
    kdiag, ktuning = {}, None
    if not a.no_extras:
        # M2P with the mesh's quadratically consistent functions (FP32), on the
        # mesh values of the mixed step; the edge table is built once per mesh
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        mq = ops.MeshQCSF(mesh, dev)
        e1.record()
        torch.cuda.synchronize()
        qsetup = e0.elapsed_time(e1)
        qout = torch.empty_like(out32)

        def m2p_q():
            mq.interpolate(mesh32, pos, out=qout)

        run_q = as_graph(m2p_q)
        if run_q is not m2p_q:
            try:
                check_replay(run_q, m2p_q, [qout])
            except RuntimeError as exc:
                graph_notes.append(f"{exc}; eager launches timed")
                run_q = m2p_q
        qms32 = time_loop(run_q)
        log(f"M2P with mesh QCSF (FP32) {qms32:.4f} ms, table {qsetup:.3f} ms once")

        # the same round trip with the linear FE particle functions (P2M_LINEAR:
        # triangle located, rings and solves skipped), weights rebuilt every step
        wlin = ops.p2m_build_weights(mesh, cloud.h, pos, P2M_WEIGHTS_F32 | ops.P2M_LINEAR, check_diag=True)
        lmesh32, lout32 = torch.empty_like(mesh32), torch.empty_like(out32)

        def step_linear():
            ops.p2m_build_weights(mesh, cloud.h, pos, P2M_WEIGHTS_F32 | ops.P2M_LINEAR, weights=wlin,
                                  check_diag=False)
            ops.p2m_project(wlin, v32, out=lmesh32)
            ops.m2p_interpolate(mesh, lmesh32, pos, out=lout32)

        run_lin = as_graph(step_linear)
        if run_lin is not step_linear:
            try:
                check_replay(run_lin, step_linear, [lmesh32, lout32])
            except RuntimeError as exc:
                graph_notes.append(f"{exc}; eager launches timed")
                run_lin = step_linear
        lms32 = time_loop(run_lin)
        log(f"linear FE round trip (mixed) {lms32:.4f} ms")

        # the same round trip in the paper's periodic box: (-1, 1)^2, k = pi,
        # the same mesh and lattice sizes, weights rebuilt every step
        pcl = wl.periodic_tg_cloud(mesh.nx, 4, 0.30, seed=2)
        ppos = torch.from_numpy(pcl.pos).to(dev)
        pv32 = torch.from_numpy(pcl.vals).to(dev, torch.float32)
        pflags = P2M_WEIGHTS_F32 | ops.P2M_PERIODIC
        wper = ops.p2m_build_weights(pcl.mesh, pcl.h, ppos, pflags, check_diag=True)
        pmesh32 = torch.empty((pcl.mesh.n_nodes, pv32.shape[1]), dtype=torch.float32, device=dev)
        pout32 = torch.empty_like(pv32)

        def step_periodic():
            ops.p2m_build_weights(pcl.mesh, pcl.h, ppos, pflags, weights=wper, check_diag=False)
            ops.p2m_project(wper, pv32, out=pmesh32)
            ops.m2p_interpolate(pcl.mesh, pmesh32, ppos, out=pout32)

        run_per = as_graph(step_periodic)
        if run_per is not step_periodic:
            try:
                check_replay(run_per, step_periodic, [pmesh32, pout32])
            except RuntimeError as exc:
                graph_notes.append(f"{exc}; eager launches timed")
                run_per = step_periodic
        pms32 = time_loop(run_per)
        pdiag = wper.diag(check_status=False)
        log(f"periodic round trip (mixed) {pms32:.4f} ms, diag {pdiag}")

        # one step of the periodic kinematic loop: the periodic flow (a quarter
        # cell per step) carries particles across the box sides, wrapped back
        pamp, pdt = 0.1, 0.25 * pcl.mesh.H / (0.1 * 2.0 * math.pi)
        pkmesh = pmesh32.clone()

        def step_periodic_kinematic():
            ops.m2p_interpolate(pcl.mesh, pkmesh, ppos, out=pout32)
            ops.p2m_advect(pcl.mesh, ppos, pamp, pdt, periodic=True)
            ops.p2m_build_weights(pcl.mesh, pcl.h, ppos, pflags, weights=wper, check_diag=False)
            ops.p2m_project(wper, pout32, out=pkmesh)

        # as for the bounded loop: shear the cloud, then tune the options for it
        for _ in range(24):
            step_periodic_kinematic()
        torch.cuda.synchronize()
        pktuning = None
        if not a.no_tune and not a.set:
            from paper_1610_05266_amd import tune

            pkkey = tune.workload_key(torch.cuda.get_device_name(dev), N, pcl.mesh.n_nodes, pcl.h / pcl.mesh.H,
                                      pflags) + "|sheared"
            pkres = tune.autotune(
                lambda: ops.p2m_build_weights(pcl.mesh, pcl.h, ppos, pflags, weights=wper, check_diag=False),
                lambda hd: ops.p2m_project(hd, pout32), pkkey)
            pktuning = {"options": pkres.options, "build_ms_tuned": round(pkres.median_ms, 5),
                        "build_ms_default": round(pkres.default_ms, 5), "cached": pkres.cached}
            log(f"periodic kinematic tuning {pktuning}")
        pkms32 = time_loop(as_graph(step_periodic_kinematic))
        if pktuning is not None:
            from paper_1610_05266_amd import tune

            tune.apply_options(tuning["options"])
        pkdiag = wper.diag(check_status=False)
        log(f"periodic kinematic step (mixed) {pkms32:.4f} ms, diag {pkdiag}")
        del wper, ppos, pv32, pmesh32, pout32, pkmesh

        # one step of the kinematic projection loop (mixed form): particle values
        # from the mesh, the particles moved one midpoint step in the cellular flow
        # of the box (about a quarter cell), their functions rebuilt, and P2M.  The
        # particles move at every replay, so replays are not compared with an
        # eager step; a copy of the positions keeps the other measurements intact.
        kpos = pos.clone()
        kamp, kdt = 0.1, 0.25 * mesh.H / (0.1 * math.pi)
        wk = ops.p2m_build_weights(mesh, cloud.h, kpos, P2M_WEIGHTS_F32, check_diag=True)
        kmesh, kvals = mesh32.clone(), torch.empty_like(out32)

        def step_kinematic():
            ops.m2p_interpolate(mesh, kmesh, kpos, out=kvals)
            ops.p2m_advect(mesh, kpos, kamp, kdt)
            ops.p2m_build_weights(mesh, cloud.h, kpos, P2M_WEIGHTS_F32, weights=wk, check_diag=False)
            ops.p2m_project(wk, kvals, out=kmesh)

        # shear the cloud first (as a loop does within a few dozen steps), then
        # tune the build options for that cloud unless tuning is off: a sheared
        # cloud has long thin triangles whose circumdisks leave the default radius
        for _ in range(24):
            step_kinematic()
        torch.cuda.synchronize()
        ktuning = None
        if not a.no_tune and not a.set:
            from paper_1610_05266_amd import tune

            kkey = tune.workload_key(torch.cuda.get_device_name(dev), N, nn, cloud.h / mesh.H, P2M_WEIGHTS_F32) + "|sheared"
            kres = tune.autotune(
                lambda: ops.p2m_build_weights(mesh, cloud.h, kpos, P2M_WEIGHTS_F32, weights=wk, check_diag=False),
                lambda hd: ops.p2m_project(hd, kvals), kkey)
            ktuning = {"options": kres.options, "build_ms_tuned": round(kres.median_ms, 5),
                       "build_ms_default": round(kres.default_ms, 5), "cached": kres.cached}
            log(f"kinematic tuning {ktuning}")
        kms32 = time_loop(as_graph(step_kinematic))
        kdiag = wk.diag(check_status=False)
        log(f"kinematic loop step (mixed) {kms32:.4f} ms, diag after the loop {kdiag}")
        if ktuning is not None:
            # the other measurements keep the options tuned for the ordered cloud
            from paper_1610_05266_amd import tune

            tune.apply_options(tuning["options"])

    large = None
    if not a.no_large:
        large = large_workloads(a, dev, time_loop, as_graph, check_replay, phase_times, graph_notes, tuning, log)

    # accuracy of the mixed form against the FP64 form (both full outputs)
    e_mesh = rel_errs(mesh32.cpu().numpy(), mesh64.cpu().numpy())
    e_part = rel_errs(out32.cpu().numpy(), out64.cpu().numpy())
    result_err = {"mixed_vs_fp64_mesh": e_mesh, "mixed_vs_fp64_particles": e_part}

    if not a.no_oracle_check:
        log("sampled oracle check")
        from oracle import Mesh as OMesh, P2MOracle

        om = OMesh.from_spec(cloud.mesh)
        rng = np.random.default_rng(0)
        sample = np.unique(np.concatenate([rng.choice(nn, 256, replace=False), [0, mesh.nx, nn - 1]]))
        orc = P2MOracle(cloud.pos, om, cloud.h, mode="local")
        Ws, _ = orc.matrix(sample)
        ref = Ws @ cloud.vals
        result_err["fp64_vs_oracle_sampled_nodes"] = rel_errs(mesh64.cpu().numpy()[sample], ref)
        result_err["mixed_vs_oracle_sampled_nodes"] = rel_errs(mesh32.cpu().numpy()[sample], ref)

    # per-kernel rooflines (times: the library's events around each launch)
    b32 = N * (2 * 16 + (4 + 4) * C) + nn * C * (4 + 4)
    ni, nc = diag["interior_nodes"], diag["closure_nodes"]
    # the fast pass's Delaunay work depends on the algorithm: its FP64 work
    # per launch as counted by the committed instruction counters (lane
    # operations issued on this workload), the hand model when they are stale
    fast_name = f"k_build_fast<{int(ops.p2m_get_option('fast_slots'))}>"
    fast_counted = counted_flops(fast_name)
    fast_work = fast_counted if fast_counted else FAST_FLOP_INTERIOR * ni + FAST_FLOP_RING * nc
    fast_unit = (f"{fast_counted / nn:.0f} FP64 flop/node counted (rocprofv3 FP64 instruction counters)"
                 if fast_counted else
                 f"{FAST_FLOP_INTERIOR:g} FP64 flop/interior node, {FAST_FLOP_RING:g}/ring node (model)")
    kern = {
        "k_build_fast": ("alu", fast_work, ph32["build_fast"], fast_unit),
        "k_weights": ("alu", WEIGHTS_FLOP_INTERIOR * ni + WEIGHTS_FLOP_CLOSURE * nc, ph32["k_weights"],
                      f"{WEIGHTS_FLOP_INTERIOR:g} FP64 flop/interior node, {WEIGHTS_FLOP_CLOSURE:g}/closure node"),
        "binning": ("hbm", 36.0 * N, ph32["bin"], "36 B/particle (16 in, 20 out)"),
        "k_project": ("hbm", N * 4 * C + nn * C * 4, ph32["project"], "values in + mesh out, FP32"),
        "k_m2p": ("hbm", N * (16 + 4 * C) + nn * 4 * C, ph32["m2p"], "positions + mesh in + values out, FP32"),
    }
    kernels = {}
    counted_names = {"k_build_fast": fast_name, "k_weights": "k_weights_slow<false, StoreRows>"}
    for name, (bound, work, ms, per_unit) in kern.items():
        if bound == "alu":
            ach = work / (ms * 1e-3) / 1e12
            kernels[name] = {"bound": "alu", "achieved": round(ach, 4), "peak": FP64_VECTOR_PEAK_TFS,
                             "unit": "TFLOP/s", "frac": round(ach / FP64_VECTOR_PEAK_TFS, 5),
                             "avg_launch_ms": round(ms, 5), "algorithmic_per_launch": f"{work:.4g} flop ({per_unit})"}
            cf = counted_flops(counted_names[name])
            if cf:
                # every FP64 lane operation the kernel issued (redundant lanes
                # of a quad included): its FP64 issue rate against the peak
                kernels[name]["counted_fp64_flop_per_launch"] = cf
                kernels[name]["counted_frac"] = round(cf / (ms * 1e-3) / 1e12 / FP64_VECTOR_PEAK_TFS, 5)
            cv = counted_valu(counted_names[name])
            if cv:
                # VALU instruction issue against the chip's issue rate: the
                # bound these kernels meet first (most of their instructions
                # are integer, compare, select and exchange work)
                rate = cv / (ms * 1e-3) / 1e9
                kernels[name]["valu_issue"] = {"achieved": round(rate, 2), "peak": VALU_ISSUE_PEAK_G,
                                               "unit": "G wave-instructions/s",
                                               "frac": round(rate / VALU_ISSUE_PEAK_G, 5),
                                               "per_launch": cv}
        else:
            ach = work / (ms * 1e-3) / 1e9
            kernels[name] = {"bound": "hbm", "achieved": round(ach, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": round(ach / HBM_PEAK_GBS, 5), "avg_launch_ms": round(ms, 5),
                             "algorithmic_per_launch": f"{work:.4g} B ({per_unit})"}
    dom = max(kernels, key=lambda k: kernels[k]["avg_launch_ms"])
    roof = dict(kernels[dom])
    roof["kernel"] = dom
    # the counter summary names template instances: the fast pass by its
    # candidate slots per lane
    prof_name = fast_name if dom == "k_build_fast" else dom
    roof["traffic"] = measured_traffic(prof_name)
    b64 = N * (2 * 16 + (8 + 8) * C) + nn * C * (8 + 8)
    rt = {"algorithmic_bytes": b32, "achieved_GBs": round(b32 / (ms32_head * 1e-3) / 1e9, 2),
          "frac": round(b32 / (ms32_head * 1e-3) / 1e9 / HBM_PEAK_GBS, 5)}
    rt64 = {"algorithmic_bytes": b64, "achieved_GBs": round(b64 / (ms64_head * 1e-3) / 1e9, 2),
            "frac": round(b64 / (ms64_head * 1e-3) / 1e9 / HBM_PEAK_GBS, 5)}

    cached_rt = {
        "note": "P2M + M2P with the weights of the last build (no rebuild); same algorithmic bytes",
        "mixed": {"ms_per_step": round(cms32, 5), "Mparticles_per_s": round(N / (cms32 * 1e-3) / 1e6, 3),
                  "achieved_GBs": round(b32 / (cms32 * 1e-3) / 1e9, 2),
                  "frac": round(b32 / (cms32 * 1e-3) / 1e9 / HBM_PEAK_GBS, 5)},
        "fp64": {"ms_per_step": round(cms64, 5), "Mparticles_per_s": round(N / (cms64 * 1e-3) / 1e6, 3),
                 "achieved_GBs": round(b64 / (cms64 * 1e-3) / 1e9, 2),
                 "frac": round(b64 / (cms64 * 1e-3) / 1e9 / HBM_PEAK_GBS, 5)},
    }

    cpu = None
    if not a.no_cpu_baseline:
        log("timing the CPU oracle")
        cpu = cpu_baseline(cloud, a.cpu_side)
        log(f"cpu baseline {cpu}")

    out = {
        "metric": METRIC,
        "value": round(N / (ms32_head * 1e-3) / 1e6, 3),
        "unit": "Mparticles/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms32_head, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32 values/weights/sums + fp64 geometry/solves",
        "data": "synthetic",
        "config": {"workload": "Taylor-Green round trip, 256x256 mesh (H=1/256), 1024x1024 jittered lattice "
                               "(h=H/4, jitter 0.3h, seed 2, permuted), 3 channels (u, v, p), weights rebuilt "
                               "every step", "particles": N, "nodes": nn, "channels": C,
                   "form": head_form},
        "forms": {"note": "stored: p2m_build_weights + p2m_project + m2p_interpolate; fused: p2m_project_fused "
                          "(no weights kept for the fast path's rows) + m2p_interpolate; the same bits",
                  "stored": stored, "fused": fused},
        "roofline": roof,
        "kernels": kernels,
        "round_trip_hbm": rt,
        "cached_weights": cached_rt,
        "kinematic_loop": None if kms32 is None else {"note": "one step of the kinematic projection loop, mixed form: M2P, the particles "
                                   "moved one midpoint step in the cellular flow of the box (a quarter cell), "
                                   "functions rebuilt, P2M; HIP graph replays, particles moving at every replay; "
                                   "build options tuned on the cloud after 24 steps of shear",
                           "ms_per_step": round(kms32, 5), "Mparticles_per_s": round(N / (kms32 * 1e-3) / 1e6, 3),
                           "failed_nodes_after": int(kdiag["failed_nodes"]),
                           "slow_nodes_after": int(kdiag["slow_nodes"]), "tuning": ktuning},
        "m2p_qcsf": None if qms32 is None else {
            "note": "M2P with the mesh's quadratically consistent functions (FP32 sums, FP64 edge table built "
                    "once per mesh), HIP graph replays; compare the linear M2P's phases_ms.m2p",
            "ms": round(qms32, 5), "Mparticles_per_s": round(N / (qms32 * 1e-3) / 1e6, 3),
            "table_ms_once": round(qsetup, 4)},
        "linear_fe": None if lms32 is None else {"note": "the same round trip with linear FE particle functions at interior nodes "
                              "(P2M_LINEAR: the node's particle triangle located, rings and solves skipped), "
                              "mixed form, weights rebuilt every step",
                      "ms_per_step": round(lms32, 5), "Mparticles_per_s": round(N / (lms32 * 1e-3) / 1e6, 3)},
        "periodic": None if pms32 is None else {
            "note": "the round trip in the paper's periodic box (-1, 1)^2 with k = pi (P2M_PERIODIC): the same "
                    "mesh and lattice sizes (256x256 cells, 1024x1024 jittered lattice, h=H/4, jitter 0.3h, "
                    "seed 2), mixed form, weights rebuilt every step; nodes whose search window reaches a box "
                    "side take the exact path",
            "ms_per_step": round(pms32, 5), "Mparticles_per_s": round(N / (pms32 * 1e-3) / 1e6, 3),
            "slow_nodes": int(pdiag["slow_nodes"]), "failed_nodes": int(pdiag["failed_nodes"]),
            "closure_nodes": int(pdiag["closure_nodes"]),
            "kinematic_step_ms": round(pkms32, 5),
            "kinematic_note": "one step of the periodic kinematic loop (M2P, p2m_advect_periodic: a quarter cell per "
                              "step in the periodic cellular flow, particles wrapped across the sides, rebuild, "
                              "P2M), HIP graph replays, particles moving at every replay; build options tuned on "
                              "the cloud after 24 steps of shear",
            "kinematic_tuning": pktuning,
            "kinematic_failed_nodes_after": int(pkdiag["failed_nodes"]),
            "kinematic_slow_nodes_after": int(pkdiag["slow_nodes"])},
        "launch": "eager" if (a.no_graph or graph_notes) else "HIP graph replay of the whole step",
        "launch_notes": graph_notes,
        "tuning": tuning,
        "cpu_baseline": cpu,
        "fp64": {"value": round(N / (ms64_head * 1e-3) / 1e6, 3), "ms_per_step": round(ms64_head, 5),
                 "round_trip_hbm": rt64, "phases_ms": {k: round(v, 5) for k, v in ph64.items()}},
        "phases_ms": {k: round(v, 5) for k, v in ph32.items()},
        "errors": result_err,
        "diag": diag,
        "step_stats": step_stats,
        "large": large,
    }
    print(json.dumps(out), flush=True)
    if a.copy_probe:
        n = a.copy_probe * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: {n * 4} bytes read, {n * 4} bytes written")
    return 0


if __name__ == "__main__":
    sys.exit(main())
