"""Kinematic transport of the particles, and one step of the kinematic
projection loop (oracle; test infrastructure only).

The paper's kinematic tests (Secs. 3.1-3.2: a slotted disk and a
Taylor-Green field carried by a prescribed velocity) move the particles with
a known velocity and rebuild the particle functions at every step, since the
particles have moved.  The reading taken for a bounded box: the cellular
flow of streamfunction

    psi(x, y) = A sin(pi (x - x0) / Lx) sin(pi (y - y0) / Ly),
    u = d psi / d y,  v = - d psi / d x,

whose normal velocity vanishes on the box boundary (Lx = nx H, Ly = ny H),
so that particles stay in the box (a rotation would carry the corners out).
One time step is the explicit midpoint rule

    r* = r + dt/2 u(r),   r' = r + dt u(r*),

followed by clamping into the box (the midpoint rule can overshoot a wall by
O(dt^3)).  One step of the loop, in this order:

    alpha_mu = M2P(alpha_i, r)            eq. (m2p)
    r        = midpoint step of r
    psi_mu   rebuilt at the new r         App. B
    alpha_i  = P2M(alpha_mu, r)           eq. (p2m)

In the periodic box of the paper's runs (``periodic=True``) the flow is

    psi(x, y) = A cos(2 pi (x - x0) / Lx) cos(2 pi (y - y0) / Ly),

periodic on the box, with cells centred on the box corners and centre, so
that the flow crosses the box sides; a moved particle is wrapped back into
[x0, x0 + Lx) x [y0, y0 + Ly) (x - Lx floor((x - x0) / Lx), one rounding; a
result that rounds onto the far side is taken as the near one); the loop
rebuilds the periodic functions.

All arithmetic is FP64.
"""
from __future__ import annotations

import numpy as np

from .m2p import m2p
from .mesh import Mesh
from .qcsf import P2MOracle


def velocity(mesh: Mesh, amp: float, pos, periodic: bool = False):
    """u(r) of the cellular flow, [N, 2]."""
    pos = np.asarray(pos, dtype=np.float64)
    lx, ly = mesh.nx * mesh.H, mesh.ny * mesh.H
    if periodic:
        ax = 2.0 * np.pi * (pos[:, 0] - mesh.x0) / lx
        ay = 2.0 * np.pi * (pos[:, 1] - mesh.y0) / ly
        u = -amp * (2.0 * np.pi / ly) * np.cos(ax) * np.sin(ay)
        v = amp * (2.0 * np.pi / lx) * np.sin(ax) * np.cos(ay)
        return np.stack([u, v], axis=1)
    ax = np.pi * (pos[:, 0] - mesh.x0) / lx
    ay = np.pi * (pos[:, 1] - mesh.y0) / ly
    u = amp * (np.pi / ly) * np.sin(ax) * np.cos(ay)
    v = -amp * (np.pi / lx) * np.cos(ax) * np.sin(ay)
    return np.stack([u, v], axis=1)


def wrap(mesh: Mesh, pos):
    """Positions moved by whole periods into [x0, x0+Lx) x [y0, y0+Ly)."""
    pos = np.array(pos, dtype=np.float64)
    for d, (o, L) in enumerate(((mesh.x0, mesh.nx * mesh.H), (mesh.y0, mesh.ny * mesh.H))):
        x = pos[:, d]
        x = x - np.floor((x - o) / L) * L
        pos[:, d] = np.where(x >= o + L, o, x)
    return pos


def midpoint_step(mesh: Mesh, amp: float, dt: float, pos, periodic: bool = False):
    """One explicit midpoint step of every particle, clamped into the box
    (wrapped into it in the periodic box)."""
    pos = np.asarray(pos, dtype=np.float64)
    mid = pos + 0.5 * dt * velocity(mesh, amp, pos, periodic)
    new = pos + dt * velocity(mesh, amp, mid, periodic)
    if periodic:
        return wrap(mesh, new)
    x1, y1 = mesh.x0 + mesh.nx * mesh.H, mesh.y0 + mesh.ny * mesh.H
    new[:, 0] = np.clip(new[:, 0], mesh.x0, x1)
    new[:, 1] = np.clip(new[:, 1], mesh.y0, y1)
    return new


def kinematic_step(mesh: Mesh, h: float, amp: float, dt: float, pos, mesh_vals, periodic: bool = False):
    """One loop step; returns (new positions, new mesh values)."""
    vals = m2p(mesh, mesh_vals, pos)
    pos = midpoint_step(mesh, amp, dt, pos, periodic)
    if periodic:
        from .periodic import PeriodicP2MOracle
        return pos, PeriodicP2MOracle(pos, mesh, h).project(vals)
    return pos, P2MOracle(pos, mesh, h).project(vals)
