"""Seeded synthetic inputs shared by the GPU path's tests/bench and the oracle.

This module only draws particle clouds and evaluates closed-form test fields.
It holds none of the projection method's arithmetic (no shape functions, no
triangulation, no interpolation), so both sides of every parity check can take
their inputs from here without sharing method code.

The workloads stand in for the paper's analytic test cases (the Taylor-Green
vortex sheet of Sec. 3.2, eq. TG_vel and its pressure) on a bounded unit
square: particles on a cell-centred lattice of spacing h with i.i.d. uniform
jitter, a fixed mesh of spacing H with h = H/2 or H/4, and Taylor-Green /
quadratic fields.  Particle order is randomly permuted so the binning step has
real work to do.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Tuple

import numpy as np

__all__ = [
    "MeshSpec",
    "Cloud",
    "jittered_lattice",
    "tg_u",
    "tg_v",
    "tg_p",
    "quad_q",
    "config1",
    "config2",
    "config3",
    "config4",
    "config5",
    "small_cloud",
    "cluster_void_cloud",
    "conic_cloud",
    "hub_cloud",
    "CONFIGS",
]


@dataclasses.dataclass(frozen=True)
class MeshSpec:
    """Uniform fixed mesh: nodes (x0 + i*H, y0 + j*H), 0 <= i <= nx, 0 <= j <= ny.

    Node k = j*(nx+1) + i (x fastest).
    """

    nx: int
    ny: int
    H: float
    x0: float = 0.0
    y0: float = 0.0

    @property
    def n_nodes(self) -> int:
        return (self.nx + 1) * (self.ny + 1)

    def node_xy(self) -> np.ndarray:
        """Node coordinates, shape [n_nodes, 2], computed as x0 + i*H in FP64."""
        i = np.arange(self.nx + 1, dtype=np.float64)
        j = np.arange(self.ny + 1, dtype=np.float64)
        X = self.x0 + i[None, :] * self.H
        Y = self.y0 + j[:, None] * self.H
        X, Y = np.broadcast_arrays(X, Y)
        return np.stack([X.ravel(), Y.ravel()], axis=1)


@dataclasses.dataclass
class Cloud:
    """One particle set with its mesh and channel values (channels last)."""

    name: str
    mesh: MeshSpec
    h: float
    pos: np.ndarray  # f64 [N, 2], user (permuted) order
    vals: np.ndarray  # f64 [N, C]
    channels: Tuple[str, ...]
    extra: Dict[str, np.ndarray] = dataclasses.field(default_factory=dict)

    @property
    def N(self) -> int:
        return int(self.pos.shape[0])


# ---------------------------------------------------------------- fields ---
# Taylor-Green vortex sheet (Sec. 3.2, eq. TG_vel) with k = pi on the unit
# square, unit amplitude; pressure as p = -(cos 2kx + cos 2ky)/4 (the sign the
# benchmark configuration uses; projection is linear so the sign is immaterial).

def tg_u(x, y, a=1.0, k=math.pi):
    return a * np.sin(k * x) * np.cos(k * y)


def tg_v(x, y, a=1.0, k=math.pi):
    return -a * np.cos(k * x) * np.sin(k * y)


def tg_p(x, y, a=1.0, k=math.pi):
    return -(a * a) * (np.cos(2 * k * x) + np.cos(2 * k * y)) / 4.0


def tg_w(x, y, a=1.0, k=math.pi):
    """Vorticity dv/dx - du/dy of the field above."""
    return 2.0 * k * a * np.sin(k * x) * np.sin(k * y)


def quad_q(x, y):
    """A fixed full quadratic used as a test channel."""
    return 1.0 + 2.0 * x - 3.0 * y + 0.5 * x * x - 1.5 * x * y + 2.0 * y * y


# ---------------------------------------------------------------- clouds ---

def jittered_lattice(m: int, jitter: float, rng: np.random.Generator,
                     lo: float = 0.0, length: float = 1.0,
                     permute: bool = True) -> Tuple[np.ndarray, float]:
    """m x m cell-centred lattice in [lo, lo+length]^2 with uniform jitter.

    Particle (kx, ky) sits at lo + (k + 1/2) h with h = length/m, plus an
    i.i.d. U(-jitter*h, +jitter*h) offset per coordinate, drawn x then y per
    particle in row-major lattice order (kx fastest).  The particle order is
    then randomly permuted with the same generator.
    """
    h = length / m
    g = lo + (np.arange(m, dtype=np.float64) + 0.5) * h
    X, Y = np.meshgrid(g, g, indexing="xy")
    pos = np.stack([X.ravel(), Y.ravel()], axis=1)
    pos = pos + rng.uniform(-jitter * h, jitter * h, size=pos.shape)
    if permute:
        pos = pos[rng.permutation(pos.shape[0])]
    return np.ascontiguousarray(pos), h


def _fields(pos: np.ndarray, names: Tuple[str, ...], a=1.0, phase=(0.0, 0.0)) -> np.ndarray:
    x = pos[:, 0] - phase[0]
    y = pos[:, 1] - phase[1]
    table = {
        "u": lambda: tg_u(x, y, a),
        "v": lambda: tg_v(x, y, a),
        "p": lambda: tg_p(x, y, a),
        "w": lambda: tg_w(x, y, a),
        "q": lambda: quad_q(pos[:, 0], pos[:, 1]),
    }
    return np.ascontiguousarray(np.stack([table[c]() for c in names], axis=1))


def config1() -> Cloud:
    """Plain FP64: 32x32 cells, 64x64 lattice (h = H/2), jitter 0.25h, (u, v, q)."""
    rng = np.random.default_rng(1)
    pos, h = jittered_lattice(64, 0.25, rng)
    mesh = MeshSpec(32, 32, 1.0 / 32)
    ch = ("u", "v", "q")
    return Cloud("C1", mesh, h, pos, _fields(pos, ch), ch)


def config2() -> Cloud:
    """256x256 cells, 1024x1024 lattice (h = H/4), jitter 0.3h, (u, v, p)."""
    rng = np.random.default_rng(2)
    pos, h = jittered_lattice(1024, 0.30, rng)
    mesh = MeshSpec(256, 256, 1.0 / 256)
    ch = ("u", "v", "p")
    return Cloud("C2", mesh, h, pos, _fields(pos, ch), ch)


def config3(n_sets: int = 64, lo: int = 64, hi: int = 384) -> List[Cloud]:
    """64 independent sets; n_s = round(lo*(hi/lo)^U), (2 n_s)^2 lattice, h = H/2.

    Each set draws, from its own child of SeedSequence(3): U, then the
    amplitude a ~ U[0.5, 2], then the phase (px, py) ~ U[0,1)^2, then the
    lattice jitter (0.25h) and the order permutation.  Channels are the
    Taylor-Green (u, v, p, vorticity) with that amplitude and phase.
    """
    out = []
    ratio = hi / lo
    for s, child in enumerate(np.random.SeedSequence(3).spawn(n_sets)):
        rng = np.random.default_rng(child)
        u = rng.uniform(0.0, 1.0)
        n = int(round(lo * ratio ** u))
        amp = rng.uniform(0.5, 2.0)
        phase = tuple(rng.uniform(0.0, 1.0, size=2))
        pos, h = jittered_lattice(2 * n, 0.25, rng)
        mesh = MeshSpec(n, n, 1.0 / n)
        ch = ("u", "v", "p", "w")
        out.append(Cloud(f"C3[{s}]", mesh, h, pos, _fields(pos, ch, amp, phase), ch,
                         extra={"amp": np.array(amp), "phase": np.array(phase)}))
    return out


def config4() -> Cloud:
    """512x512 cells, 2048x2048 lattice (h = H/4), jitter 0.25h.

    The mesh input field f = TG(x-0.05, y+0.03) (u, v) and the target
    g = TG(x, y) are given at mesh nodes in ``extra``; ``vals`` holds f at the
    particles for convenience.
    """
    rng = np.random.default_rng(4)
    pos, h = jittered_lattice(2048, 0.25, rng)
    mesh = MeshSpec(512, 512, 1.0 / 512)
    ch = ("u", "v")
    nodes = mesh.node_xy()
    f_mesh = _fields(nodes, ch, 1.0, (0.05, -0.03))
    g_mesh = _fields(nodes, ch)
    return Cloud("C4", mesh, h, pos, _fields(pos, ch, 1.0, (0.05, -0.03)), ch,
                 extra={"f_mesh": f_mesh, "g_mesh": g_mesh})


def advect_euler(pos: np.ndarray, dt: float, steps: int, device: str = "cpu") -> np.ndarray:
    """Explicit Euler through the steady vortex u = (sin pi x cos pi y, -cos pi x sin pi y).

    Input generation only (FP64).  Runs on torch for speed; the velocity has
    zero normal component on the unit-square boundary, so particles stay in it.
    """
    import torch

    r = torch.from_numpy(np.ascontiguousarray(pos)).to(device=device, dtype=torch.float64)
    pi = math.pi
    for _ in range(steps):
        x = r[:, 0]
        y = r[:, 1]
        ux = torch.sin(pi * x) * torch.cos(pi * y)
        uy = -torch.cos(pi * x) * torch.sin(pi * y)
        r = r + dt * torch.stack([ux, uy], dim=1)
    return np.ascontiguousarray(r.cpu().numpy())


def config5(steps: int = 200, device: str = "cpu", m: int = 4096, n: int = 1024) -> Cloud:
    """1024x1024 cells, 4096x4096 lattice (h = H/4), jitter 0.25h, then 200
    explicit Euler steps r += 0.2 h u(r); (u, v, p) at the final positions."""
    rng = np.random.default_rng(5)
    pos, h = jittered_lattice(m, 0.25, rng)
    pos = advect_euler(pos, 0.2 * h, steps, device)
    mesh = MeshSpec(n, n, 1.0 / n)
    ch = ("u", "v", "p")
    return Cloud("C5", mesh, h, pos, _fields(pos, ch), ch)


def small_cloud(n: int, ratio: int, jitter: float, seed: int,
                channels: Tuple[str, ...] = ("u", "v", "q")) -> Cloud:
    """Scaled-down lattice workload: n x n cells, (ratio*n)^2 particles."""
    rng = np.random.default_rng(seed)
    pos, h = jittered_lattice(ratio * n, jitter, rng)
    mesh = MeshSpec(n, n, 1.0 / n)
    return Cloud(f"small{n}x{ratio}", mesh, h, pos, _fields(pos, channels), channels)


def periodic_tg_cloud(n: int, ratio: int, jitter: float, seed: int,
                      channels: Tuple[str, ...] = ("u", "v", "p")) -> Cloud:
    """The paper's periodic Taylor-Green box (Sec. 3.2): (-1, 1)^2, k = pi
    (period 2 = the box), n x n cells, a (ratio*n)^2 jittered lattice."""
    rng = np.random.default_rng(seed)
    pos, h = jittered_lattice(ratio * n, jitter, rng, lo=-1.0, length=2.0)
    mesh = MeshSpec(n, n, 2.0 / n, -1.0, -1.0)
    return Cloud(f"periodic{n}x{ratio}", mesh, h, pos, _fields(pos, channels), channels)


def cluster_void_cloud(n: int, N: int, seed: int,
                       channels: Tuple[str, ...] = ("u", "v", "q")) -> Cloud:
    """Conditioning stress input: Gaussian clusters plus a uniform background
    with two circular voids, all inside the unit square (not a benchmark)."""
    rng = np.random.default_rng(seed)
    n_bg = N // 2
    bg = rng.uniform(0.0, 1.0, size=(n_bg, 2))
    voids = [((0.3, 0.6), 0.12), ((0.7, 0.3), 0.08)]
    keep = np.ones(n_bg, bool)
    for (cx, cy), rad in voids:
        keep &= (bg[:, 0] - cx) ** 2 + (bg[:, 1] - cy) ** 2 > rad * rad
    bg = bg[keep]
    n_cl = N - bg.shape[0]
    centres = rng.uniform(0.15, 0.85, size=(6, 2))
    which = rng.integers(0, 6, size=n_cl)
    cl = centres[which] + rng.normal(0.0, 0.04, size=(n_cl, 2))
    cl = np.clip(cl, 1e-3, 1.0 - 1e-3)
    pos = np.concatenate([bg, cl])
    pos = np.ascontiguousarray(pos[rng.permutation(pos.shape[0])])
    mesh = MeshSpec(n, n, 1.0 / n)
    h = 1.0 / math.sqrt(N)
    return Cloud(f"cluster{n}", mesh, h, pos, _fields(pos, channels), channels)


def conic_cloud(n: int, n_pts: int, delta: float, seed: int,
                channels: Tuple[str, ...] = ("u", "v", "q")) -> Cloud:
    """Conditioning stress input (not a benchmark): n_pts particles on a
    rotated ellipse inside the unit square, at seeded random angles, each
    moved off the ellipse radially by a factor 1 + delta * U(-1, 1).  Every
    particle is a hull vertex, so every support of a node lies within
    relative distance delta of one conic: the moment systems of such
    supports are nearly rank-deficient, with condition numbers growing like
    1 / delta."""
    rng = np.random.default_rng(seed)
    t = np.sort(rng.uniform(0.0, 2.0 * math.pi, size=n_pts))
    r = 1.0 + delta * rng.uniform(-1.0, 1.0, size=n_pts)
    ex, ey = 0.41 * r * np.cos(t), 0.29 * r * np.sin(t)
    c, s = math.cos(0.35), math.sin(0.35)
    pos = np.stack([0.5 + c * ex - s * ey, 0.5 + s * ex + c * ey], 1)
    pos = np.ascontiguousarray(pos[rng.permutation(n_pts)])
    mesh = MeshSpec(n, n, 1.0 / n)
    h = 2.2 / n_pts
    return Cloud(f"conic{n}", mesh, h, pos, _fields(pos, channels), channels)


def hub_cloud(n: int, hubs: Tuple[Tuple[float, float, int], ...], seed: int,
              channels: Tuple[str, ...] = ("u", "v", "q")) -> Cloud:
    """Support-size stress input (not a benchmark): a jittered lattice
    (h = H/2) with "hub" particles of high Delaunay degree.  Each hub
    (cx, cy, degree) is one particle at (cx, cy) ringed by `degree`
    particles on a circle of radius 1.5 H (equal angles with a 2 % angular
    jitter and a 1e-3 relative radial jitter); the lattice is cleared within
    1.7 H of the hub.  Every mesh node inside the circle lies in a triangle
    of the hub's fan, so its support holds the hub's whole ring."""
    rng = np.random.default_rng(seed)
    pos, _ = jittered_lattice(2 * n, 0.25, rng, permute=False)
    H = 1.0 / n
    parts = []
    keep = np.ones(pos.shape[0], bool)
    for cx, cy, deg in hubs:
        keep &= (pos[:, 0] - cx) ** 2 + (pos[:, 1] - cy) ** 2 > (1.7 * H) ** 2
        t = (np.arange(deg) + 0.02 * rng.uniform(-1.0, 1.0, size=deg)) * (2.0 * math.pi / deg)
        r = 1.5 * H * (1.0 + 1e-3 * rng.uniform(-1.0, 1.0, size=deg))
        parts.append(np.array([[cx, cy]]))
        parts.append(np.stack([cx + r * np.cos(t), cy + r * np.sin(t)], 1))
    pos = np.concatenate([pos[keep]] + parts)
    pos = np.ascontiguousarray(pos[rng.permutation(pos.shape[0])])
    mesh = MeshSpec(n, n, H)
    return Cloud(f"hub{n}", mesh, H / 2, pos, _fields(pos, channels), channels)


def periodic_void_cloud(n: int, N: int, seed: int,
                        channels: Tuple[str, ...] = ("u", "v", "p")) -> Cloud:
    """Periodic stress input on the Taylor-Green box (-1, 1)^2 (not a
    benchmark): uniform particles with two circular voids centred on the box
    corner and on a side, so that both wrap across the sides, plus a Gaussian
    cluster that crosses the right side, wrapped into the box."""
    rng = np.random.default_rng(seed)
    pos = rng.uniform(-1.0, 1.0, size=(N, 2))
    keep = np.ones(N, bool)
    for (cx, cy), rad in (((-1.0, -1.0), 0.25), ((-1.0, 0.3), 0.18)):
        dx = pos[:, 0] - cx
        dy = pos[:, 1] - cy
        dx -= 2.0 * np.rint(dx / 2.0)
        dy -= 2.0 * np.rint(dy / 2.0)
        keep &= dx * dx + dy * dy > rad * rad
    cl = np.array([0.95, -0.4]) + rng.normal(0.0, 0.05, size=(N // 8, 2))
    cl = np.mod(cl + 1.0, 2.0) - 1.0
    pos = np.concatenate([pos[keep], cl])
    pos = np.ascontiguousarray(pos[rng.permutation(pos.shape[0])])
    mesh = MeshSpec(n, n, 2.0 / n, -1.0, -1.0)
    h = 2.0 / math.sqrt(pos.shape[0])
    return Cloud(f"periodic_void{n}", mesh, h, pos, _fields(pos, channels), channels)


CONFIGS = {
    "C1": config1,
    "C2": config2,
    "C3": config3,
    "C4": config4,
    "C5": config5,
}
