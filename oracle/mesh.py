"""Fixed uniform mesh of the oracle (test infrastructure only).

The paper's fixed mesh has spacing H (Sec. 1, Fig. idea).  The oracle works on
a bounded rectangle of (nx+1) x (ny+1) nodes at (x0 + i*H, y0 + j*H), node id
k = j*(nx+1) + i.  (The paper's runs are periodic; the bounded rectangle is the
default reading here, and ``periodic`` forms the periodic box on the same
node layout.)
"""
from __future__ import annotations

import dataclasses

import numpy as np


class DomainError(ValueError):
    """A particle lies outside the mesh rectangle."""


@dataclasses.dataclass(frozen=True)
class Mesh:
    nx: int
    ny: int
    H: float
    x0: float = 0.0
    y0: float = 0.0

    @classmethod
    def from_spec(cls, spec) -> "Mesh":
        return cls(int(spec.nx), int(spec.ny), float(spec.H), float(spec.x0), float(spec.y0))

    @property
    def n_nodes(self) -> int:
        return (self.nx + 1) * (self.ny + 1)

    def nodes(self) -> np.ndarray:
        """All node positions [n_nodes, 2]; x = x0 + i*H evaluated in FP64."""
        i = np.arange(self.nx + 1, dtype=np.float64)
        j = np.arange(self.ny + 1, dtype=np.float64)
        X = np.broadcast_to(self.x0 + i[None, :] * self.H, (self.ny + 1, self.nx + 1))
        Y = np.broadcast_to(self.y0 + j[:, None] * self.H, (self.ny + 1, self.nx + 1))
        return np.stack([X.ravel(), Y.ravel()], axis=1)

    def node_ij(self, k):
        k = np.asarray(k)
        return k % (self.nx + 1), k // (self.nx + 1)

    def on_boundary_ring(self, k) -> np.ndarray:
        i, j = self.node_ij(k)
        return (i == 0) | (j == 0) | (i == self.nx) | (j == self.ny)

    def check_inside(self, pos: np.ndarray) -> None:
        x1 = self.x0 + self.nx * self.H
        y1 = self.y0 + self.ny * self.H
        if not np.all(np.isfinite(pos)):
            raise DomainError("non-finite particle position")
        bad = (pos[:, 0] < self.x0) | (pos[:, 0] > x1) | (pos[:, 1] < self.y0) | (pos[:, 1] > y1)
        if np.any(bad):
            raise DomainError(f"{int(bad.sum())} particle(s) outside the mesh rectangle")
