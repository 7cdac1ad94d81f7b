"""Oracle (test infrastructure): MAC grid geometry.

Sec. 3 places pressure and all scalars at cell centres of a Cartesian grid
with velocities on faces (marker-and-cell). x and y are periodic; z is bounded
by walls. The paper uses equal spacing; z may here also be stretched, with
cell centres at face midpoints.
"""
from __future__ import annotations

import numpy as np


class Grid:
    """Cells [nz, ny, nx]; z faces zf[0..nz] (zf[0] = 0, zf[nz] = lz).

    h[k]  = zf[k+1] - zf[k]          cell height
    zc[k] = (zf[k] + zf[k+1]) / 2    cell centre
    g[k]  = zc[k] - zc[k-1]          centre gap across interior face k (k = 1..nz-1);
                                     g[0] and g[nz] are unused (walls) and set to nan
    vol[k] = dx * dy * h[k]          cell volume
    """

    def __init__(self, nx, ny, nz, lx, ly, lz, zf=None):
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.lx, self.ly, self.lz = float(lx), float(ly), float(lz)
        self.dx = self.lx / self.nx
        self.dy = self.ly / self.ny
        if zf is None:
            zf = np.arange(self.nz + 1, dtype=np.float64) * (self.lz / self.nz)
        self.zf = np.asarray(zf, dtype=np.float64).copy()
        assert self.zf.shape == (self.nz + 1,)
        self.h = np.diff(self.zf)
        self.zc = 0.5 * (self.zf[:-1] + self.zf[1:])
        self.g = np.full(self.nz + 1, np.nan)
        self.g[1:self.nz] = np.diff(self.zc)
        self.vol = self.dx * self.dy * self.h

    @classmethod
    def from_spec(cls, spec):
        return cls(spec.nx, spec.ny, spec.nz, spec.lx, spec.ly, spec.lz, spec.zf)

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def n(self):
        return self.nx * self.ny * self.nz

    def volume_field(self):
        """Cell volume broadcast to [nz, ny, nx]."""
        return np.broadcast_to(self.vol[:, None, None], self.shape)
