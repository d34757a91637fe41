"""The oracle's periodic box split into z-slabs with ghost planes, advanced
with one ghost exchange per Runge-Kutta stage.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``; the product path never
imports it.  It shares no code with the HIP library: every grid operation is
the oracle's own (``Grid.c2p``, ``Grid.rhs``), and the Runge-Kutta stages are
written out below as ``orc_step`` states them.

The paper decomposes the domain over MPI ranks and refills ghost zones before
each of INT, REC and DER within a substep (Sec. 3); its closing section
proposes a halo deep enough that one exchange per substep suffices, at the
price of redundant work in the ghost zones.  This module is that second
reading for a decomposition along z only: each slab keeps G ghost planes
below and above its nz_s interior planes, runs the whole stage on its
nz_s + 2G planes as if they were a periodic box of their own (the wrap only
touches ghost planes, whose results are thrown away), and after each stage
copies the 8 state arrays and the Newton guess W of the G planes next to each
of its edges into the neighbours' ghost planes.

The depth G follows from the stencils.  A stage's update of plane k reads the
face fluxes of the z faces k-1/2 and k+1/2 and the edge fields on k-1/2 and
k+1/2, which reconstruct primitives of planes k-3..k+3 (MP5: a face reads
three cells on either side, the edge fields reconstruct y- and x-face values
along z over the same span); primitives of plane m come from INT of the
z faces m-1/2 and m+1/2, i.e. of the face arrays at planes m-1 and m.  So
plane k depends on planes k-4..k+3 of the state: G = 4.  With HO the DER
differences read fluxes of six faces (k-5/2..k+5/2) and INT reads six faces
(m-5/2..m+5/2): primitives of planes k-5..k+5, face arrays k-8..k+7: G = 8.
The global timestep is the maximum over the slabs of each slab's maximum over
its interior planes, an exact operation, so the split run reproduces the
undivided one bit for bit.
"""
from __future__ import annotations

import numpy as np

from . import Grid


def ghost_depth(ho: bool) -> int:
    """Ghost planes per side for one exchange per stage: 4, or 8 with HO."""
    return 8 if ho else 4


class SlabRun:
    """A periodic nx x ny x nz box (unit cells of width L/n) advanced as
    z-slabs.  `bounds`: the interior plane counts of the slabs, bottom to top
    (they sum to nz, each >= G); `ghost`: G."""

    def __init__(self, n, bounds, ghost, L=(1.0, 1.0, 1.0), **grid_kw):
        nx, ny, nz = (n, n, n) if np.isscalar(n) else n
        if sum(bounds) != nz:
            raise ValueError("slab heights must sum to nz")
        if min(bounds) < ghost:
            raise ValueError("every slab needs at least G interior planes")
        self.n = (nx, ny, nz)
        self.G = ghost
        self.bounds = list(bounds)
        self.z0 = [int(sum(bounds[:s])) for s in range(len(bounds))]
        self.grid_kw = grid_kw
        dz = L[2] / nz
        self.dx = (L[0] / nx, L[1] / ny, dz)
        self.grids = [Grid(nx, ny, h + 2 * ghost, lx=L[0], ly=L[1], lz=dz * (h + 2 * ghost),
                           **grid_kw) for h in bounds]
        self.t = 0.0
        self.dt = 0.0

    # ------------------------------------------------------------ layout
    def _planes(self, s):
        """Global plane index of each of slab s's nz_s + 2G planes."""
        nz = self.n[2]
        return (np.arange(self.bounds[s] + 2 * self.G) + self.z0[s] - self.G) % nz

    def scatter(self, a):
        """Per-slab copies (ghosts included) of a global (nz, ny, nx) array."""
        return [np.ascontiguousarray(a[self._planes(s)]) for s in range(len(self.bounds))]

    def gather(self, parts):
        """The global array from the slabs' interior planes."""
        G = self.G
        return np.concatenate([p[G:G + h] for p, h in zip(parts, self.bounds)], axis=0)

    def set_state(self, cons, bf, W):
        """Global conserved arrays (5), face B (3) and W, split into slabs."""
        self.cons = [[c for c in self.scatter(a)] for a in cons]   # [var][slab]
        self.bf = [[b for b in self.scatter(a)] for a in bf]
        self.W = self.scatter(W)

    def state(self):
        return ([self.gather(v) for v in self.cons], [self.gather(v) for v in self.bf],
                self.gather(self.W))

    def _arrays(self, s):
        """The 9 exchanged arrays of slab s: D, Sx, Sy, Sz, U, the face B, W."""
        return [self.cons[n][s] for n in range(5)] + [self.bf[d][s] for d in range(3)] + \
            [self.W[s]]

    def exchange(self):
        """Ghost planes of every slab from its neighbours' edge interior
        planes (the periodic box: the bottom slab's lower neighbour is the top
        slab)."""
        G, ns = self.G, len(self.bounds)
        for s in range(ns):
            lo, hi = (s - 1) % ns, (s + 1) % ns
            h, hlo = self.bounds[s], self.bounds[lo]
            for a, alo, ahi in zip(self._arrays(s), self._arrays(lo), self._arrays(hi)):
                a[:G] = alo[hlo:hlo + G]          # lower neighbour's top G planes
                a[G + h:] = ahi[G:2 * G]          # upper neighbour's bottom G planes

    # ------------------------------------------------------------ stepping
    def _interior_amax(self, s, apm):
        """max over slab s's interior cells of sum_d max(a+, a-)_d / dx_d, in
        the order orc_rhs forms it."""
        G, h = self.G, self.bounds[s]
        acc = np.zeros_like(apm[0][G:G + h])
        for d in range(3):
            acc = acc + np.maximum(apm[2 * d][G:G + h], apm[2 * d + 1][G:G + h]) / self.dx[d]
        return float(acc.max())

    def step(self, nsteps=1):
        cfg = self.grids[0].cfg
        nstage = 2 if cfg.time_order == 2 else 3
        ns = len(self.bounds)
        for _ in range(nsteps):
            u0 = [[a.copy() for a in self._arrays(s)[:8]] for s in range(ns)]
            for st in range(1, nstage + 1):
                rhs, amax = [], []
                for s, g in enumerate(self.grids):
                    cons = [self.cons[n][s] for n in range(5)]
                    bf = [self.bf[d][s] for d in range(3)]
                    prim, _, _ = g.c2p(cons, bf, self.W[s])
                    r, _, det = g.rhs(prim, bf, detail=True)
                    rhs.append(r)
                    amax.append(self._interior_amax(s, det["apm"]))
                if st == 1:
                    self.dt = cfg.dt_fixed if cfg.dt_fixed > 0.0 else cfg.cfl / max(amax)
                dt = self.dt
                for s in range(ns):
                    for n, a in enumerate(self._arrays(s)[:8]):
                        a0, r = u0[s][n], rhs[s][n]
                        if st == 1:
                            a[...] = a0 + dt * r
                        elif nstage == 2:
                            a[...] = 0.5 * a0 + 0.5 * (a + dt * r)
                        elif st == 2:
                            a[...] = 0.75 * a0 + 0.25 * (a + dt * r)
                        else:
                            a[...] = (1.0 / 3.0) * a0 + (2.0 / 3.0) * (a + dt * r)
                self.exchange()
            self.t += self.dt
