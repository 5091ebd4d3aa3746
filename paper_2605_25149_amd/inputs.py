"""Seeded synthetic inputs shared by the HIP path's tests/benchmark and the oracle.

This module holds none of the method's arithmetic: it only draws potentials and
starting blocks from a seed.  Grids are interior points of the box
[0, L_0] x ... with spacing h_k = L_k / (n_k + 1); a grid function is stored
with x fastest (index i + n_0*(j + n_1*k)); a block of N grid functions is
column-major (Ng rows, each column contiguous).

Workload families (the paper's own experiments use finite elements and
external eigensolvers; these synthetic families stand in for them):
  * harmonic(n, dim, omega2, centre):  V = 1/2 omega2 |x - c|^2 (separable)
  * gaussian_wells(n, dim, seed):       V = -sum_k d_k exp(-|x-c_k|^2 / (2 w_k^2)),
        8 wells, depths d ~ U[5,20], widths w ~ U[0.05,0.15], centres ~ U[0,1]^dim,
        drawn in that order from numpy default_rng(seed)
  * random_block(ng, N, seed):          i.i.d. N(0,1) entries, column after column,
        from numpy default_rng(seed) (not orthonormal)
"""
from __future__ import annotations

import numpy as np


def grid_coords(n, L=(1.0, 1.0, 1.0)):
    """Coordinates of the interior points, one (Ng,) array per axis, x fastest."""
    dim = len(n)
    axes = [(np.arange(n[k]) + 1.0) * (L[k] / (n[k] + 1)) for k in range(dim)]
    mesh = np.meshgrid(*axes[::-1], indexing="ij")  # slowest axis first
    return [m.reshape(-1) for m in mesh[::-1]]


def harmonic(n, omega2=100.0, centre=None, L=(1.0, 1.0, 1.0)):
    dim = len(n)
    if centre is None:
        centre = [0.5 * L[k] for k in range(dim)]
    xs = grid_coords(n, L)
    r2 = sum((xs[k] - centre[k]) ** 2 for k in range(dim))
    return 0.5 * omega2 * r2


def well_params(dim, seed, nwells=8, depth=(5.0, 20.0), width=(0.05, 0.15)):
    rng = np.random.default_rng(seed)
    d = rng.uniform(depth[0], depth[1], nwells)
    w = rng.uniform(width[0], width[1], nwells)
    c = rng.uniform(0.0, 1.0, (nwells, dim))
    return d, w, c


def gaussian_wells(n, seed=0, nwells=8, depth=(5.0, 20.0), width=(0.05, 0.15),
                   L=(1.0, 1.0, 1.0)):
    dim = len(n)
    d, w, c = well_params(dim, seed, nwells, depth, width)
    xs = grid_coords(n, L)
    V = np.zeros_like(xs[0])
    for k in range(nwells):
        r2 = sum((xs[a] - c[k, a] * L[a]) ** 2 for a in range(dim))
        V -= d[k] * np.exp(-r2 / (2.0 * w[k] ** 2))
    return V


def random_block(ng, N, seed=1):
    """(ng, N) column-major block with i.i.d. standard normal entries."""
    rng = np.random.default_rng(seed)
    return np.asfortranarray(rng.standard_normal((N, ng)).T)
