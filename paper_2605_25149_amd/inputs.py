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
  * batch_instances(count, seed):       the independent 2-D problems of a batch: side
        ~ {64, 96, 128, 192, 256}, N ~ U{8..64}, V = harmonic (omega2 ~ U[50,150],
        centre ~ U[0.3,0.7]^2) minus 4 Gaussian wells (depths U[2,8], widths
        U[0.05,0.15], centres U[0.1,0.9]^2), drawn in that order per instance
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


def harmonic_wells(n, omega2, centre, depths, widths, centres, L=(1.0, 1.0)):
    """1/2 omega2 |x - c|^2 - sum_k d_k exp(-|x - c_k|^2 / (2 w_k^2))."""
    dim = len(n)
    xs = grid_coords(n, L)
    V = 0.5 * omega2 * sum((xs[a] - centre[a]) ** 2 for a in range(dim))
    for k in range(len(depths)):
        r2 = sum((xs[a] - centres[k][a]) ** 2 for a in range(dim))
        V = V - depths[k] * np.exp(-r2 / (2.0 * widths[k] ** 2))
    return V


def batch_instances(count, seed=0, sides=(64, 96, 128, 192, 256), nrange=(8, 64)):
    """Descriptions of `count` independent 2-D problems: dicts with n, N, V and sigma.

    sigma = max(0, 1 - min V) makes V + sigma >= 1, so H_sigma is positive definite."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        side = int(rng.choice(sides))
        N = int(rng.integers(nrange[0], nrange[1] + 1))
        omega2 = rng.uniform(50.0, 150.0)
        centre = rng.uniform(0.3, 0.7, 2)
        depths = rng.uniform(2.0, 8.0, 4)
        widths = rng.uniform(0.05, 0.15, 4)
        centres = rng.uniform(0.1, 0.9, (4, 2))
        n = (side, side)
        V = harmonic_wells(n, omega2, centre, depths, widths, centres)
        out.append({"n": n, "N": N, "V": V, "sigma": max(0.0, 1.0 - float(V.min()))})
    return out
