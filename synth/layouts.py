"""Seeded particle layouts, sources and receivers shaped like the paper's workloads.

The paper (Section 6) places identical inclusions at random in the middle
layer with random orientations, keeping them well separated.  Here the
placement is sequential rejection: draw a candidate x, then y, uniformly in
the strip and accept it when it is at least ``min_sep`` away from every
centre accepted so far.  Rotations are drawn afterwards, uniform in [0, 2pi).

Nothing in this module evaluates any part of the scattering method.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np


def _grid_ok(grid, cell, x, y, min_sep, xy):
    cx = int(math.floor(x / cell))
    cy = int(math.floor(y / cell))
    m2 = min_sep * min_sep
    for gx in range(cx - 1, cx + 2):
        for gy in range(cy - 1, cy + 2):
            for j in grid.get((gx, gy), ()):
                dx = xy[j][0] - x
                dy = xy[j][1] - y
                if dx * dx + dy * dy < m2:
                    return False
    return True


def rejection_layout(n: int, x_range, y_range, min_sep: float, seed: int,
                     max_draws: Optional[int] = None):
    """Sequential rejection placement of ``n`` centres in a rectangle.

    Returns ``(xy, rot)``: float64 arrays of shape (n, 2) and (n,).
    Raises RuntimeError when ``max_draws`` candidates did not give n centres.
    """
    rng = np.random.default_rng(seed)
    x0, x1 = map(float, x_range)
    y0, y1 = map(float, y_range)
    cell = float(min_sep)
    grid: dict = {}
    xy: list = []
    limit = max_draws if max_draws is not None else 200 * n + 1000
    draws = 0
    while len(xy) < n:
        if draws >= limit:
            raise RuntimeError(f"rejection placement stalled at {len(xy)} of {n}")
        draws += 1
        x = rng.uniform(x0, x1)
        y = rng.uniform(y0, y1)
        if _grid_ok(grid, cell, x, y, min_sep, xy):
            key = (int(math.floor(x / cell)), int(math.floor(y / cell)))
            grid.setdefault(key, []).append(len(xy))
            xy.append((x, y))
    rot = rng.uniform(0.0, 2.0 * math.pi, size=n)
    return np.asarray(xy, dtype=np.float64), rot.astype(np.float64)


def perturbed_layout(xy, rot, sigma: float, seed: int, min_sep: float,
                     y_range=None):
    """Perturb centres and rotations by N(0, sigma^2), one particle at a time.

    A centre move that would break ``min_sep`` (or leave ``y_range``) is
    rejected and the particle keeps its old centre.
    """
    rng = np.random.default_rng(seed)
    xy = np.array(xy, dtype=np.float64, copy=True)
    rot = np.array(rot, dtype=np.float64, copy=True)
    n = xy.shape[0]
    cell = float(min_sep)
    grid: dict = {}
    for j in range(n):
        key = (int(math.floor(xy[j, 0] / cell)), int(math.floor(xy[j, 1] / cell)))
        grid.setdefault(key, []).append(j)
    m2 = min_sep * min_sep
    for j in range(n):
        dx, dy = rng.normal(0.0, sigma, size=2)
        nx, ny = xy[j, 0] + dx, xy[j, 1] + dy
        ok = True
        if y_range is not None and not (y_range[0] <= ny <= y_range[1]):
            ok = False
        if ok:
            cx, cy = int(math.floor(nx / cell)), int(math.floor(ny / cell))
            for gx in range(cx - 1, cx + 2):
                for gy in range(cy - 1, cy + 2):
                    for i in grid.get((gx, gy), ()):
                        if i == j:
                            continue
                        ex = xy[i, 0] - nx
                        ey = xy[i, 1] - ny
                        if ex * ex + ey * ey < m2:
                            ok = False
        if ok:
            old = (int(math.floor(xy[j, 0] / cell)), int(math.floor(xy[j, 1] / cell)))
            grid[old].remove(j)
            xy[j, 0], xy[j, 1] = nx, ny
            grid.setdefault((int(math.floor(nx / cell)), int(math.floor(ny / cell))), []).append(j)
    rot = rot + rng.normal(0.0, sigma, size=n)
    return xy, rot


def receivers(n: int, x_range, y_range, centres, seed: int, particle_excl: float,
              source=None, source_excl: float = 0.05):
    """Uniform receivers in a rectangle, rejecting points near particles/source."""
    rng = np.random.default_rng(seed)
    centres = np.asarray(centres, dtype=np.float64)
    out = []
    cell = max(particle_excl, 1e-3)
    grid: dict = {}
    for j, (x, y) in enumerate(centres):
        grid.setdefault((int(math.floor(x / cell)), int(math.floor(y / cell))), []).append(j)
    e2 = particle_excl * particle_excl
    while len(out) < n:
        x = rng.uniform(*x_range)
        y = rng.uniform(*y_range)
        ok = True
        cx, cy = int(math.floor(x / cell)), int(math.floor(y / cell))
        for gx in range(cx - 1, cx + 2):
            for gy in range(cy - 1, cy + 2):
                for j in grid.get((gx, gy), ()):
                    ex = centres[j, 0] - x
                    ey = centres[j, 1] - y
                    if ex * ex + ey * ey < e2:
                        ok = False
        if ok and source is not None:
            if (x - source[0]) ** 2 + (y - source[1]) ** 2 < source_excl ** 2:
                ok = False
        if ok:
            out.append((x, y))
    return np.asarray(out, dtype=np.float64)


@dataclasses.dataclass
class Workload:
    """One synthetic problem: layers, particle type, geometry, sources, contour."""

    name: str
    k1: complex
    k2: complex
    k3: complex
    d: float
    kp: complex
    shape: str                 # "disk" or "star"
    shape_params: tuple        # disk: (R,); star: (a1, a2, a3)
    r_enclose: float
    p: int
    xy: np.ndarray             # (N, 2) float64
    rot: np.ndarray            # (N,) float64, CCW radians
    src: np.ndarray            # (n_rhs, 2) float64 point sources in layer 1
    n_nodes: int
    b: float
    t_max: float
    tol: float
    n_bdry: int = 256

    @property
    def n(self) -> int:
        return int(self.xy.shape[0])

    @property
    def P(self) -> int:
        return 2 * self.p + 1


# Workload recipes.  Layers k = (6, 9, 12), stars r(t) = 0.25 + 0.05 cos 5t
# (enclosing radius 0.3), particle wavenumber 15, min centre separation 0.75.
CONFIGS = {
    # 16 Mie disks, p = 8, d = 8, 256 contour nodes.
    "c1": dict(n=16, shape="disk", shape_params=(0.25,), r_enclose=0.25, p=8,
               x_range=(-4.0, 4.0), y_range=(-7.0, -1.0), d=8.0, seed=0,
               n_nodes=256, b=0.2, tol=1e-10),
    # 1000 stars, p = 12, 200 x 18 strip, d = 20, 512 nodes.
    "c2": dict(n=1000, shape="star", shape_params=(0.25, 0.05, 5), r_enclose=0.3,
               p=12, x_range=(-100.0, 100.0), y_range=(-19.0, -1.0), d=20.0,
               seed=1, n_nodes=512, b=0.01, tol=1e-10),
    # 5000 stars, p = 16, 400 x 38 strip, d = 40, 1024 nodes.
    "c3": dict(n=5000, shape="star", shape_params=(0.25, 0.05, 5), r_enclose=0.3,
               p=16, x_range=(-200.0, 200.0), y_range=(-39.0, -1.0), d=40.0,
               seed=2, n_nodes=1024, b=0.005, tol=1e-6),
    # 2000 stars, p = 12 (batched-source geometry).
    "c4": dict(n=2000, shape="star", shape_params=(0.25, 0.05, 5), r_enclose=0.3,
               p=12, x_range=(-100.0, 100.0), y_range=(-19.0, -1.0), d=20.0,
               seed=3, n_nodes=512, b=0.01, tol=1e-10),
    # Small parity cases at the particle density of c2/c3 (about 0.3 per unit
    # area): several 64-wide tiles plus a ragged tail.
    "s200p16": dict(n=200, shape="star", shape_params=(0.25, 0.05, 5), r_enclose=0.3,
                    p=16, x_range=(-40.0, 40.0), y_range=(-9.0, -1.0), d=10.0,
                    seed=11, n_nodes=256, b=0.025, tol=1e-10),
    "s150p12": dict(n=150, shape="star", shape_params=(0.25, 0.05, 5), r_enclose=0.3,
                    p=12, x_range=(-31.0, 31.0), y_range=(-9.0, -1.0), d=10.0,
                    seed=12, n_nodes=256, b=0.03, tol=1e-10),
    # Largest serving size: 20000 stars, p = 16, strip of height d - 2 = 38
    # and width N / (0.3 (d - 2)) = 1754 (the FMM regime).
    "c5max": dict(n=20000, shape="star", shape_params=(0.25, 0.05, 5), r_enclose=0.3,
                  p=16, x_range=(-877.0, 877.0), y_range=(-39.0, -1.0), d=40.0,
                  seed=21, n_nodes=1024, b=0.001, tol=1e-6),
    "s70p8": dict(n=70, shape="disk", shape_params=(0.25,), r_enclose=0.25,
                  p=8, x_range=(-30.0, 30.0), y_range=(-5.0, -1.0), d=6.0,
                  seed=13, n_nodes=256, b=0.03, tol=1e-10),
}


def make_workload(name: str, n_rhs: int = 1, src_seed: Optional[int] = None,
                  n: Optional[int] = None, cut: Optional[int] = None) -> Workload:
    """Build a named workload.  ``n`` overrides the particle count (same strip);
    ``cut`` keeps only the ``cut`` particles of the full layout nearest to
    x = 0 (smallest |x|, ties by index, original order): a window of the strip
    at the recipe's density."""
    c = dict(CONFIGS[name])
    nn = int(n) if n is not None else c["n"]
    xy, rot = rejection_layout(nn, c["x_range"], c["y_range"], 0.75, c["seed"])
    if cut is not None:
        keep = np.sort(np.lexsort((np.arange(xy.shape[0]), np.abs(xy[:, 0])))[:int(cut)])
        xy, rot = xy[keep], rot[keep]
    if n_rhs == 1 and src_seed is None:
        src = np.array([[0.0, 2.0]])
    else:
        rng = np.random.default_rng(src_seed if src_seed is not None else 4)
        src = np.stack([rng.uniform(c["x_range"][0], c["x_range"][1], n_rhs),
                        rng.uniform(1.0, 3.0, n_rhs)], axis=1)
    return Workload(name=name, k1=6.0, k2=9.0, k3=12.0, d=c["d"], kp=15.0,
                    shape=c["shape"], shape_params=c["shape_params"],
                    r_enclose=c["r_enclose"], p=c["p"], xy=xy, rot=rot, src=src,
                    n_nodes=c["n_nodes"], b=c["b"], t_max=32.0, tol=c["tol"])
