"""Seeded synthetic cloth scenes.

This module only builds input data: grid meshes, rest and initial positions,
pin masks, obstacle descriptions and the numeric settings of each workload.
It holds none of the solver's arithmetic, so both the HIP library (through its
Python binding) and the CPU oracle may take their inputs from here.

Scenes stand in for the paper's garment, drape and blender workloads
(Table 1, the drape-on-a-sphere and cloth-blender rows), which ship no assets:
square grids of 1 m side, alternating diagonals, in the x-z plane with
gravity along -y.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

SPHERE = 0
CYLINDER = 1


@dataclass
class Obstacle:
    kind: int                      # SPHERE or CYLINDER
    center: tuple
    radius: float
    axis: tuple = (1.0, 0.0, 0.0)  # cylinder axis (unit)
    half_length: float = 0.0       # cylinder half length
    omega: float = 0.0             # spin about the axis, rad/s (recorded only)


@dataclass
class Scene:
    name: str
    n_side: int
    tris: np.ndarray               # (T,3) int32, consistently oriented
    rest: np.ndarray               # (N,3) float32 rest shape
    x0: np.ndarray                 # (N,3) float32 initial positions
    v0: np.ndarray                 # (N,3) float32 initial velocities
    pinned: np.ndarray             # (N,) uint8
    obstacles: List[Obstacle]
    dt: float
    gravity: tuple
    steps: int
    r: int
    iters_outer: int
    iters_inner: int
    self_contact: bool
    d_hat: float
    density: float = 0.3           # kg / m^2
    k_stretch: float = 160.0
    k_bend: float = 3e-4
    seed: int = 0
    precision: str = "fp32"        # "fp32" or "mixed"

    @property
    def nv(self) -> int:
        return int(self.rest.shape[0])

    @property
    def nt(self) -> int:
        return int(self.tris.shape[0])


def grid_triangles(n: int) -> np.ndarray:
    """Triangles of an n x n vertex grid; vertex (i, j) has index i*n + j.

    The quad diagonal alternates with the parity of i + j, and every
    triangle's normal points along +y for the x-z layout used here.
    """
    i, j = np.meshgrid(np.arange(n - 1), np.arange(n - 1), indexing="ij")
    i = i.ravel()
    j = j.ravel()
    v00 = i * n + j
    v01 = v00 + 1
    v10 = v00 + n
    v11 = v10 + 1
    even = ((i + j) % 2) == 0
    t1 = np.where(even[:, None], np.stack([v00, v11, v01], 1), np.stack([v00, v10, v01], 1))
    t2 = np.where(even[:, None], np.stack([v00, v10, v11], 1), np.stack([v01, v10, v11], 1))
    tris = np.empty((2 * len(i), 3), dtype=np.int64)
    tris[0::2] = t1
    tris[1::2] = t2
    return tris.astype(np.int32)


def grid_positions(n: int, side: float, height: float = 0.0) -> np.ndarray:
    e = side / (n - 1)
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    pos = np.zeros((n * n, 3), dtype=np.float64)
    pos[:, 0] = (j * e).ravel()
    pos[:, 1] = height
    pos[:, 2] = (i * e).ravel()
    return pos


def sinusoid_heights(xz: np.ndarray, rng: np.random.Generator, count: int = 8,
                     amp: float = 1.25e-3) -> np.ndarray:
    """Sum of `count` plane waves with random wave vectors (|k| in [2pi, 8pi]/m)."""
    h = np.zeros(xz.shape[0])
    for _ in range(count):
        kmag = rng.uniform(2 * math.pi, 8 * math.pi)
        ang = rng.uniform(0, 2 * math.pi)
        phi = rng.uniform(0, 2 * math.pi)
        k = kmag * np.array([math.cos(ang), math.sin(ang)])
        h += amp * np.sin(xz @ k + phi)
    return h


def mean_edge_length(pos: np.ndarray, tris: np.ndarray) -> float:
    e = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]])
    e = np.unique(np.sort(e, axis=1), axis=0)
    return float(np.linalg.norm(pos[e[:, 0]] - pos[e[:, 1]], axis=1).mean())


def hanging_cloth(n: int = 32, seed: int = 0, r: int = 16, steps: int = 10,
                  iters: int = 20, jitter: float = 0.05) -> Scene:
    """Small square cloth pinned at the two corners of grid row 0, starting
    horizontal and swinging down under gravity; in-plane jitter of +/- jitter
    times the edge length on every vertex (rest shape = initial shape)."""
    rng = np.random.default_rng(seed)
    side = 1.0
    e = side / (n - 1)
    pos = grid_positions(n, side)
    pos[:, 0] += rng.uniform(-jitter * e, jitter * e, n * n)
    pos[:, 2] += rng.uniform(-jitter * e, jitter * e, n * n)
    pinned = np.zeros(n * n, np.uint8)
    pinned[0] = 1
    pinned[n - 1] = 1
    rest = pos.astype(np.float32)
    return Scene(name=f"hang{n}", n_side=n, tris=grid_triangles(n), rest=rest, x0=rest.copy(),
                 v0=np.zeros_like(rest), pinned=pinned, obstacles=[], dt=1.0 / 200,
                 gravity=(0.0, -9.8, 0.0), steps=steps, r=r, iters_outer=1, iters_inner=iters,
                 self_contact=False, d_hat=1e-3, seed=seed)


def drop_cloth(n: int, seed: int, obstacle: str, r: int, steps: int,
               iters_outer: int = 3, iters_inner: int = 10, side: float = 1.0,
               drop: float = 0.3, d_hat: Optional[float] = None,
               precision: str = "fp32", radius_scale: float = 1.0) -> Scene:
    """Flat-rest cloth, perturbed by eight seeded sinusoids (|h| <= 1 cm at
    1 m side), whose centre starts `drop` above the top of a sphere or of a
    horizontal cylinder (axis along x) centred under it."""
    rng = np.random.default_rng(seed)
    cx = cz = side / 2
    if obstacle == "sphere":
        R = 0.25 * side * radius_scale
        top = R
        obs = [Obstacle(SPHERE, (cx, 0.0, cz), R)]
    elif obstacle == "cylinder":
        R = 0.2 * side * radius_scale
        top = R
        obs = [Obstacle(CYLINDER, (cx, 0.0, cz), R, axis=(1.0, 0.0, 0.0),
                        half_length=0.75 * side, omega=2.0)]
    else:
        raise ValueError(obstacle)
    y0 = top + drop * side
    rest64 = grid_positions(n, side, y0)
    h = sinusoid_heights(rest64[:, [0, 2]], rng, amp=1.25e-3 * side)
    x0 = rest64.copy()
    x0[:, 1] += h
    tris = grid_triangles(n)
    if d_hat is None:
        d_hat = min(1e-3, 0.4 * mean_edge_length(rest64, tris))
    rest = rest64.astype(np.float32)
    return Scene(name=f"{obstacle}{n}", n_side=n, tris=tris, rest=rest,
                 x0=x0.astype(np.float32), v0=np.zeros_like(rest),
                 pinned=np.zeros(n * n, np.uint8), obstacles=obs, dt=1.0 / 200,
                 gravity=(0.0, -9.8, 0.0), steps=steps, r=r, iters_outer=iters_outer,
                 iters_inner=iters_inner, self_contact=True, d_hat=float(d_hat), seed=seed,
                 precision=precision)


def draped_state(sc: Scene, gap_scale: float = 0.5, seed: int = 0) -> np.ndarray:
    """A seeded draped configuration of a cylinder-drop scene: the rest grid
    laid over the cylinder's top along arc length (the z coordinate measured
    from the axis becomes the angle over a circle of radius R + gap_scale
    d_hat) and hanging straight down beyond the two tangent lines, lifted
    radially by the absolute value of a seeded sum of eight sinusoids
    (|h| <= 1 cm x side).  Arc length is kept along z, so the sheet starts
    nearly unstretched and touching the obstacle's contact band over the arc.
    Input data only: it holds no solver arithmetic."""
    ob = sc.obstacles[0]
    if ob.kind != CYLINDER:
        raise ValueError("draped_state needs a cylinder scene")
    rng = np.random.default_rng(seed)
    cy, cz = ob.center[1], ob.center[2]
    Ro = ob.radius + gap_scale * sc.d_hat
    rest = sc.rest.astype(np.float64)
    side = float(rest[:, 2].max() - rest[:, 2].min())
    h = np.abs(sinusoid_heights(rest[:, [0, 2]], rng, amp=1.25e-3 * side))
    s = rest[:, 2] - cz                      # arc length from the top line
    half = 0.5 * math.pi * Ro
    th = np.clip(s / Ro, -0.5 * math.pi, 0.5 * math.pi)
    x = np.empty_like(rest)
    x[:, 0] = rest[:, 0]
    on = np.abs(s) <= half
    # over the arc: radius Ro + h at angle th from the top
    x[on, 1] = cy + (Ro + h[on]) * np.cos(th[on])
    x[on, 2] = cz + (Ro + h[on]) * np.sin(th[on])
    # hanging: straight down from the tangent lines, pushed out by h
    off = ~on
    sg = np.sign(s[off])
    x[off, 1] = cy - (np.abs(s[off]) - half)
    x[off, 2] = cz + sg * (Ro + h[off])
    return x.astype(np.float32)


def config(idx: int, **over) -> Scene:
    """The five workloads: 0 small hanging cloth, 1 sphere drape 256^2,
    2 cylinder drape 600^2 (mixed precision), 3/4 are multi-scene sets built by
    `batch_scenes` / `serving_scenes`."""
    if idx == 0:
        return hanging_cloth(32, seed=0, r=16, steps=10, iters=20, **over)
    if idx == 1:
        kw = dict(n=256, seed=1, obstacle="sphere", r=64, steps=100, d_hat=1e-3)
        kw.update(over)
        return drop_cloth(**kw)
    if idx == 2:
        kw = dict(n=600, seed=2, obstacle="cylinder", r=128, steps=200, precision="mixed")
        kw.update(over)
        return drop_cloth(**kw)
    raise ValueError("configs 3 and 4 are scene sets: use batch_scenes / serving_scenes")


def batch_scenes(count: int = 64, seed: int = 3, r: int = 32) -> List[Scene]:
    """Uneven cloths, side vertex count uniform in 16..128 and edge length
    1/127 m, each over its own sphere (radius 0.25 x side, 0.3 x side below)."""
    rng = np.random.default_rng(seed)
    out = []
    for s in range(count):
        n = int(rng.integers(16, 129))
        side = (n - 1) / 127.0
        out.append(drop_cloth(n, seed=int(rng.integers(1 << 30)), obstacle="sphere",
                              r=min(r, n * n // 4), steps=1, side=side, precision="mixed"))
    return out


def serving_scenes(count: int = 200, seed: int = 4, r: int = 64,
                   nmin: int = 4096, nmax: int = 360000) -> List[Scene]:
    """Scenes with vertex counts log-uniform in [nmin, nmax], alternating the
    sphere and cylinder drops."""
    rng = np.random.default_rng(seed)
    out = []
    for s in range(count):
        N = math.exp(rng.uniform(math.log(nmin), math.log(nmax)))
        n = max(16, int(round(math.sqrt(N))))
        out.append(drop_cloth(n, seed=int(rng.integers(1 << 30)),
                              obstacle="sphere" if s % 2 == 0 else "cylinder",
                              r=r, steps=1, precision="mixed"))
    return out
