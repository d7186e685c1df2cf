"""Seeded synthetic inputs for the shell Poisson solve.

This module holds data generation only (grids, random fields, manufactured
fields sampled at cell centres, batch and arrival draws); it contains none of
the solver's arithmetic.  Both the GPU path and the CPU oracle read their
inputs from here.

The paper's Poisson right-hand sides come from DNS runs that are not
available; these generators stand in for them with the paper's geometry
(radius ratio 0.6, gap d = 1, tanh radial clustering of eq. (stretching)) and
grid scales of the same order as its runs (Sec. 4, Table results).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np

MAP_IDENTITY, MAP_SPHERE, MAP_OBLATE, MAP_TRIAXIAL = 0, 1, 2, 3

THETA0 = 0.05
THETA1 = math.pi - 0.05


@dataclass
class Shell:
    """Grid of n_r x n_theta x n_phi cells; arrays are [r][theta][phi], phi
    periodic and contiguous."""
    n_r: int
    n_theta: int
    n_phi: int
    map: int = MAP_SPHERE
    r_inner: float = 1.5
    r_outer: float = 2.5
    theta0: float = THETA0
    theta1: float = THETA1
    radial_stretch: float = 0.0
    flattening: float = 0.0
    skew: float = 0.0

    @property
    def shape(self):
        return (self.n_r, self.n_theta, self.n_phi)

    @property
    def cells(self) -> int:
        return self.n_r * self.n_theta * self.n_phi


def cell_centres(g: Shell):
    """Normalised radial coordinate, colatitude and azimuth at cell centres
    (index positions a+1/2, b+1/2, c+1/2)."""
    xi = (np.arange(g.n_r) + 0.5) / g.n_r
    th = g.theta0 + (np.arange(g.n_theta) + 0.5) / g.n_theta * (g.theta1 - g.theta0)
    ph = 2.0 * np.pi * (np.arange(g.n_phi) + 0.5) / g.n_phi
    return xi, th, ph


def manufactured_p(g: Shell) -> np.ndarray:
    """p = cos(pi xi) sin(2 phi) sin(theta) at cell centres, xi the
    normalised radial coordinate (zero slope at both radial walls)."""
    xi, th, ph = cell_centres(g)
    return (np.cos(np.pi * xi)[:, None, None] * np.sin(th)[None, :, None]
            * np.sin(2.0 * ph)[None, None, :])


def smoothed_noise(shape, seed: int = 0, passes: int = 3) -> np.ndarray:
    """N(0,1) field from numpy's default_rng(seed), smoothed by `passes`
    weighted-Jacobi passes x <- x + 2/3 (mean of the 6 index neighbours - x),
    mirrored at the r and theta ends and wrapped in phi; mean removed."""
    x = np.random.default_rng(seed).standard_normal(shape)
    for _ in range(passes):
        p = np.pad(x, ((1, 1), (1, 1), (0, 0)), mode="edge")
        nb = (p[2:, 1:-1] + p[:-2, 1:-1] + p[1:-1, 2:] + p[1:-1, :-2]
              + np.roll(x, 1, axis=2) + np.roll(x, -1, axis=2))
        x = x + (2.0 / 3.0) * (nb / 6.0 - x)
    return x - x.mean()


def config1() -> Shell:
    """32^3 sphere shell, uniform spacing."""
    return Shell(32, 32, 32)


def velocity_field(shape, seed: int = 0) -> np.ndarray:
    """Synthetic intermediate velocity u*** for the projection step:
    [3][n_r][n_theta][n_phi] Cartesian components, each a smoothed N(0,1)
    field (seeds seed, seed + 1, seed + 2)."""
    return np.stack([smoothed_noise(shape, seed + q) for q in range(3)])


def config2() -> Shell:
    """Paper-scale shell 192(r) x 256(theta) x 512(phi), tanh clustering
    with stretching factor 2.0."""
    return Shell(192, 256, 512, radial_stretch=2.0)


# size set of the batched and serving forms
SIZE_SET = [(16, 16, 16), (32, 32, 32), (64, 64, 128), (96, 128, 256), (128, 128, 256)]


@dataclass
class Problem:
    grid: Shell
    seed: int

    def rhs(self) -> np.ndarray:
        return smoothed_noise(self.grid.shape, self.seed)


def batch_problems(n: int = 64, seed: int = 4, sizes=None) -> list:
    """Batched form: size index from default_rng(seed).integers(0, len, n);
    even i sphere, odd i oblate with flattening 0.1; RHS seed 1000 + i."""
    sizes = sizes or SIZE_SET
    pick = np.random.default_rng(seed).integers(0, len(sizes), n)
    out = []
    for i in range(n):
        nr, nt, np_ = sizes[int(pick[i])]
        g = Shell(nr, nt, np_, map=MAP_SPHERE if i % 2 == 0 else MAP_OBLATE,
                  flattening=0.0 if i % 2 == 0 else 0.1)
        out.append(Problem(g, 1000 + i))
    return out


@dataclass
class Arrival:
    t: float
    problem: Problem
    rid: int


def arrival_stream(rate: float = 200.0, duration: float = 60.0, seed: int = 5,
                   sizes=None) -> list:
    """Serving form: exponential inter-arrival times (mean 1/rate) from
    default_rng(seed) until `duration`; size uniform over the size set;
    sphere with probability 1/2, else oblate with flattening U(0, 0.15);
    RHS seed 10**6 + request id."""
    sizes = sizes or SIZE_SET
    rng = np.random.default_rng(seed)
    out, t, rid = [], 0.0, 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        nr, nt, np_ = sizes[int(rng.integers(0, len(sizes)))]
        if rng.random() < 0.5:
            g = Shell(nr, nt, np_)
        else:
            g = Shell(nr, nt, np_, map=MAP_OBLATE, flattening=float(rng.uniform(0.0, 0.15)))
        out.append(Arrival(t, Problem(g, 10**6 + rid), rid))
        rid += 1
    return out


def with_dims(g: Shell, shape) -> Shell:
    return replace(g, n_r=shape[0], n_theta=shape[1], n_phi=shape[2])
