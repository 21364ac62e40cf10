"""Seeded synthetic workloads (problem data only; none of the method's arithmetic).

Each problem is the Helmholtz impedance problem of Sec. 2 on (0,1)^2:
-Lap u - kappa^2 (1 - b) u = s,  d_n u + i eta u = t,  eta = kappa.  This module
draws the problem parameters (mesh, order, wavenumber, coefficient bumps,
plane-wave direction) from numpy's PCG64 and returns plain callables that
evaluate b(x, y) and t(x, y, n) at whatever points the caller supplies.  Both
the oracle and the GPU path evaluate them at their own nodes.

Workloads (the paper's experiment uses a Gaussian bump on a 64x64, N=16 mesh;
these are synthetic stand-ins of the same shape):

* ``c1``: 4x4 elements, N=8, kappa=10, b=0, plane-wave t, d=(cos .3, sin .3).
* ``c2``: 16x16, N=16, kappa=40, b = 1.5 exp(-|x-(.5,.5)|^2/0.02).
* ``c3``: 64x64, N=16, kappa=200, b = sum of 8 seeded Gaussian bumps.
* ``c4``: 256 problems, n in {8,16,32}, N in {8,12,16}, kappa ~ U[20,120],
  1-6 bumps, random plane-wave direction.
* ``c5``: Poisson arrivals (mean gap 20 ms for 60 s); each request drawn as in
  c4, or with probability 0.1 a 128x128, N=16, kappa=400 problem.
* ``x1``: the paper's own experiment: the Gaussian bump 1.5 exp(-160 r^2),
  the scattering source of the incident wave exp(i kappa x), t = 0, N = 16,
  9.6 points per wavelength (kappa = 670 on 64x64).
"""
import math
from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np

D_DEFAULT = (math.cos(0.3), math.sin(0.3))


@dataclass
class Bumps:
    """b(x) = sum_k a_k exp(-|x - c_k|^2 / w_k)."""
    a: np.ndarray
    cx: np.ndarray
    cy: np.ndarray
    w: np.ndarray

    def __call__(self, x, y):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        out = np.zeros(np.broadcast(x, y).shape)
        for a, cx, cy, w in zip(self.a, self.cx, self.cy, self.w):
            out += a * np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / w)
        return out


def zero_field(x, y):
    return np.zeros(np.broadcast(np.asarray(x), np.asarray(y)).shape)


def draw_bumps(rng, count):
    a = rng.uniform(-0.8, 0.8, count)
    c = rng.uniform(0.1, 0.9, (count, 2))
    w = rng.uniform(0.01, 0.05, count)
    return Bumps(a, c[:, 0], c[:, 1], w)


@dataclass
class PlaneWave:
    """u = exp(i kappa d.x); its impedance data t = (d_n + i eta) u."""
    kappa: float
    eta: float
    d: tuple = D_DEFAULT

    def u(self, x, y):
        return np.exp(1j * self.kappa * (self.d[0] * x + self.d[1] * y))

    def t(self, x, y, nx, ny):
        dn = self.d[0] * nx + self.d[1] * ny
        return 1j * (self.kappa * dn + self.eta) * self.u(x, y)


@dataclass
class Problem:
    n: int
    N: int
    kappa: float
    eta: float
    b: Callable
    wave: PlaneWave
    s: Optional[Callable] = None
    levels: int = 0            # 0: top level
    coarse_iters: int = 5
    tol: float = 1e-8
    name: str = ""
    arrival: float = 0.0

    @property
    def skeleton_dof(self):
        return 4 * (self.N - 1) * self.n * (self.n - 1)


def c1():
    k = 10.0
    return Problem(4, 8, k, k, zero_field, PlaneWave(k, k), levels=4,
                   coarse_iters=5, tol=1e-10, name="c1")


def c2_bump(x, y):
    return 1.5 * np.exp(-((np.asarray(x) - 0.5) ** 2 + (np.asarray(y) - 0.5) ** 2) / 0.02)


def c2(coarse_iters=5):
    k = 40.0
    return Problem(16, 16, k, k, c2_bump, PlaneWave(k, k), levels=8,
                   coarse_iters=coarse_iters, tol=1e-10, name="c2")


def c3(seed=3):
    rng = np.random.default_rng(seed)
    k = 200.0
    return Problem(64, 16, k, k, draw_bumps(rng, 8), PlaneWave(k, k), levels=12,
                   coarse_iters=5, tol=1e-8, name="c3")


def _draw_c4_like(rng):
    n = int(rng.choice([8, 16, 32]))
    N = int(rng.choice([8, 12, 16]))
    k = float(rng.uniform(20.0, 120.0))
    K = int(rng.integers(1, 7))
    b = draw_bumps(rng, K)
    th = float(rng.uniform(0.0, 2 * math.pi))
    return Problem(n, N, k, k, b, PlaneWave(k, k, (math.cos(th), math.sin(th))),
                   levels=0, coarse_iters=5, tol=1e-8)


def c4(count=256, seed=4):
    ss = np.random.SeedSequence(seed)
    out = []
    for i, child in enumerate(ss.spawn(count)):
        pr = _draw_c4_like(np.random.default_rng(child))
        pr.name = f"c4[{i}]"
        out.append(pr)
    return out


def c5(duration=60.0, rate=50.0, big_frac=0.1, seed=5, big_n=128, big_kappa=400.0):
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    i = 0
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t >= duration:
            break
        if rng.uniform() < big_frac:
            K = int(rng.integers(1, 7))
            b = draw_bumps(rng, K)
            th = float(rng.uniform(0.0, 2 * math.pi))
            pr = Problem(big_n, 16, big_kappa, big_kappa, b,
                         PlaneWave(big_kappa, big_kappa, (math.cos(th), math.sin(th))),
                         levels=0, coarse_iters=5, tol=1e-8)
        else:
            pr = _draw_c4_like(rng)
        pr.name = f"c5[{i}]"
        pr.arrival = t
        out.append(pr)
        i += 1
    return out


@dataclass
class ZeroData:
    """Zero impedance data t = 0 (the scattered-field problem)."""
    kappa: float
    eta: float

    def t(self, x, y, nx, ny):
        return np.zeros(np.broadcast(np.asarray(x), np.asarray(y)).shape, dtype=np.complex128)


def x1_bump(x, y):
    return 1.5 * np.exp(-160.0 * ((np.asarray(x) - 0.5) ** 2 + (np.asarray(y) - 0.5) ** 2))


@dataclass
class ScatteringSource:
    """s = -kappa^2 b(x) exp(i kappa x): the source of the field scattered by
    the coefficient b when the plane wave exp(i kappa x) is incident (the
    total field solves the homogeneous equation)."""
    kappa: float
    b: Callable

    def __call__(self, x, y):
        x = np.asarray(x, dtype=np.float64)
        return -self.kappa ** 2 * self.b(x, y) * np.exp(1j * self.kappa * x)


def x1(n=64, N=16, points_per_wavelength=9.6, levels=0, coarse_iters=5):
    """The paper's experiment (Sec. 5): b = 1.5 exp(-160 |x - (0.5, 0.5)|^2),
    s = -kappa^2 b exp(i kappa x), t = 0, GLL order N, kappa from the points
    per wavelength over the n N GLL intervals of a side: kappa = 2 pi n N /
    points_per_wavelength (670.2 on the paper's 64 x 64, N = 16 mesh)."""
    k = 2.0 * math.pi * n * N / points_per_wavelength
    return Problem(n, N, k, k, x1_bump, ZeroData(k, k), s=ScatteringSource(k, x1_bump), levels=levels,
                   coarse_iters=coarse_iters, tol=1e-8, name=f"x1_{n}")


def by_name(name):
    return {"c1": c1, "c2": c2, "c3": c3, "x1": x1}[name]()
