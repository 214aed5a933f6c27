"""Seeded synthetic inputs for the planar photoacoustic reconstruction.

This module holds no reconstruction arithmetic.  It draws phantom parameters
from a seeded PCG64 generator and evaluates textbook closed forms of the
measured signal, so that the CPU oracle, the tests and the benchmark all see
the same inputs.

Phantoms
--------
* 3D: uniformly heated balls ``f = A * 1{|x - x0| < a}``.  The pressure trace
  of one ball on the detector plane ``y = 0`` follows from the radial
  d'Alembert solution ``r p(r, t) = ((r - v t) f(r - v t) + (r + v t) f(r + v t)) / 2``
  (the wave problem of Section 2 with zero initial velocity).  For a detector
  at distance ``r > a`` from the centre this is the N-shaped pulse
  ``p = A (r - v t) / (2 r)`` for ``|r - v t| < a`` and zero otherwise.
* 2D: uniform disks rasterised at the pixel centres ``(m dx, q dz)``.

Geometry convention (Section 4 discretisation): detector ``m`` sits at
``x = m dx`` on the plane ``y = 0``, time sample ``n`` at ``t = n dt`` and image
sample ``q`` at depth ``y = q dz``.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def rng(seed: int) -> np.random.Generator:
    """The one generator family used for every synthetic input."""
    return np.random.Generator(np.random.PCG64(int(seed)))


@dataclass(frozen=True)
class Balls:
    centres: np.ndarray  # (n, 3): (x1, x2, depth), physical units
    radii: np.ndarray    # (n,)
    amps: np.ndarray     # (n,)


def draw_balls(n: int, seed: int, L: float = 1.0, n1: int = 128,
               gen: np.random.Generator | None = None) -> Balls:
    """``n`` balls with radius ``U[0.05, 0.2] L``, centre uniform in
    ``[a + 2 dx, L - a - 2 dx]^3`` (inside the volume, clear of the detector
    plane) and amplitude ``U[0.5, 1]``; ``dx = L / n1``."""
    g = rng(seed) if gen is None else gen
    dx = L / n1
    radii = g.uniform(0.05, 0.2, size=n) * L
    lo = radii + 2 * dx
    hi = L - radii - 2 * dx
    centres = lo[:, None] + (hi - lo)[:, None] * g.uniform(0.0, 1.0, size=(n, 3))
    amps = g.uniform(0.5, 1.0, size=n)
    return Balls(centres=centres, radii=radii, amps=amps)


def ball_traces(balls: Balls, n1: int, n2: int, nt: int, dx: float, dt: float,
                vs: float = 1.0, dtype=np.float64) -> np.ndarray:
    """Closed-form detector data ``p[m1, m2, n]`` (t fastest) of a sum of balls.

    Evaluated in float64 one detector row at a time, then cast to ``dtype``.
    """
    out = np.zeros((n1, n2, nt), dtype=dtype)
    x2 = np.arange(n2) * dx
    t = np.arange(nt) * dt
    for m1 in range(n1):
        row = np.zeros((n2, nt))
        x1 = m1 * dx
        for (cx, cy, cz), a, amp in zip(balls.centres, balls.radii, balls.amps):
            r = np.sqrt((x1 - cx) ** 2 + (x2 - cy) ** 2 + cz ** 2)  # (n2,)
            d = r[:, None] - vs * t[None, :]
            row += np.where(np.abs(d) < a, amp * d / (2.0 * r[:, None]), 0.0)
        out[m1] = row
    return out


def ball_volume(balls: Balls, n1: int, n2: int, nz: int, dx: float, dz: float,
                dtype=np.float64) -> np.ndarray:
    """The phantom itself sampled at the voxel centres ``(m1 dx, m2 dx, q dz)``."""
    x1 = np.arange(n1)[:, None, None] * dx
    x2 = np.arange(n2)[None, :, None] * dx
    z = np.arange(nz)[None, None, :] * dz
    f = np.zeros((n1, n2, nz))
    for (cx, cy, cz), a, amp in zip(balls.centres, balls.radii, balls.amps):
        f += amp * (((x1 - cx) ** 2 + (x2 - cy) ** 2 + (z - cz) ** 2) < a * a)
    return f.astype(dtype)


@dataclass(frozen=True)
class Disks:
    centres: np.ndarray  # (n, 2) in pixels: (x, depth)
    radii: np.ndarray    # (n,) in pixels
    amps: np.ndarray


def draw_disks(n: int, seed: int, npx: int = 128) -> Disks:
    """``n`` disks: radius ``U[4, 16]`` px, centre ``U[r + 2, npx - r - 2]`` px on
    both axes, amplitude ``U[0.5, 1]``."""
    g = rng(seed)
    radii = g.uniform(4.0, 16.0, size=n)
    lo = radii + 2.0
    hi = npx - radii - 2.0
    centres = lo[:, None] + (hi - lo)[:, None] * g.uniform(0.0, 1.0, size=(n, 2))
    amps = g.uniform(0.5, 1.0, size=n)
    return Disks(centres=centres, radii=radii, amps=amps)


def disk_image(disks: Disks, nx: int, nz: int, dtype=np.float64) -> np.ndarray:
    """Disks rasterised at pixel centres: ``f[m, q]``, depth fastest."""
    m = np.arange(nx)[:, None]
    q = np.arange(nz)[None, :]
    f = np.zeros((nx, nz))
    for (cx, cz), r, amp in zip(disks.centres, disks.radii, disks.amps):
        f += amp * (((m - cx) ** 2 + (q - cz) ** 2) < r * r)
    return f.astype(dtype)


def add_noise(p: np.ndarray, sigma: float, gen: np.random.Generator) -> np.ndarray:
    """Additive white Gaussian noise of standard deviation ``sigma``."""
    return (p + gen.normal(0.0, sigma, size=p.shape)).astype(p.dtype)


def random_array(shape, seed: int, dtype=np.float64) -> np.ndarray:
    """Standard-normal test array (parity cases that need no phantom)."""
    return rng(seed).standard_normal(size=shape).astype(dtype)


# ---------------------------------------------------------------------------
# Workload recipes.  Each returns plain numpy arrays plus the geometry numbers
# as a dict; nothing here depends on the reconstruction library.

def planar_case(n: int, n_balls: int, seed: int, noise: float = 1e-3,
                L: float = 1.0, dtype=np.float64):
    """3D planar case: ``n x n`` detectors, ``nt = 2 n`` samples, ``nz = n``
    depth samples, ``dx = dz = dt = L / n``, ``v_s = 1``."""
    gen = rng(seed)
    balls = draw_balls(n_balls, seed, L=L, n1=n, gen=gen)
    dx = L / n
    geom = dict(n1=n, n2=n, nt=2 * n, nz=n, dx=dx, dt=dx, dz=dx, vs=1.0)
    p = ball_traces(balls, n, n, 2 * n, dx, dx)
    if noise > 0:
        p = add_noise(p, noise, gen)
    return p.astype(dtype), geom, balls


def batched_sizes(seed: int = 5000):
    """Sixteen plane edges 64, 72, ..., 184 in a seeded order."""
    edges = 64 + 8 * np.arange(16)
    return [int(e) for e in rng(seed).permutation(edges)]


def batched_case(seed: int = 5000, dtype=np.float64):
    """Sixteen uneven planar instances; instance ``j`` uses seed ``seed + j``,
    ``4..24`` balls and no noise."""
    cases = []
    for j, e in enumerate(batched_sizes(seed)):
        g = rng(seed + 1 + j)
        nb = int(g.integers(4, 25))
        p, geom, balls = planar_case(e, nb, seed + 1 + j, noise=0.0, dtype=dtype)
        cases.append((p, geom, balls))
    return cases


# ---------------------------------------------------------------------------
# 2D circular object of Section 5: f = (2/a) sqrt(a^2 - |x - x0|^2) inside the
# circle, which is (1/a) times the projection of a uniform ball of radius a;
# its data on y = 0 is therefore (1/a) times the line integral of the ball's
# N-shaped pulse, in closed form
#   p(x, t) = (1/a) Re[(s+ - s-) - t log((s+ + t + a) / (s- + t - a))],
#   s+- = ((t +- a)^2 - rho^2)^(1/2),  rho = |(x, 0) - x0|,
# principal branches (the sign under the root corrected; v_s = 1 units).

def circle_image(x0: float, y0: float, a: float, nx: int, nz: int, dx: float, dz: float,
                 dtype=np.float64) -> np.ndarray:
    """``f[m, q]`` at ``(m dx, q dz)``."""
    x = np.arange(nx)[:, None] * dx
    y = np.arange(nz)[None, :] * dz
    r2 = (x - x0) ** 2 + (y - y0) ** 2
    return ((2.0 / a) * np.sqrt(np.maximum(a * a - r2, 0.0))).astype(dtype)


def circle_traces(x0: float, y0: float, a: float, nx: int, nt: int, dx: float, dt: float,
                  vs: float = 1.0, dtype=np.float64) -> np.ndarray:
    """Closed-form data ``p[m, n]`` of the circle at detector ``m dx`` (plane
    ``y = 0``) and time ``n dt`` (distances in units of ``vs`` time)."""
    x = np.arange(nx)[:, None] * dx
    t = vs * np.arange(nt)[None, :] * dt
    rho2 = (x - x0) ** 2 + y0 * y0
    with np.errstate(invalid="ignore", divide="ignore"):
        sp = np.sqrt(((t + a) ** 2 - rho2).astype(np.complex128))
        sm = np.sqrt(((t - a) ** 2 - rho2).astype(np.complex128))
        val = (sp - sm) - t * np.log((sp + t + a) / (sm + t - a))
    p = np.real(val) / a
    return np.where(np.isfinite(p), p, 0.0).astype(dtype)


def circle_case(n: int = 512, seed: int = 1006, noise_var_frac: float = 0.0):
    """The circle experiment: ``n`` line detectors on ``[0, 1)``, ``nt = nz = n``
    (data on ``(0, 1)^2``, ``dx = dt = dz = 1/n``, ``v_s = 1``); centre and
    radius drawn from the seed (the paper gives neither): ``a ~ U[0.1, 0.2]``,
    ``x0 ~ U[0.3, 0.7]``, ``y0 ~ U[a + 0.1, 0.6]``.  ``noise_var_frac`` adds
    Gaussian noise of variance that fraction of the largest data value."""
    g = rng(seed)
    a = float(g.uniform(0.1, 0.2))
    x0 = float(g.uniform(0.3, 0.7))
    y0 = float(g.uniform(a + 0.1, 0.6))
    d = 1.0 / n
    p = circle_traces(x0, y0, a, n, n, d, d)
    if noise_var_frac > 0:
        sigma = np.sqrt(noise_var_frac * np.abs(p).max())
        p = p + sigma * g.standard_normal(p.shape)
    geom = dict(n1=n, n2=1, nt=n, nz=n, dx=d, dt=d, dz=d, vs=1.0)
    return p, geom, (x0, y0, a)
