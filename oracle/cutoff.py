"""Smooth cut-off w_cut of the partial-data model (eq. data-part; its
construction at the start of Section 5).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The data are known on the open box (0, X)^d of detector and time coordinates
(d = 2 for line detectors: (x1, t); d = 3 for the planar array: (x1, x2, t))
and enter the reconstruction as ``w_cut * p``.  The paper builds w_cut by
convolving a mollifier with a box indicator.  Two readings make that
construction usable:

* Mollifier: the standard bump of radius ``eps``,
  ``phi(y) = C exp(-1 / (1 - |y|^2 / eps^2))`` on ``|y| < eps``, normalised to
  unit mass.  (The printed ``exp(-1/(eps - |y|^2)^4)`` underflows to zero in
  double precision for every ``|y|`` once eps is a few sampling steps; its
  normalised limit is a point mass, i.e. no smoothing at all.)
* Box: the indicator of ``[eps, n_i - eps]`` on each axis (the data box shrunk
  by eps).  Only then is w_cut zero outside (0, X)^d, as the paper requires;
  with the unshrunk box it would be 1/2 on the faces and non-zero outside.

Coordinates are in sampling steps of each axis: sample ``s`` of an axis with
``n`` samples sits at ``s``, the data box is ``[0, n]``, and eps is a number of
steps (the paper takes dx = dt and eps a small multiple of the step).  So

    w(s) = int phi(y) prod_i 1{ eps <= s_i - y_i <= n_i - eps } dy.

``weight_of`` evaluates that integral by nested Gauss-Legendre quadrature
along chords of the ball (outer axis first; each inner interval is the chord
of the ball at the outer coordinates, cut to the box), with
``numpy.polynomial.legendre.leggauss`` nodes.  The bump is flat to all orders
at the sphere, so the nested rule converges fast; values are cached per
distinct clipped box up to reflections and permutations of the axes.

``weights(g, eps)``  the (n1, n2, nt) array of w over the data grid;
``apply(x, g, eps)``  ``w * x`` for a data-shaped array (2D (n1, nt) accepted).
With the cut-off the operators become ``R(w p)``, ``w R^T(q)``, ``w A(f)``
and ``A^T(w p)``.
"""
from __future__ import annotations

from functools import lru_cache

import numpy as np

_NODES = 96


def _gl(a: float, b: float):
    x, w = np.polynomial.legendre.leggauss(_NODES)
    h = 0.5 * (b - a)
    return a + h * (x + 1.0), h * w


def bump(r2, eps: float):
    """Unnormalised ``exp(-1/(1 - r^2/eps^2))`` inside the ball, 0 outside."""
    r2 = np.asarray(r2, dtype=np.float64)
    q = 1.0 - r2 / (eps * eps)
    out = np.zeros_like(q)
    inside = q > 0
    out[inside] = np.exp(-1.0 / q[inside])
    return out


def _integral(box, eps: float) -> float:
    """int of the unnormalised bump over the ball cut to ``box``, a list of
    (lo, hi) per axis (1 to 3 axes).  Level i integrates axis i over the chord
    of the ball left by the outer coordinates, cut to the box; the node arrays
    of level i carry one dimension per outer axis."""
    x, w = np.polynomial.legendre.leggauss(_NODES)
    r2 = np.zeros(())        # squared radius used by the outer coordinates
    wt = np.ones(())         # product of the outer weights
    for lo_b, hi_b in box:
        rho = np.sqrt(np.maximum(eps * eps - r2, 0.0))
        lo = np.maximum(-rho, lo_b)
        hi = np.maximum(np.minimum(rho, hi_b), lo)   # empty chords get zero length
        h = 0.5 * (hi - lo)
        y = lo[..., None] + h[..., None] * (x + 1.0)
        wt = wt[..., None] * h[..., None] * w
        r2 = r2[..., None] + y * y
    return float(np.sum(wt * bump(r2, eps)))


@lru_cache(maxsize=None)
def mass(eps: float, d: int) -> float:
    """Unnormalised mass of the bump in d dimensions (the constant 1/C)."""
    return _integral([(-eps, eps)] * d, eps)


_cache: dict = {}


def weight_of(s, n, eps: float) -> float:
    """w at the sample ``s`` (one coordinate per axis) of a grid with ``n``
    samples per axis."""
    box = []
    for si, ni in zip(s, n):
        lo = float(si) - (float(ni) - eps)   # s - y <= n - eps
        hi = float(si) - eps                 # s - y >= eps
        box.append((max(lo, -eps), min(hi, eps)))
    # the bump is invariant under reflecting any axis and permuting the axes:
    # boxes equal up to those motions share one value
    canon = []
    for lo, hi in box:
        if hi >= eps > -lo:
            lo, hi = -hi, -lo
        canon.append((lo, hi))
    box = sorted(canon)
    key = (eps, tuple(box))
    if key not in _cache:
        if any(hi <= lo for lo, hi in box):
            val = 0.0
        elif all(lo <= -eps and hi >= eps for lo, hi in box):
            val = 1.0
        else:
            val = _integral(box, eps) / mass(eps, len(box))
        _cache[key] = val
    return _cache[key]


def weights(g, eps: float):
    """w over the data grid, shape (n1, n2, nt); 2D geometries (n2 = 1) use
    the two-dimensional bump over (x1, t)."""
    n1, n2, nt = g["n1"], g["n2"], g["nt"]
    out = np.empty((n1, n2, nt))
    for a in range(n1):
        for b in range(n2):
            for t in range(nt):
                if n2 == 1:
                    out[a, b, t] = weight_of((a, t), (n1, nt), eps)
                else:
                    out[a, b, t] = weight_of((a, b, t), (n1, n2, nt), eps)
    return out


def apply(x, g, eps: float):
    """``w * x`` for a data-shaped array."""
    x = np.asarray(x)
    w = weights(g, eps)
    return x * (w[:, 0, :] if x.ndim == 2 else w)
