"""Kaiser-Bessel window and its Fourier transform (Section 3.2).

TEST INFRASTRUCTURE ONLY (see the package docstring).

``psi(theta)``  window ``I0(K sqrt(alpha^2 - theta^2)) / I0(alpha K)`` on
                ``|theta| <= alpha``, zero outside.
``psi_hat(w)``  its transform ``int exp(-i w theta) psi(theta) dtheta``
                ``= 2 sinh(alpha s) / (I0(alpha K) s)``, ``s = sqrt(K^2 - w^2)``;
                for ``|w| > K`` the root is imaginary and the same expression
                becomes ``2 sin(alpha |s|) / (I0(alpha K) |s|)``; at ``|w| = K``
                the limit is ``2 alpha / I0(alpha K)``.
``fourmont_bound``  the truncation-error estimate quoted at the end of
                Section 3.2: ``30 / (pi I0(K pi sqrt(alpha^2 - 1) / c^2))``.

``I0`` is ``numpy.i0`` (a library primitive).
"""
from __future__ import annotations

import numpy as np


def psi(theta, K: float, alpha: float):
    theta = np.asarray(theta, dtype=np.float64)
    inside = np.abs(theta) <= alpha
    arg = K * np.sqrt(np.where(inside, alpha * alpha - theta * theta, 0.0))
    return np.where(inside, np.i0(arg) / np.i0(alpha * K), 0.0)


def psi_hat(w, K: float, alpha: float):
    w = np.asarray(w, dtype=np.float64)
    s2 = K * K - w * w
    out = np.empty_like(w)
    pos = s2 > 0
    neg = s2 < 0
    zero = ~(pos | neg)
    s = np.sqrt(np.abs(s2))
    out[pos] = 2.0 * np.sinh(alpha * s[pos]) / s[pos]
    out[neg] = 2.0 * np.sin(alpha * s[neg]) / s[neg]
    out[zero] = 2.0 * alpha
    return out / np.i0(alpha * K)


def fourmont_bound(c: float, K: float, alpha: float) -> float:
    return 30.0 / (np.pi * float(np.i0(K * np.pi * np.sqrt(alpha * alpha - 1.0) / (c * c))))
