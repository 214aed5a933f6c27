"""The paper's one-dimensional NUFFT (Section 3.1), for pinning only.

TEST INFRASTRUCTURE ONLY (see the package docstring).

``ndft(g, omega)``   the definition, eq. (dft): ``sum_n exp(-i omega n 2 pi/N) g_n``.
``nufft(g, omega, c, K, alpha)``  the approximation of the NUFFT algorithm in
   Section 3.1, step by step:

   1. scale ``g_n`` by ``1 / Psi(2 pi n / N - pi)`` and by the constant of the
      oversampled DFT (eq. nufft-c),
   2. append ``(c - 1) N`` zeros,
   3. FFT of length ``c N`` (giving ``hat G_j``, periodic in ``j``),
   4. for each node keep the terms ``|j - c omega| <= c K`` of eq. (nufft-a),
      each weighted by ``exp(-i pi (omega - j/c)) Psi_hat(omega - j/c)``.

Two readings of the printed text are taken here (both follow from the proof of
the NUFFT proposition and are pinned against ``ndft`` by the tests):

* constant: the Fourier series of ``theta -> exp(-i omega theta) Psi(theta)`` on
  the period ``2 pi c`` has coefficients ``Psi_hat(omega - j/c) / (2 pi c)``,
  so the constant is ``1 / (2 pi c)`` (the printed ``c / (2 pi)`` is exact only
  for ``c = 1``);
* phase: the factor is ``exp(-i pi (omega - j/c))`` as in eq. (nufft-a), not the
  ``exp(-i (omega - j/c) pi / c)`` of the algorithm's precomputation line.
"""
from __future__ import annotations

import numpy as np

from .kb import psi, psi_hat


def ndft(g, omega):
    g = np.asarray(g, dtype=np.complex128)
    N = g.shape[-1]
    n = np.arange(N)
    ph = np.mod(np.outer(np.asarray(omega, dtype=np.float64), n), N)
    return np.exp(-2j * np.pi * ph / N) @ g


def nufft(g, omega, c: float, K: float, alpha: float, constant: str = "1/(2 pi c)",
          phase: str = "pi"):
    """NUFFT of one vector ``g`` at nodes ``omega``.

    ``constant`` and ``phase`` select the reading; the alternatives ("c/(2 pi)",
    "pi/c") exist only so that tests can show the printed forms fail.
    """
    g = np.asarray(g, dtype=np.complex128)
    N = g.shape[0]
    cN = int(round(c * N))
    assert abs(c * N - cN) < 1e-9 and cN % 2 == 0
    n = np.arange(N)
    const = 1.0 / (2 * np.pi * c) if constant == "1/(2 pi c)" else c / (2 * np.pi)
    h = g / psi(2 * np.pi * n / N - np.pi, K, alpha) * const
    h = np.concatenate([h, np.zeros(cN - N, dtype=np.complex128)])
    Ghat = np.fft.fft(h)
    out = np.zeros(len(omega), dtype=np.complex128)
    for i, w in enumerate(np.asarray(omega, dtype=np.float64)):
        j = np.arange(int(np.ceil(c * w - c * K)), int(np.floor(c * w + c * K)) + 1)
        u = w - j / c
        ph = np.exp(-1j * np.pi * u) if phase == "pi" else np.exp(-1j * u * np.pi / c)
        out[i] = np.sum(ph * psi_hat(u, K, alpha) * Ghat[np.mod(j, cN)])
    return out
