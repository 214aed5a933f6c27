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


# ---------------------------------------------------------------------------
# The other ways of evaluating eq. (fft-2) that Section 4 compares with the
# NUFFT-based algorithm (interpolation-based and truncated sinc), each written
# from its description there.  Tap windows are half-open,
# ``c omega - c K < j <= c omega + c K`` (``2 c K`` taps), which is the closed
# window ``|j - c omega| <= c K`` except when its ends are integers.

def _window(w, c, K):
    j0 = int(np.floor(c * w - c * K)) + 1
    return np.arange(j0, j0 + int(round(2 * c * K)))


def sinc_hat(u, c: float):
    """Fourier transform of the indicator of ``[-c pi, c pi]``:
    ``int exp(-i u theta) dtheta = 2 sin(c pi u) / u`` (``2 c pi`` at 0)."""
    u = np.asarray(u, dtype=np.float64)
    return 2.0 * np.pi * c * np.sinc(c * u)  # numpy sinc(x) = sin(pi x) / (pi x)


def truncated_sinc(g, omega, c: float, K: float):
    """Truncated sinc reconstruction: the NUFFT algorithm with ``Psi`` the
    indicator of ``[-c pi, c pi]``.  ``Psi = 1`` on every sample, so nothing is
    deconvolved: ``g`` zero-padded to ``c N``, FFT, then per node the ``2 c K``
    taps ``exp(-i pi (omega - j/c)) Psi_hat(omega - j/c) Ghat_j / (2 pi c)``."""
    g = np.asarray(g, dtype=np.complex128)
    N = g.shape[0]
    cN = int(round(c * N))
    Ghat = np.fft.fft(np.concatenate([g, np.zeros(cN - N, dtype=np.complex128)]))
    out = np.zeros(len(omega), dtype=np.complex128)
    for i, w in enumerate(np.asarray(omega, dtype=np.float64)):
        j = _window(w, c, K)
        u = w - j / c
        out[i] = np.sum(np.exp(-1j * np.pi * u) * sinc_hat(u, c) * Ghat[np.mod(j, cN)]) / (2 * np.pi * c)
    return out


def interpolated(g, omega, c: float, kind: str):
    """Interpolation-based algorithm: ``ghat(j/c) = sum_n exp(-i (j/c) n 2 pi/N) g_n``
    at ``j = 0 .. c N - 1`` by one FFT of ``g`` zero-padded to ``c N`` (periodic
    in ``j``), then at each node ``omega`` either the nearest grid value
    (``j = floor(c omega + 1/2)``) or the linear interpolant between
    ``j = floor(c omega)`` and ``j + 1``."""
    g = np.asarray(g, dtype=np.complex128)
    N = g.shape[0]
    cN = int(round(c * N))
    assert abs(c * N - cN) < 1e-9
    ghat = np.fft.fft(np.concatenate([g, np.zeros(cN - N, dtype=np.complex128)]))
    x = c * np.asarray(omega, dtype=np.float64)
    if kind == "nearest":
        return ghat[np.mod(np.floor(x + 0.5).astype(np.int64), cN)]
    if kind == "linear":
        j = np.floor(x).astype(np.int64)
        d = x - j
        return (1.0 - d) * ghat[np.mod(j, cN)] + d * ghat[np.mod(j + 1, cN)]
    raise ValueError(kind)


def evaluate(g, omega, kind: str, c: float, K: float = 3.0, alpha: float = 0.0):
    """``sum_n exp(-2 pi i omega n / N) g_n`` by the method ``kind``:
    "direct" (eq. dft), "kb" (the NUFFT algorithm with the Kaiser-Bessel window;
    ``alpha = 0`` selects ``0.98 pi (2c - 1)``), "sinc", "linear" or "nearest"."""
    if kind == "direct":
        return ndft(g, omega)
    if kind == "kb":
        a = alpha if alpha > 0 else 0.98 * np.pi * (2 * c - 1)
        return nufft(g, omega, c, K, a)
    if kind == "sinc":
        return truncated_sinc(g, omega, c, K)
    return interpolated(g, omega, c, kind)
