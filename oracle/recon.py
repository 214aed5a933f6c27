"""Direct Fourier reconstruction, its transpose, and the spectral forward model.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain FP64 NumPy; the
nonuniform sums are evaluated directly (no NUFFT, no kernel, no tables shared
with the HIP library).

Geometry (a plain dict): ``n1, n2`` detectors per transverse axis (``n2 = 1``
for the 2D line geometry), ``nt`` time samples, ``nz`` depth samples, spacings
``dx, dt, dz`` and speed of sound ``vs``.  Arrays are ``(n1, n2, nt)`` /
``(n1, n2, nz)`` (2D arrays ``(n1, nt)`` / ``(n1, nz)`` are accepted), last axis
fastest.  Frequencies ``k_i`` run over ``[-n_i/2, n_i/2)`` and ``l`` over
``[-nz/2, nz/2)``.

Reconstruction R (Section 4, the direct Fourier algorithm):

* eq. (fft-1a): ``G[k, n] = sum_m exp(-2 pi i k.m / N) p[m, n]``;
* eq. (fft-2):  ``Ghat[k, l] = sum_n exp(-2 pi i nu_{k,l} n / nt) G[k, n]`` with
  the nodes of eq. (dft-2d), here in time-bin units for unequal grids,
  ``nu_{k,l} = sign(l) nt dt vs |K| / (2 pi)``, ``K = (2 pi k_i / (n_i dx),
  2 pi l / (nz dz))``, and ``sign(0) = 0``;
* eq. (fft-0):  ``Fhat = W Ghat`` with the Jacobian weight of eq. (inv),
  ``W = 2 vs (dt/dz) |K_z| / |K|``, read with ``K_z`` (the depth frequency) in
  the numerator, and ``W = 0`` at ``l = 0``;
* eq. (fft-1):  ``f = Re( inverse DFT over (k, l) of Fhat )`` with the
  ``1 / (n1 n2 nz)`` normalisation.

Forward model A: the semi-discrete solution of the wave problem of Section 2
on the periodic sampling grid: every plane wave ``exp(i K.x)`` of the initial
pressure evolves as ``cos(vs |K| t)``, so the trace on ``y = 0`` at ``t = n dt`` is
``p[m, n] = Re( (1/(n1 n2)) sum_k exp(2 pi i k.m/N) (1/nz) sum_l F[k, l]
cos(2 pi nu+_{k,l} n / nt) )`` with ``F`` the DFT of ``f`` over all axes and
``nu+ = |nu|``.
"""
from __future__ import annotations

import numpy as np


def int_freqs(n: int) -> np.ndarray:
    """Integer frequencies in DFT storage order: 0..n/2-1, -n/2..-1."""
    return np.rint(np.fft.fftfreq(n) * n).astype(np.int64)


def _as3(a, g):
    a = np.asarray(a, dtype=np.float64)
    if a.ndim == 2:
        assert g["n2"] == 1
        return a[:, None, :], True
    return a, False


def wavenumbers(k1, k2, l, g):
    """``(|K_x|^2, K_z)`` in physical units for integer frequencies."""
    kx2 = (2 * np.pi * k1 / (g["n1"] * g["dx"])) ** 2 + (2 * np.pi * k2 / (g["n2"] * g["dx"])) ** 2
    kz = 2 * np.pi * np.asarray(l, dtype=np.float64) / (g["nz"] * g["dz"])
    return kx2, kz


def node_plus(k1, k2, l, g):
    """``nu+ = nt dt vs |K| / (2 pi)``: the modulus of the node, time-bin units."""
    kx2, kz = wavenumbers(k1, k2, l, g)
    return g["nt"] * g["dt"] * g["vs"] * np.sqrt(kx2 + kz * kz) / (2 * np.pi)


def nodes(k1, k2, l, g):
    """Signed nodes ``nu_{k,l} = sign(l) nu+`` of eq. (dft-2d)."""
    return np.sign(np.asarray(l, dtype=np.float64)) * node_plus(k1, k2, l, g)


def weights(k1, k2, l, g):
    """Jacobian weight ``2 vs (dt/dz) |K_z| / |K|``, zero at ``l = 0``."""
    kx2, kz = wavenumbers(k1, k2, l, g)
    kabs = np.sqrt(kx2 + kz * kz)
    with np.errstate(invalid="ignore", divide="ignore"):
        w = 2.0 * g["vs"] * (g["dt"] / g["dz"]) * np.abs(kz) / kabs
    return np.where(np.asarray(l) == 0, 0.0, w)


def _phase(nu, nt):
    """``exp(-2 pi i nu n / nt)`` for all (node, n), argument reduced mod nt."""
    n = np.arange(nt)
    return np.exp(-2j * np.pi * np.mod(np.outer(nu, n), nt) / nt)


def _cos(nu, nt):
    n = np.arange(nt)
    return np.cos(2 * np.pi * np.mod(np.outer(nu, n), nt) / nt)


def _groups(g):
    """Lines grouped by ``(|k1|, |k2|)``: the nodes and weights depend on k
    only through ``k1^2`` and ``k2^2``."""
    groups = {}
    for i1, k1 in enumerate(int_freqs(g["n1"])):
        for i2, k2 in enumerate(int_freqs(g["n2"])):
            groups.setdefault((abs(int(k1)), abs(int(k2))), []).append((i1, i2))
    return {key: (np.array([a for a, _ in v]), np.array([b for _, b in v]))
            for key, v in groups.items()}


def transverse_dft(p, g):
    """eq. (fft-1a): full complex transverse spectrum ``G[k1, k2, n]``."""
    p3, _ = _as3(p, g)
    return np.fft.fft2(p3, axes=(0, 1))


def spectrum(p, g):
    """``Fhat[k1, k2, l] = W Ghat`` for every line (DFT storage order)."""
    G = transverse_dft(p, g)
    l = int_freqs(g["nz"])
    out = np.empty((g["n1"], g["n2"], g["nz"]), dtype=np.complex128)
    for (a, b), (i1, i2) in _groups(g).items():
        E = _phase(nodes(a, b, l, g), g["nt"])           # (nz, nt)
        out[i1, i2, :] = (G[i1, i2, :] @ E.T) * weights(a, b, l, g)
    return out


def spectrum_lines(p, g, lines):
    """``Fhat`` for selected signed lines ``[(k1, k2), ...]`` only:
    returns ``(len(lines), nz)`` in DFT storage order of ``l``."""
    G = transverse_dft(p, g)
    l = int_freqs(g["nz"])
    out = np.empty((len(lines), g["nz"]), dtype=np.complex128)
    for i, (k1, k2) in enumerate(lines):
        E = _phase(nodes(k1, k2, l, g), g["nt"])
        out[i] = (E @ G[k1 % g["n1"], k2 % g["n2"], :]) * weights(k1, k2, l, g)
    return out


def adjoint_lines(q, g, lines):
    """The transverse spectrum of R^T q on selected signed lines, before the
    real part: ``X[k, n] = (1/nz) sum_l exp(+2 pi i nu_{k,l} n / nt) W_{k,l}
    Q[k, l]`` with ``Q`` the DFT of ``q`` over all axes; returns
    ``(len(lines), nt)``.  (R^T q itself is ``Re(IDFT_x(X))``, so the DFT over
    x of R^T q at k is ``(X[k] + conj(X[-k])) / 2``.)"""
    q3, _ = _as3(q, g)
    Q = np.fft.fftn(q3, axes=(0, 1, 2))
    l = int_freqs(g["nz"])
    out = np.empty((len(lines), g["nt"]), dtype=np.complex128)
    for i, (k1, k2) in enumerate(lines):
        E = _phase(nodes(k1, k2, l, g), g["nt"])           # (nz, nt)
        out[i] = ((Q[k1 % g["n1"], k2 % g["n2"], :] * weights(k1, k2, l, g)) @ np.conj(E)) / g["nz"]
    return out


def forward_lines(f, g, lines):
    """The transverse spectrum of A f on selected signed lines, before the
    real part: ``P[k, n] = (1/nz) sum_l F[k, l] cos(2 pi nu+_{k,l} n / nt)``,
    ``(len(lines), nt)``."""
    f3, _ = _as3(f, g)
    F = np.fft.fftn(f3, axes=(0, 1, 2))
    l = int_freqs(g["nz"])
    out = np.empty((len(lines), g["nt"]), dtype=np.complex128)
    for i, (k1, k2) in enumerate(lines):
        C = _cos(node_plus(k1, k2, l, g), g["nt"])
        out[i] = (F[k1 % g["n1"], k2 % g["n2"], :] @ C) / g["nz"]
    return out


def forward_adjoint_lines(p, g, lines):
    """The spectrum of A^T p on selected signed lines, before the real part:
    ``Y[k, l] = sum_n cos(2 pi nu+_{k,l} n / nt) P[k, n]`` with ``P`` the DFT of
    ``p`` over x, ``(len(lines), nz)``; the DFT over all axes of A^T p at
    ``(k, l)`` is ``(Y[k, l] + conj(Y[-k, -l])) / 2``."""
    P = transverse_dft(p, g)
    l = int_freqs(g["nz"])
    out = np.empty((len(lines), g["nz"]), dtype=np.complex128)
    for i, (k1, k2) in enumerate(lines):
        C = _cos(node_plus(k1, k2, l, g), g["nt"])
        out[i] = C @ P[k1 % g["n1"], k2 % g["n2"], :]
    return out


def reconstruct(p, g):
    """R: detector data ``p`` -> image ``f`` (direct Fourier reconstruction)."""
    _, flat = _as3(p, g)
    f = np.real(np.fft.ifftn(spectrum(p, g), axes=(0, 1, 2)))
    return f[:, 0, :] if flat else f


def reconstruct_with(p, g, kind: str, c: float, K: float = 3.0, alpha: float = 0.0):
    """R with the nonuniform sums of eq. (fft-2) evaluated by one of the
    methods Section 4 compares (``oracle.nufft.evaluate``: "kb", "sinc",
    "linear", "nearest"; "direct" gives ``reconstruct``), for the
    accuracy-against-time study."""
    from .nufft import evaluate
    _, flat = _as3(p, g)
    G = transverse_dft(p, g)
    l = int_freqs(g["nz"])
    out = np.empty((g["n1"], g["n2"], g["nz"]), dtype=np.complex128)
    for (a, b), (i1, i2) in _groups(g).items():
        nu = nodes(a, b, l, g)
        w = weights(a, b, l, g)
        for x, y in zip(i1, i2):
            out[x, y, :] = evaluate(G[x, y, :], nu, kind, c, K, alpha) * w
    f = np.real(np.fft.ifftn(out, axes=(0, 1, 2)))
    return f[:, 0, :] if flat else f


def reconstruct_adjoint(q, g):
    """R^T (transpose for the real inner product): image-shaped ``q`` ->
    data-shaped output, ``Re( D_x^H T^H (W . D_xz q) ) / (n1 n2 nz)`` with
    ``(T^H v)_n = sum_l exp(+2 pi i nu_l n / nt) v_l``."""
    q3, flat = _as3(q, g)
    Q = np.fft.fftn(q3, axes=(0, 1, 2))
    l = int_freqs(g["nz"])
    X = np.empty((g["n1"], g["n2"], g["nt"]), dtype=np.complex128)
    for (a, b), (i1, i2) in _groups(g).items():
        E = _phase(nodes(a, b, l, g), g["nt"])           # (nz, nt)
        X[i1, i2, :] = (Q[i1, i2, :] * weights(a, b, l, g)) @ np.conj(E)
    out = np.real(np.fft.ifft2(X, axes=(0, 1))) / g["nz"]
    return out[:, 0, :] if flat else out


def forward(f, g):
    """A: image ``f`` -> detector data, the cosine form of the spectral solution."""
    f3, flat = _as3(f, g)
    F = np.fft.fftn(f3, axes=(0, 1, 2))
    l = int_freqs(g["nz"])
    P = np.empty((g["n1"], g["n2"], g["nt"]), dtype=np.complex128)
    for (a, b), (i1, i2) in _groups(g).items():
        C = _cos(node_plus(a, b, l, g), g["nt"])          # (nz, nt)
        P[i1, i2, :] = (F[i1, i2, :] @ C) / g["nz"]
    out = np.real(np.fft.ifft2(P, axes=(0, 1)))
    return out[:, 0, :] if flat else out


def forward_adjoint(p, g):
    """A^T: data ``p`` -> image-shaped output,
    ``Re( IDFT_{x,z}( sum_n cos(2 pi nu+ n / nt) P[k, n] ) )``, ``P = D_x p``."""
    p3, flat = _as3(p, g)
    P = np.fft.fft2(p3, axes=(0, 1))
    l = int_freqs(g["nz"])
    Y = np.empty((g["n1"], g["n2"], g["nz"]), dtype=np.complex128)
    for (a, b), (i1, i2) in _groups(g).items():
        C = _cos(node_plus(a, b, l, g), g["nt"])
        Y[i1, i2, :] = P[i1, i2, :] @ C.T
    out = np.real(np.fft.ifftn(Y, axes=(0, 1, 2)))
    return out[:, 0, :] if flat else out


def forward_padded(f, g, pad_x: int, nz_pad: int):
    """A evaluated on a zero-padded grid and cropped back to the detectors, so
    that no periodic image of the object reaches a detector within the
    recording time (needs ``pad_x >= vs nt dt / dx`` on each side of every
    padded transverse axis and ``nz_pad dz >= vs nt dt + nz dz``)."""
    f3, flat = _as3(f, g)
    n1, n2, nz = f3.shape
    gp = dict(g)
    gp["n1"] = n1 + 2 * pad_x
    gp["n2"] = n2 + 2 * pad_x if n2 > 1 else 1
    gp["nz"] = nz_pad
    o2 = pad_x if n2 > 1 else 0
    big = np.zeros((gp["n1"], gp["n2"], nz_pad))
    big[pad_x:pad_x + n1, o2:o2 + n2, :nz] = f3
    pbig = forward(big, gp)
    p = pbig[pad_x:pad_x + n1, o2:o2 + n2, :]
    return p[:, 0, :] if flat else p
