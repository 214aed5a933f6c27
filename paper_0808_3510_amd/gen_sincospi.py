"""Coefficients of the float sin(pi s), cos(pi s) used for the node phase
exp(-i pi nu) in the interpolation and spreading kernels.

On |s| <= 1/4:  sin(pi s) ~ s (a0 + a1 u + a2 u^2 + a3 u^3),
                cos(pi s) ~ b0 + b1 u + b2 u^2 + b3 u^3 + b4 u^4,  u = s^2,
fitted by least squares on Chebyshev points of u in [0, 1/16] (relative
error for sin, absolute for cos; near-minimax for such smooth functions).
The kernels reduce nu to s and a quarter-turn count q and rotate.
Run:  python -m paper_0808_3510_amd.gen_sincospi
"""
import numpy as np


def fit(n_sin=4, n_cos=5, pts=400):
    k = np.arange(pts)
    u = (1 / 32) * (1 - np.cos(np.pi * (k + 0.5) / pts))  # Chebyshev points on [0, 1/16]
    s = np.sqrt(u)
    A = np.stack([u ** j for j in range(n_sin)], 1)
    a = np.linalg.lstsq(A, np.where(s > 0, np.sin(np.pi * s) / np.where(s > 0, s, 1), np.pi), rcond=None)[0]
    B = np.stack([u ** j for j in range(n_cos)], 1)
    b = np.linalg.lstsq(B, np.cos(np.pi * s), rcond=None)[0]
    return a, b


def max_errors(a, b, n=200001):
    """Largest errors when evaluated in float32 Horner form over s in [-1/4, 1/4]."""
    s = np.linspace(-0.25, 0.25, n).astype(np.float32)
    u = s * s
    a32, b32 = a.astype(np.float32), b.astype(np.float32)
    ps = a32[-1] * np.ones_like(u)
    for c in a32[-2::-1]:
        ps = ps * u + c
    pc = b32[-1] * np.ones_like(u)
    for c in b32[-2::-1]:
        pc = pc * u + c
    sd = s.astype(np.float64)
    return (float(np.max(np.abs(s * ps - np.sin(np.pi * sd)))), float(np.max(np.abs(pc - np.cos(np.pi * sd)))))


if __name__ == "__main__":
    a, b = fit()
    print("sin:", ", ".join(f"{float(np.float32(x))!r}f" for x in a))
    print("cos:", ", ".join(f"{float(np.float32(x))!r}f" for x in b))
    print("max abs error (float32 evaluation): sin %.3g, cos %.3g" % max_errors(a, b))
