"""NUFFT-based Fourier reconstruction for planar photoacoustic imaging on MI355X.

Importing the package loads nothing native; the HIP library is loaded on first
use by :mod:`paper_0808_3510_amd.pat` (which fails loudly if it is missing).
"""
__all__ = ["inputs"]
