"""CPU FP64 oracle for the planar photoacoustic Fourier reconstruction.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link
or execute anything in this package: only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the
HIP library: node positions, weights, transforms and scaling are written out
here from the paper's definitions, independently of ``paper_0808_3510_amd``.

Modules
-------
``recon``  direct Fourier reconstruction R (Section 4, eqs. fft-1a, fft-2,
           fft-0, fft-1; "direct Fourier algorithm" of Section 4), its
           transpose, the spectral forward model A and its transpose, all by
           direct nonuniform DFT sums.
``kb``     the Kaiser-Bessel window and its Fourier transform (Section 3.2).
``nufft``  the paper's NUFFT (Section 3.1, Proposition on the NUFFT identity
           and the NUFFT algorithm), which pins the readings of its constant
           and phase against the direct sum, and the other evaluations of the
           nonuniform sums that Section 4 compares (truncated sinc, linear
           and nearest interpolation of the oversampled FFT).
``cutoff`` the smooth cut-off w_cut of the partial-data model (eq. data-part,
           Section 5) by nested quadrature of its defining convolution.

Parity status: every function is pinned by a test under ``tests/`` against a
closed form, a printed value of the paper, a library routine on a special case
or a transpose identity; none is "parity unpinned".
"""
from . import cutoff, kb, nufft, recon  # noqa: F401
