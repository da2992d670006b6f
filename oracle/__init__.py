"""Plain FP64 CPU oracle for the interlaced, order-p Fourier-space estimators.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
path (``paper_1512_07295_amd``) and imports nothing from it.

It follows Sefusatti, Crocce, Scoccimarro & Couchman, "Accurate Estimators of
Correlation Functions in Fourier Space" (arXiv:1512.07295), step by step and
in the paper's order:

* ``kernels``   - the order-p B-spline assignment kernels (Sec. 2.3, NGP/CIC/
                  TSC/PCS) and their Fourier window (eq. intkerFT).
* ``assign``    - wrap, locate and deposit onto the primary grid and onto the
                  grid shifted by H/2 (eq. delgrid, Sec. 3.1).
* ``spectrum``  - FFT, interlace combination (eq. intdelta), window
                  deconvolution (eq. windowcorrection) and |k|-shell binning
                  into P(k) (eq. ps and the direct-summation estimator).
* ``bispectrum``- the FFT-shell bispectrum estimator (eqs. Best, VBest, Best2,
                  IntI).
* ``adjoint``   - the exact derivative of the binned P(k) with respect to the
                  particle positions (not in the paper; the derivative of the
                  forward computed here).
* ``direct``    - direct-summation density (eq. deltaDS) and the footprint DFT.
* ``native``    - the deposit and footprint DFT as plain C loops (same
                  arithmetic) for inputs too large for numpy.
* ``theory``    - closed forms used as pins: aliased white-noise spectra,
                  the residual factor F_res (eqs. res, Fres, res1Di, res1Dnoi).

All floating point is float64.  Readings of points where the paper is silent
or garbled are listed in each function's docstring.

Parity status: every function here is pinned by a ``-m "not gpu"`` test
against something other than itself (closed forms, brute force on tiny
inputs, library routines for special cases); none is "parity unpinned".
"""

from . import kernels, assign, spectrum, bispectrum, adjoint, direct, theory, native  # noqa: F401
from .spectrum import power  # noqa: F401
from .bispectrum import bispectrum as bispectrum_fn  # noqa: F401
