"""FP64 CPU oracle for the modal bispectrum estimator (Fergusson & Shellard,
"Optimal Polyspectra Estimation").

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link anything in this package: only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the
HIP library; the only common dependency is ``modal_inputs`` (seeded input
data, no estimator arithmetic).

Every function is the plain definition of what the GPU path computes, written
in numpy float64 (library primitives used as single steps: matrix products,
``numpy.fft``, ``numpy.linalg``).  Pins against closed forms, the Wigner-3j
Gaunt integral, brute-force triple sums, Parseval, finite differences and the
bivector closed forms live in ``tests/test_oracle_*.py``; ``lowrank`` holds the
low-rank (bivector / principal-component) covariance of Sec. III B, ``shapes``
the theory mode coefficients of separable bispectra (eq. abispect), ``power``
the modal power-spectrum estimator of Sec. IV, ``trispectrum`` the modal
trispectrum estimator of Sec. IV.

Functions whose parity is not pinned by anything but themselves say so in
their docstring ("parity unpinned").
"""
from . import grid, legendre, wigner, modal, closed_forms, sims, lowrank, shapes, power, trispectrum, frame  # noqa: F401
