"""CPU oracle for the volume-integral-equation operator and solve.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The GPU library
never calls it and shares no code with it.

Plain, slow, FP64 NumPy code that computes the discrete operator from its
definition:

* ``symbol``       truncated free-space kernel transform and the Fourier symbols
                   of grad div V, (grad div + omega^2) V and curl V
                   (Sections 2-4, eqs. Vo, Todef, Vw, represent_Maxwell).
* ``tables``       the windowed real-space kernel K_m obtained by sampling the
                   symbol on the oversampled frequency grid (Section 5, steps
                   (a)-(c) of the truncated-kernel method).
* ``operator``     contrast H = (a + I)^{-1}(a - I) (eq. rhodef), the direct
                   convolution sum, FFT routes, the matvec of eqs. intLap,
                   intH (sign as derived), contraction_Maxwell(_reduced).
* ``solve``        dense LU for tiny grids, plain GMRES, Bi-CGStab, Neumann series.
* ``closed_forms`` Gaussian-density potentials and the dielectric sphere.
"""
