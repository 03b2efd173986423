"""CPU oracle for the ChASE hot path: test infrastructure, not product code.

Only the test suite, the package's smoke check and the benchmark's CPU
baseline leg import this package.  It shares no code with the HIP path
(neither imports the other); both take their inputs from the seeded
generators in ``paper_2006_08498_amd.synth``.

Contents:

* ``eig``    -- the lowest eigenpairs of a Hermitian matrix, the plain
               definition of the solver's result (C library ``eigh.c``:
               Householder tridiagonalisation + implicit symmetric QR).
* ``steps``  -- the solver's intermediate steps in FP64 numpy (Chebyshev
               filter recurrence, spectral bounds by Lanczos, convergence
               rate of the supplement's Eq. S1, degrees, QR, Rayleigh-Ritz,
               residuals, locking) for step-level parity tests.
* ``brute``  -- exact eigenvalues of tiny Gaussian-integer Hermitian
               matrices by Sylvester inertia counts in rational arithmetic.

Parity pins live in ``tests/`` (``-m "not gpu"``).  Functions whose result
no independent fact fixes are marked "parity unpinned" in their docstring.
"""
