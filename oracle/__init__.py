"""FP64 CPU oracle for the D3Q7 compressible Navier-Stokes-Fourier scheme.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import anything under this package.  It shares no code
with the HIP library and imports nothing from it; the only inputs it shares
with the HIP path are the seeded generators of the ``workloads`` package.

Modules
-------
lbm          vectorised FP64 scheme (Eq. (2), Section 2.2, Eqs. (3)-(6))
brute        independent per-cell loop transcription, for tiny grids
diagnostics  Eq. (7) averages with spectral derivatives, conservation sums
exact        exact Sod Riemann solution, Becker closed form, norms, thickness
characteristics  numerical flux-Jacobian eigenvalues of the declared system
"""
