"""FP64 CPU oracle for the randomized PSD projection (Jones & Anderson).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package: only the test-suite, the package smoke
check and the CPU-baseline leg of the benchmark use it.  It shares no code
with the GPU library (no kernels, headers, helpers, tables or constants);
the two meet only through the seeded inputs produced by ``workloads``.

Contents
--------
philox   -- Philox4x32-10 counter-based generator and Box-Muller Gaussians,
            written from the generator's published definition (Salmon,
            Moraes, Dror, Shaw, "Parallel random numbers: as easy as
            1, 2, 3", SC'11).
rnla     -- the method: range finder (Alg. 1), plain randomized projection
            (Alg. 2), scaled randomized projection (Alg. 3), power
            iteration (Alg. 4), minimum-eigenvalue estimate (Alg. 5), the
            exact projection (Thm 1) and the error metrics of Sec. 4.
bounds   -- the expected-error bounds eps1/eps2 (Sec. 3.1), Cor. 1 and
            Prop. 2.
srht     -- the structured (subsampled randomized Hadamard) test matrix, the
            alternative to Gaussian test vectors named in Sec. 3.1.
sdls     -- dual gradient descent for the semidefinite least-squares problem
            (Alg. 6, supplementary SDP section), with the exact, plain or
            scaled projection.

Every function is plain FP64 numpy; LAPACK (through numpy.linalg) supplies
the Householder QR and the symmetric eigensolver as library steps.
"""
from . import philox, srht, rnla, bounds, sdls  # noqa: F401
