"""FP64 CPU oracle for CG-based greedy compressive-sensing recovery.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link
or execute this package: it is used by ``tests/``, by ``__graft_entry__.smoke()``
and by the ``cpu_baseline`` leg of ``bench.py``, and by the script that writes
stored expected values under ``tests/golden/``.

It is a plain, slow, obviously correct restatement of what the recovery
computes, written from the paper (Hsieh, Lu, Pei, "Fast Greedy Approaches for
Compressive Sensing of Large-Scale Signals"):

* ``operator``  - the sensing operator A = D F R of Eq. (7) (Sec. III-A) with
                  F the orthonormal DCT-II and R a +-1 sign flip; dense cosine
                  formula for small N as a second route.
* ``cpf``       - partial complex Fourier sensing of a real signal,
                  A = D FFT R (the D(FFT(x)) operator of Sec. II), with complex
                  measurements and the real-inner-product adjoint.
* ``gram``      - closed-form Gram matrix A_S^T A_S of that operator
                  (a Toeplitz-plus-Hankel form derived from the cosine
                  product-to-sum identity; derived here, not in the paper).
* ``lsq``       - the least-squares step s_S = (A_S^T A_S)^-1 A_S^T y of
                  Sec. II step 3 / Eq. (9), by an explicit pseudo-inverse
                  (dense QR or Cholesky of the Gram).  Where the Gram would
                  not fit in memory an FP64 operator CG to 1e-13 is used.
* ``greedy``    - OMP (Sec. II steps 1-4, Alg. 1), SP and OMPR (named in
                  Sec. IV, restated from their original authors' papers), step
                  by step, with the tie-break rules spelled out.
* ``bruteforce``- exhaustive l0 search (Eq. (3)) on tiny inputs.
* ``adjoint``   - dense FP64 gradient of ||s_hat - t||^2 with respect to y on
                  a frozen support.

Parity status: every function here is pinned by the tests in
``tests/test_oracle_pins.py`` (closed forms, invariants, brute force,
special cases) except the greedy trajectories on noisy data, for which the
paper prints no values: those are "parity unpinned" beyond the invariants
(residual orthogonality on the returned support, exact recovery of
noiseless well-separated inputs, the M = N special case).
"""
from .operator import SRM, dct2_matrix, rdft_matrix  # noqa: F401
from .cpf import CPF  # noqa: F401
from .gram import gram_generator, gram_matrix  # noqa: F401
from .lsq import ls, ls_dense, ls_gram, ls_cg  # noqa: F401
from .greedy import omp, sp, ompr, cosamp, topk_order, argmax_excluding  # noqa: F401
from .bruteforce import l0_bruteforce  # noqa: F401
from .adjoint import adjoint_gradient  # noqa: F401
