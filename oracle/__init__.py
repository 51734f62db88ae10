"""Oracle for the shifted Newton-Schulz reflector library.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
``bench.py``'s CPU-baseline leg may import, call or link anything here.  The
product library under ``paper_2605_24840_amd/`` never does, and the oracle
imports nothing from it: the two share no code.

Contents
--------
``jacobi.c``  plain FP64 cyclic Jacobi eigensolver (C, OpenMP).
``oracle.py`` the exact reflector R_k = I - 2 Q_k Q_k^T (Prop. 2.1), the
              shifted sign sgn(H - sI), the plain FP64 Newton-Schulz iterates
              (eq. NS) and their split-BF16 arithmetic model, the scalar
              polynomials p_m (eq. pm) and the error
              recurrence (Prop. 3.6), the midpoint rule (Prop. 4.1) and the
              Prop. 4.2 admissibility test, reference certificate values, and
              the block-Lanczos estimate of the gap endpoints, error radius,
              midpoint shift and spectral radius (section 4.3) with its
              SplitMix64 start block.
``build.py``  compiles ``jacobi.c`` into ``liboracle_jacobi.so``.
"""
from .oracle import *  # noqa: F401,F403
