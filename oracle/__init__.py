"""Oracle for the permanent hot path.  TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct CPU implementations of what the GPU path
computes, written from the paper (arXiv 2602.10141, "Permanents of matrix
ensembles: computation, distribution, and geometry"):

* ``native``     -- ctypes front end of ``ryser.c``: single-threaded Ryser
                    (Gray order, Kahan sums) over C, R and F_p, plus directly
                    evaluated Glynn-term range sums (Sec. 1, Sec. 1 Note,
                    Sec. 2.1-2.2).
* ``reference``  -- brute force over S_n and Laplace expansion in exact
                    Python arithmetic (the definition, Sec. 1).
* ``crt``        -- primes p = 1 (mod n), primitive n-th roots of unity,
                    Schur residue matrices, the textbook Chinese-remainder
                    lift to a signed integer, and the exact Schur count in the
                    group ring Z[x]/(x^n - 1) (Sec. 2.1).

Only ``tests/``, the package smoke check and the benchmark's CPU-baseline leg
may import this package.  It shares no code with the HIP path and imports
nothing from it.
"""
from . import native, reference, crt  # noqa: F401
