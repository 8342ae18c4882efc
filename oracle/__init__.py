"""FP64 CPU oracle for the low-rank ChebyshevT matrix-equation solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library; the only common dependency is the seeded input generator
``workloads`` (which contains none of the method's arithmetic).

Contents (all float64, NumPy/SciPy, deliberately plain and unoptimised):

* ``lowrank``   - the plain definition of the result: the operator
                  L(X) = sum_i K_i X D_i, its Kronecker (vector) form and
                  column-wise direct solves, the relative residual, and the
                  truncation operator T (QR + SVD, rank cap + relative tail).
* ``chebyshev`` - the mean-based preconditioner, the Chebyshev interval and
                  the preconditioned, truncated Chebyshev iteration (ChebyshevT).
* ``driver``    - little-endian ordering, subset sizes, upper median index and
                  the Newton-on-subset driver (Algorithm 1).
* ``mlp``       - forward, backward and Adam for the surrogate network used as
                  a learned initial guess (not part of the paper).

Functions whose result is not fixed by an independent pin say
"parity unpinned" in their docstring.
"""
