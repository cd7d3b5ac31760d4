"""Plain FP64 CPU oracle of the overlapping-domain-decomposition preconditioner.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call,
link or execute anything in this package: only the tests, the smoke check
and the benchmark's CPU-baseline leg use it.  It shares no code with the HIP
implementation; both sides receive their inputs from the ``synth`` module.

Each function cites the passage of Chen & Biros, "Overlapping domain
decomposition preconditioner for integral equations" (arXiv 2108.12574) it
follows.  The code is written for clarity, not speed: dense numpy/scipy
primitives (matmul, Cholesky, triangular solves) serve as steps, and the one
O(N^2) dense matvec is a plain C double loop (``oracle/c/matvec.c``).

Parity status of each function is stated in its docstring; the one result
with several correct answers (the skeleton choice of an ID) is compared
through the preconditioner apply and the PCG solution instead.
"""
