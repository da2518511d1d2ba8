"""FP64 CPU oracle for the implicit-Euler heat solver and its discrete adjoint.

TEST INFRASTRUCTURE ONLY. The test suite, the smoke check and the CPU-baseline
leg of the benchmark call it; the product library never does, and the two
share no code. ``heat`` wraps the matrix-free C implementation
(``heat_oracle.c``); ``dense_ref`` is an independent dense NumPy assembly
used to pin it on tiny grids.
"""
