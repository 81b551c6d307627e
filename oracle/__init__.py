"""CPU parity oracle for the AES library (test infrastructure only).

Nothing in the GPU library imports this package; only the tests, the smoke check
and the benchmark's CPU-baseline leg do.
"""
