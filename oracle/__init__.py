"""CPU oracle for Compact-Table propagation (test infrastructure only).

Loaded by the tests, the smoke check and the CPU-baseline leg of the
benchmark; the GPU library never imports, links or calls it.
"""
