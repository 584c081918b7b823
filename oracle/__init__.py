"""CPU oracle of the binocular 2DGS frame path.

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and
the CPU-baseline leg of the benchmark, never by the product path.
"""
