"""CPU oracle for the SSA hot path.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the CPU-baseline
leg of the benchmark.  The product package never imports anything from here, and nothing
here imports the product package or its compiled library.
"""
