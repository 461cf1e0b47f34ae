"""FP64 CPU oracle for the synchrotron-emission path (test infrastructure only).

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import it; the product path never does.
"""
