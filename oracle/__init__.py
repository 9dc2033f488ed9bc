"""CPU FP64 oracle for the NFFT (test infrastructure only).

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
import this package.  The HIP library never does, and this package imports
nothing from it.
"""
