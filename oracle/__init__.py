"""FP64 CPU oracle for the view-interpolation network — test infrastructure.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package. It shares no code with the GPU library.
"""
