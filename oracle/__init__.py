"""FP64 CPU oracle of the SALE Lagrange + remap step (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package. It never imports the HIP package and shares no code
with it.
"""
