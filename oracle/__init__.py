"""FP64 CPU oracle of the vectorized PSDP method (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package. It shares no code with the HIP library and imports
nothing from it.
"""
