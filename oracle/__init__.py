"""FP64 CPU oracle of the SteepGS hot path (test infrastructure only).

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may use
this package; the product path must never import it.
"""
