"""FP64 CPU oracle of the spherical surfel range-image renderer.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the smoke check and the benchmark's
CPU-baseline leg.  The product package never imports it and shares no code with it.
"""
