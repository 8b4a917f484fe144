"""FP64 CPU oracle of the ADG-AT right-hand side and time loop.

TEST INFRASTRUCTURE ONLY: used by tests/, the smoke entry and the benchmark's
CPU-baseline leg. The GPU library does not import it.
"""
