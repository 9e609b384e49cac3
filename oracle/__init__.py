"""FP64 CPU oracle of the implicit mover and moment gathering.

Test infrastructure only: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.
"""
