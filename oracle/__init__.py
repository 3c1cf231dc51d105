"""FP64 CPU oracle of the multi-scale semi-Lagrangian LBM step.

Test infrastructure only: imported by the tests, the smoke check and the
benchmark's CPU baseline, never by the product path.
"""
