"""FP64 CPU oracle for SpAMM and SP2.

TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the
benchmark's CPU-baseline leg may import anything from here.  The device
library neither imports nor links it, and it shares no code with it.
"""
