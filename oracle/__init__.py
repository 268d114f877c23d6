"""CPU FP64 reference renderer for the DDGS-CT DRR splatting path.

Test infrastructure only: the test suite, the smoke check and the benchmark's
CPU-baseline leg are its only users.  It shares no code with the GPU library.
"""
