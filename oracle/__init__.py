"""The oracle: TEST INFRASTRUCTURE ONLY.

A plain, exact CPU implementation of the paper's critical-point tracking (C, with a ctypes binding) and a tiny
pure-Python literal reference.  Only tests/, the smoke check and the benchmark's CPU-baseline leg may import it;
the product path never does.
"""
