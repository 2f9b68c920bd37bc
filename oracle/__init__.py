"""FP64 CPU oracle for the TNLM operator.

TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the CPU
baseline leg of the benchmark may import it. The product library never
does, and shares no code with it.

  oracle.oracle  ctypes shim over tnlm_oracle.c (C99 + OpenMP, FP64)
  oracle.brute   pure-Python/numpy brute force for tiny grids
"""
