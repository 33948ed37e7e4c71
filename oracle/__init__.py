"""CPU oracle for the collisional FMM force pass -- test infrastructure only.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark use
this package; the GPU library never imports or links it.
"""
from .oracle import (Oracle, direct, regular, irregular, m2l_direct, m2l_rotated, m2m, l2l,
                     l2p, p2m, pk, swap_table, factorials, threads, build, lib_path)

__all__ = ["Oracle", "direct", "regular", "irregular", "m2l_direct", "m2l_rotated", "m2m",
           "l2l", "l2p", "p2m", "pk", "swap_table", "factorials", "threads", "build", "lib_path"]
