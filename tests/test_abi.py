"""The C-ABI library loads and exports every function include/fmm.h declares
(no compute calls: runs without a GPU); its swap and factorial tables equal the
oracle's, which come from an independent generator."""
import os
import re

import numpy as np

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "fmm.h")).read()
    return sorted(set(re.findall(r"\b(fmm_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    import ctypes
    from paper_2012_02207_amd import fmm
    lib = fmm.load_library()
    names = _declared()
    assert len(names) >= 12
    for s in names:
        assert hasattr(lib, s), s
    assert set(names) == set(fmm.SYMBOLS)
    assert lib.fmm_strerror(0) == b"ok"


def _parse_table(txt, name):
    body = txt.split(name)[1].split("};")[0]
    body = re.sub(r"//[^\n]*", "", body.split("{", 1)[1])
    return np.array([float.fromhex(t) if "0x" in t else float(t)
                     for t in re.split(r"[,\s]+", body) if t])


def test_gpu_tables_equal_oracle_tables():
    txt = open(os.path.join(ROOT, "paper_2012_02207_amd", "csrc", "fmm_tables.h")).read()
    sw = _parse_table(txt, "fmm_swap_table[")
    off = 0
    for n in range(31):
        d = 2 * n + 1
        assert np.array_equal(sw[off:off + d * d].reshape(d, d), oracle.swap_table(n)), n
        off += d * d
    assert off == len(sw)
    fa = _parse_table(txt, "fmm_fact_table[")
    assert np.array_equal(fa, oracle.factorials())
