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


def _check_layout(tmp_path, cname, pystruct):
    """field names, offsets and size of the C struct `cname` (include/fmm.h, as
    the C compiler lays it out) against the ctypes structure"""
    import ctypes
    import shutil
    import subprocess
    import pytest
    txt = open(os.path.join(ROOT, "include", "fmm.h")).read()
    body = txt.split("} " + cname + ";")[0].rsplit("typedef struct {", 1)[1]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    names = []
    for decl in re.findall(r"\b(?:int|int64_t|int32_t|double|size_t)\s+([a-z_0-9, ]+);", body):
        names += [d.strip() for d in decl.split(",")]
    assert [f[0] for f in pystruct._fields_] == names
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / f"layout_{cname}.c"
    prints = "".join(f'  printf("%zu\\n", offsetof({cname}, {n}));\n' for n in names)
    src.write_text("#include <stdio.h>\n#include <stddef.h>\n#include \"fmm.h\"\n"
                   f"int main(void) {{\n{prints}  printf(\"%zu\\n\", sizeof({cname}));\n"
                   "  return 0;\n}\n")
    exe = tmp_path / f"layout_{cname}"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True,
                                          text=True).stdout.split()]
    assert got == [getattr(pystruct, n).offset for n in names] + [ctypes.sizeof(pystruct)]


def test_params_layout_matches_header(tmp_path):
    """The Python Params structure has the field names, offsets and size of
    fmm_params as the C compiler lays it out from include/fmm.h, and
    fmm_default_params (host code only) fills the defaults the header states."""
    from paper_2012_02207_amd import fmm
    _check_layout(tmp_path, "fmm_params", fmm.Params)
    p = fmm.default_params()
    assert (p.p, p.err_tol, p.theta, p.theta_est, p.n_leaf) == (10, 1e-7, 1.0, 1.0, 64)
    assert (p.check_inputs, p.root_levels, p.m2l_waves, p.p2p_groups, p.p2p_start) == (0, 3, 1, 0, 0)


def test_stats_layout_matches_header(tmp_path):
    """The same for fmm_stats_t and the Python Stats structure."""
    from paper_2012_02207_amd import fmm
    _check_layout(tmp_path, "fmm_stats_t", fmm.Stats)
