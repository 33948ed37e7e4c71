"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU):
`oracle/sanitize_main.c` runs every stage of the pass, the direct sum and the
operator building blocks on small random and degenerate inputs; any
out-of-bounds access, leak or undefined operation aborts the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_clean_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "orc_san")
    odir = os.path.join(ROOT, "oracle")
    subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", "-ffp-contract=off", "-fopenmp", "-std=c99",
                           "-I" + odir, "-o", exe, os.path.join(odir, "sanitize_main.c"),
                           os.path.join(odir, "fmm_oracle.c"), "-lm"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="4")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ok" in r.stdout
