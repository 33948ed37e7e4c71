"""Host-side size limits of the GPU library (CPU only): interaction lists and
walk frontiers beyond what the int32 CSR arrays index are refused before any
kernel indexes them (the walk then returns FMM_EUNSUPPORTED)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = r"""
#include "fmm_limits.h"
#include <cstdio>
int main() {
  using namespace fmm;
  int bad = 0;
  bad += !walk_list_fits(0);
  bad += !walk_list_fits(24000000);
  bad += !walk_list_fits(kMaxWalkEntries);
  bad += walk_list_fits(kMaxWalkEntries + 1);
  bad += walk_list_fits(0x7fffffffLL);
  bad += walk_list_fits(0x80000000LL);      // a 32-bit counter would have wrapped here
  bad += walk_list_fits(-1);
  bad += walk_list_fits(1LL << 40);
  // regrown capacities of a list that fits stay below 2^32 entries
  bad += (2 * kMaxWalkEntries + 64) >= (1LL << 32);
  std::printf("%d\n", bad);
  return bad;
}
"""


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_walk_list_limit(tmp_path):
    src = tmp_path / "lim.cpp"
    src.write_text(DRIVER)
    exe = str(tmp_path / "lim")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-Xlinker", "--no-as-needed",
                           "-I" + os.path.join(ROOT, "paper_2012_02207_amd", "csrc"), str(src), "-o", exe])
    r = subprocess.run([exe], capture_output=True, text=True)
    assert r.returncode == 0 and r.stdout.strip() == "0", r.stdout + r.stderr
