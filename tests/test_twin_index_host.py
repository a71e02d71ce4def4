"""The exchange-fold index arithmetic of the library (csrc/internal.h), built
as host code: every grouped fast path of the kernels (twin groups of 4, 8 and
16 entries, the member positions the folded kernels read, the runs the folded
sigma = 4 sweep reads with one vector load, the groups the R pass skips or
reads whole) agrees entry by entry with the per-entry rule, for every stored
index at l = 2 .. 10 (sigma = d = 2), 2 .. 7 (d = 3) and 2 .. 5 (sigma = 4),
and for 2^18 hashed groups (plus the first and last) at l = 11 .. 17,
8 .. 12 and 6 .. 9, where stored indices pass 2^31 and 2^32 (up to 2^35).  The packed
layout's arithmetic (packed_index, packed_tuple, packed_group): every code
in range, the representative in the tuple's orbit with the same code, every
used code the code of its representative and as many used codes as orbits,
regular groups at consecutive codes, for every tuple at l = 2 .. 10 and for
2^18 hashed groups at l = 11 .. 18 (codes past 2^32).  No GPU is used."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def test_grouped_twin_paths_agree_with_the_per_entry_rule(tmp_path):
    if not (os.path.exists(HIPCC) or shutil.which(HIPCC)):
        pytest.skip("hipcc not found")
    exe = tmp_path / "twin_index"
    src = tmp_path / "twin_index.hip"  # hipcc treats .hip as HIP source; only host code runs
    shutil.copy(os.path.join(ROOT, "tests", "host", "twin_index.cpp"), src)
    build = subprocess.run([HIPCC, "-O1", "-std=c++17", "--offload-arch=gfx950",
                            "-I" + os.path.join(ROOT, "include"),
                            "-I" + os.path.join(ROOT, "paper_2407_10925_amd", "csrc"),
                            str(src), "-o", str(exe)], capture_output=True, text=True)
    assert build.returncode == 0, build.stderr[-2000:]
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert run.returncode == 0, run.stdout[-2000:]
    assert run.stdout.startswith("ok")
