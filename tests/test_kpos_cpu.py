"""Host check of the implicit-GEMM kernels' incremental K position.

Both GEMM kernels track the filter tap (r, s) and input channel of each
lane's 16-byte K segment from one K-tile to the next (struct KPos in
conv.hip) instead of dividing at every K-tile.  The struct is compiled for
the host and compared, at every K-tile including those past K, with the
direct decoding of the packed K order (tap-major, and channel-block-major
with 128-byte blocks), for every dtype's segment size, 128- and 64-byte
K-tiles, channel counts from 4 to 1024, filters up to 4x3 and every start
K-tile a split can have.  No GPU."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DRIVER = os.path.join(ROOT, "tests", "native", "kpos_check.cpp")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_incremental_k_position_matches_direct_decoding(tmp_path):
    src = open(os.path.join(ROOT, "paper_1811_03882_amd", "csrc", "conv.hip")).read()
    struct = re.search(r"struct KPos \{.*?\n\};", src, flags=re.S).group(0)
    (tmp_path / "kpos.h").write_text("#define __device__\n#define __forceinline__ inline\n" + struct + "\n")
    exe = tmp_path / "kpos_check"
    subprocess.run(["g++", "-O1", "-std=c++17", "-I", str(tmp_path), DRIVER, "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    print(out.stdout)
    assert out.returncode == 0, out.stdout
    assert int(out.stdout.split()[1]) > 1000000
