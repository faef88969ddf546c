"""The XCD-aware block numbering of the SpMV-type kernels (host check).

Workgroup (b, y) of a grid G blocks wide runs on XCD (y G + b) mod 8.  The
kernels renumber their blocks with xcd_rank so that each XCD gets one
contiguous range of block indices of its grid row.  This test compiles the
library's own header for the host and checks, for every G up to 1100 and
every grid row y below 70, that the renumbering is a bijection of [0, G) and
that the blocks of each XCD receive consecutive indices in launch order.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PROGRAM = r'''
#include "device_util.h"
#include <cstdio>
#include <vector>
int main()
{
    long checked = 0;
    for (int G = 1; G <= 1100; ++G)
        for (unsigned y = 0; y < 70; ++y) {
            std::vector<int> seen(G, 0);
            std::vector<std::vector<int>> per(chm::kXcds);
            for (int b = 0; b < G; ++b) {
                const int r = chm::xcd_rank(G, b, y);
                if (r < 0 || r >= G || seen[r]++) {
                    printf("not a bijection: G=%d y=%u b=%d r=%d\n", G, y, b, r);
                    return 1;
                }
                per[(y * (unsigned)G + b) % chm::kXcds].push_back(r);
            }
            for (auto &v : per)
                for (size_t i = 1; i < v.size(); ++i)
                    if (v[i] != v[i - 1] + 1) {
                        printf("not contiguous: G=%d y=%u\n", G, y);
                        return 1;
                    }
            ++checked;
        }
    printf("OK %ld\n", checked);
    return 0;
}
'''


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_xcd_rank_is_a_contiguous_bijection(tmp_path):
    src = tmp_path / "xcd.hip"
    src.write_text(PROGRAM)
    exe = tmp_path / "xcd"
    cmd = ["hipcc", "-O2", "-std=c++17", "--offload-arch=gfx950",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_2204_03575_amd", "csrc"), "-o", str(exe), str(src)]
    subprocess.run(cmd, check=True, capture_output=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout
    assert out.stdout.strip() == "OK 77000"
