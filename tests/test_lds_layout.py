"""The FP32 tracers' LDS layout (csrc/ire_internal.h, lds_layout): every region
starts on a 16-byte boundary, the regions follow each other without overlap
and each is at least as large as what it holds, for odd and even table sizes.
The escaping spectrum and the grouping scratch hold doubles updated by LDS
atomics, which need 8-byte alignment whatever the counts of 4-byte and 1-byte
table entries before them.  Built on the host with g++ (no GPU)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs the host compiler")

HARNESS = r'''
#include <cstdio>
#include "ire_internal.h"
using namespace ire;
int main() {
    int cases = 0;
    for (int n_table : {3, 4, 52, 103, 203, 5393})
    for (int K : {1, 2, 5, 8, 63, 64, 255})
    for (int nt : {2, 3, 101, 511, 512, 513})
    for (int flags = 0; flags < 4; ++flags) {
        const bool sed = flags & 1, rk = flags & 2;
        const LdsLayout L = lds_layout(n_table, K, nt, sed, rk, 1024);
        const size_t off[10] = {L.sh, L.dust, L.cdf, L.G, L.D, L.guide, L.sed, L.rk, L.agg, L.total};
        const size_t need[9] = {(size_t)(n_table + kPadBelow) * sizeof(ShellF), (size_t)K * sizeof(DustF),
                                (size_t)2 * K * 4, (size_t)nt * 4, (size_t)nt * (K | 1) * 4, guide_bytes(nt),
                                sed ? (size_t)4 * K * 8 : 0, rk ? (size_t)(n_table + kPadBelow) * 8 : 0,
                                agg_lds_bytes(1024)};
        for (int j = 0; j < 10; ++j) {
            if (off[j] % 16 != 0) { std::printf("misaligned region %d: K=%d nt=%d\n", j, K, nt); return 1; }
            if (j < 9 && off[j + 1] < off[j] + need[j]) { std::printf("overlap %d\n", j); return 2; }
            if (j < 9 && off[j + 1] >= off[j] + need[j] + 16) { std::printf("gap %d\n", j); return 3; }
        }
        ++cases;
    }
    std::printf("%d\n", cases);
    return 0;
}
'''


def test_lds_regions_aligned_and_disjoint(tmp_path):
    src = tmp_path / "lds.cpp"
    src.write_text(HARNESS)
    exe = tmp_path / "lds"
    subprocess.run(["g++", "-std=c++17", "-O1", "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include", "-I",
                    os.path.join(ROOT, "paper_2408_13807_amd", "csrc"), str(src), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert int(r.stdout.split()[0]) == 6 * 7 * 6 * 4
