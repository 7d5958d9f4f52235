"""The fragment-ordered weight copy that surrogate inference reads
(csrc/sur_internal.h, frag_index): a permutation of each weight block, and
the position of every weight is the one at which a wave's MFMA A fragment
for its output group and k step expects it (lane % 32 the output within the
group of 32, lane / 32 the half of the 16-input step, 8 inputs per lane).
Built on the host with ROCm's clang (no GPU)."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/llvm/bin/clang++"

pytestmark = pytest.mark.skipif(not os.path.exists(CLANG), reason="needs ROCm's host compiler")

HARNESS = r'''
#include <cstdio>
#include <vector>
#include "sur_internal.h"
int main() {
    long checks = 0;
    for (size_t K : {(size_t)sur::kIn, (size_t)sur::kWidth}) {
        std::vector<int> seen(sur::kWidth * K, 0);
        for (size_t o = 0; o < (size_t)sur::kWidth; ++o)
            for (size_t i = 0; i < K; ++i) {
                const size_t f = sur::frag_index(o, i, K);
                if (f >= sur::kWidth * K || seen[f]++) { std::printf("not a permutation at o=%zu i=%zu\n", o, i); return 1; }
                // decode: 512 values per (output group q, k step st), 8 per lane
                const size_t e = f % 8, lane = (f / 8) % 64, st = (f / 512) % (K / 16), q = f / (512 * (K / 16));
                if (32 * q + lane % 32 != o || 16 * st + 8 * (lane / 32) + e != i) {
                    std::printf("o=%zu i=%zu at q=%zu st=%zu lane=%zu e=%zu\n", o, i, q, st, lane, e);
                    return 1;
                }
                ++checks;
            }
    }
    std::printf("%ld\n", checks);
    return 0;
}
'''


def test_frag_index_is_the_mfma_fragment_order(tmp_path):
    src = tmp_path / "frag.cpp"
    src.write_text(HARNESS)
    exe = tmp_path / "frag"
    subprocess.run([CLANG, "-std=c++17", "-O1", "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include", "-I",
                    os.path.join(ROOT, "paper_2408_13807_amd", "csrc"), str(src), "-o", str(exe)], check=True,
                   capture_output=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert int(r.stdout.split()[0]) == 256 * (32 + 256)
