"""The four-way table search of the tracers' frequency draws
(csrc/ire_internal.h, count_le4) against a plain linear count, on random
non-decreasing tables of 1 to 300 entries with flat runs and with values
between, below, above and equal to the entries.  Built on the host with g++
(no GPU)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs the host compiler")

HARNESS = r'''
#include <cstdio>
#include <random>
#include <vector>
#include "ire_internal.h"
using namespace ire;
template <typename T> int check(std::mt19937 &rng, long &checks) {
    for (int n = 1; n <= 300; ++n)
        for (int trial = 0; trial < 20; ++trial) {
            std::vector<T> t(n);
            T c = 0;
            for (int i = 0; i < n; ++i) {
                if (rng() % 3) c += (T)(rng() % 1000) / (T)1000;   // a third of the steps flat
                t[i] = c;
            }
            for (int j = 0; j < 3 * n + 8; ++j) {
                T x;
                if (j < n) x = t[j];                                 // on an entry (and its flat run)
                else x = (T)(rng() % 100000) / (T)100000 * (c + 2) - (T)1;
                int ref = 0;
                while (ref < n && t[ref] <= x) ++ref;
                const int got = count_le4(t.data(), n, x);
                if (got != ref) { std::printf("n=%d x=%g ref=%d got=%d\n", n, (double)x, ref, got); return 1; }
                ++checks;
            }
        }
    return 0;
}
int main() {
    std::mt19937 rng(7);
    long checks = 0;
    if (check<float>(rng, checks) || check<double>(rng, checks)) return 1;
    std::printf("%ld\n", checks);
    return 0;
}
'''


def test_count_le4_equals_linear_count(tmp_path):
    src = tmp_path / "cle4.cpp"
    src.write_text(HARNESS)
    exe = tmp_path / "cle4"
    subprocess.run(["g++", "-std=c++17", "-O1", "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include", "-I",
                    os.path.join(ROOT, "paper_2408_13807_amd", "csrc"), str(src), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert int(r.stdout.split()[0]) > 500_000
