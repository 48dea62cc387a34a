"""The 32-bit entry guard of the step kernels (csrc/index_limits.h), compiled for
the host with g++: a chain set may hold at most INT32_MAX minibatch entries
(two per observation and chain).  The entry points reject larger sets with
SPIDER_E_UNSUPPORTED before any device work."""
import os
import subprocess
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2508_12117_amd", "csrc")

PROGRAM = r"""
#include <cstdio>
#include "index_limits.h"
int main() {
  using spider::entries_fit;
  const long long cases[][2] = {
    {1, 1}, {1, 1073741823}, {1, 1073741824}, {8, 134217727}, {8, 134217728},
    {68, 15790320}, {68, 15790321}, {0, 5}, {5, 0}, {-1, 5}, {3, -7},
    {1, 4611686018427387904LL}};
  for (auto& c : cases) std::printf("%lld %lld %d\n", c[0], c[1], (int)entries_fit(c[0], c[1]));
  return 0;
}
"""


def test_entries_fit_boundaries():
    with tempfile.TemporaryDirectory() as d:
        src, exe = os.path.join(d, "t.cpp"), os.path.join(d, "t")
        with open(src, "w") as f:
            f.write(PROGRAM)
        subprocess.run(["g++", "-std=c++17", "-I", CSRC, src, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    got = {(int(a), int(b)): int(v) for a, b, v in (l.split() for l in out.splitlines())}
    for (C, n), v in got.items():
        want = int(C >= 1 and n >= 1 and 2 * C * n <= 2**31 - 1)
        assert v == want, (C, n, v)
